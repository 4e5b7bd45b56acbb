// Internal declarations of the batched preconditioned-conjugate-gradient kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace mg {

enum PcgStepMode : int { PCG_UPDATE = 0, PCG_PREP = 1 };

// workgroups per problem of every PCG vector kernel; partial buffers hold
// B * pcg_blocks(n) * 2 doubles (two slots per workgroup, indexed by problem)
int pcg_blocks(int n);

// All vectors [B][n][n]; problem list[y] for y < count; per-problem scalars in coef[2b]
// (alpha) and coef[2b + 1] (beta).
//   PCG_UPDATE: u += alpha p; r -= alpha q; rt = r * dsc; partial slot 0 = |r|^2
//   PCG_PREP:   rt = r * dsc; partial slot 0 = |r|^2
void launch_pcg_step(int mode, void* u, bool u_f64, const float* p, float* r, const float* q, const float* dsc,
                     float* rt, const double* coef, double* partial, int n, int count, const int* list,
                     hipStream_t st);
// scale: z *= dsc in place; then partial slot 1 = (r, z)
void launch_pcg_rz(bool scale, float* z, const float* r, const float* dsc, double* partial, int n, int count,
                   const int* list, hipStream_t st);
// p = z + beta p (p = z where beta = 0)
void launch_pcg_dir(float* p, const float* z, const double* coef, int n, int count, const int* list,
                    hipStream_t st);
// partial slot 0 = (x, y)
void launch_pcg_dot(const float* x, const float* y, double* partial, int n, int count, const int* list,
                    hipStream_t st);
// out[2b + s] = sum over the problem's partials of slot s, s < nslot
void launch_pcg_reduce(const double* partial, int nslot, double* out, int n, int count, const int* list,
                       hipStream_t st);
void launch_pcg_fill(float* x, float v, size_t len, hipStream_t st);
void launch_pcg_sqrt(float* x, size_t len, hipStream_t st);

}  // namespace mg
