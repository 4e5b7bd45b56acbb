// Internal declarations of the batched Krylov (FGMRES) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace mg {

constexpr int KRYLOV_MAX_BASIS = 64;   // maximum restart length + 1

int krylov_blocks(int n);
void launch_apply_A(const float* a, const float* b, const float* x, float* y, int n, int B,
                    const int* active, hipStream_t st);
// out[b * 64 + i] = <w_b, V_i,b> for i < cnt (V_i at V + i * vstride); partial: B * blocks * 64
void launch_dots(const float* w, const float* V, size_t vstride, int cnt, int n, int B,
                 double* partial, double* out, const int* active, hipStream_t st);
void launch_orth_update(float* w, const float* V, size_t vstride, int cnt, int n, int B,
                        const double* h, const int* active, hipStream_t st);
void launch_scale(float* x, int n, int B, const double* s, const int* active, hipStream_t st);
void launch_combine(void* u, bool u_f64, const float* Z, size_t zstride, int cnt, int n, int B,
                    const double* y, const int* active, hipStream_t st);

}  // namespace mg
