// Internal declarations of the batched Krylov (FGMRES) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace mg {

constexpr int KRYLOV_MAX_BASIS = 64;   // maximum restart length + 1
constexpr int KRYLOV_LD = 72;          // per-problem stride of the scalar arrays (basis + norm + pad)
constexpr int KRYLOV_MAX_DEFLATE = 32; // deflation vectors kept across a restart

// Arnoldi vectors are [B][krylov_vpad(n)] float32, zero padded; Gram-Schmidt passes run over
// krylov_blocks(n) groups of elements per problem.
size_t krylov_vpad(int n);
int krylov_blocks(int n);

// y = A x ([B][n][n] in, per-problem stride ystride out), f64 stencil arithmetic
void launch_apply_A(const float* a, const float* b, const float* x, float* y, size_t ystride, int n,
                    int B, const int* active, int form, hipStream_t st);
// r = f - A u (u f32 or f64, [B][n][n]); r with per-problem stride rstride
void launch_krylov_residual(const float* a, const float* b, const float* f, const void* u, bool u_f64,
                            float* r, size_t rstride, int n, int B, const int* active, int form,
                            hipStream_t st);
// One Gram-Schmidt pass over w and V_0..V_{cnt-1} (V_i at V + i * vstride), results in
// out[b * KRYLOV_LD + slot]:
//   mode 0: out[i] = <V_i, w> (i < cnt), out[cnt] = <w, w>
//   mode 1: w -= sum_i h_i V_i, then out[i] = <V_i, w>
//   mode 2: w -= sum_i h_i V_i, then out[0] = <w, w>
// partial: B * KRYLOV_LD * krylov_blocks(n) doubles.  Returns -1 if cnt is out of range.
int launch_gs_pass(int mode, float* w, const float* V, size_t vstride, int cnt, int n, int B,
                   const double* h, double* partial, double* out, const int* active, hipStream_t st);
// rt = (v - A x) / D: v a basis vector (stride krylov_vpad(n)), x and rt [B][n][n]
void launch_inner_residual(const float* a, const float* b, const float* v, const float* x, float* rt, int n,
                           int B, const int* active, int form, hipStream_t st);
// v *= s[b * KRYLOV_LD] in place (stride krylov_vpad(n)) and rt = v / D ([B][n][n])
void launch_normalize_diag(const float* a, const float* b, float* v, float* rt, const double* s, int n,
                           int B, const int* active, int form, hipStream_t st);
// In place X_i,b = sum_{j < count_b} X_j,b C_b[j][i] for i < k (X_j at X + j * stride, problem b
// at b * plen); C_b at C + b * cstride, row-major with row length k, count_b = C_b[cstride - 1];
// count_b <= cnt.  Only the listed problems.
void launch_basis_combine(float* X, size_t stride, size_t plen, int cnt, int k, const double* C,
                          size_t cstride, int B, const int* active, hipStream_t st);
// u_b += sum_{j<cnt} y[b * KRYLOV_LD + j] Z_j,b  (Z_j at Z + j * zstride, [B][n][n])
void launch_combine(void* u, bool u_f64, const float* Z, size_t zstride, int cnt, int n, int B,
                    const double* y, const int* active, hipStream_t st);

}  // namespace mg
