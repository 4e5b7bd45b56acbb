// Batched vector kernels for the Krylov (FGMRES) solve with the MGCNN network as a fixed
// right preconditioner (Sec. 2.2: the linear network serves as the preconditioner of a
// Krylov method).  Every kernel handles a batch of independent problems [B][n][n]; problems
// whose flag in `active` is zero are skipped.
#include "mgcnn_device.h"
#include "mgcnn_internal.h"
#include "mgcnn_krylov.h"

namespace mg {

// y = A x (divergence form, harmonic faces, upwind convection), f64 arithmetic, f32 in/out.
__global__ __launch_bounds__(256) void apply_A_kernel(const float* __restrict__ a,
                                                      const float* __restrict__ bvec,
                                                      const float* __restrict__ x,
                                                      float* __restrict__ y, int n, int tiles_x,
                                                      int tiles_per_prob, const int* __restrict__ active) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int j = (tile % tiles_x) * 64 + (threadIdx.x & 63);
  const int i = (tile / tiles_x) * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const size_t base = (size_t)b * n * n;
  const float* A = a + base;
  const float* X = x + base;
  const int ij = i * n + j;
  auto H = [](double p, double q) { return 2.0 * p * q / (p + q); };
  const double ac = A[ij];
  const double aE = (j + 1 < n) ? H(ac, A[ij + 1]) : ac;
  const double aW = (j > 0) ? H(ac, A[ij - 1]) : ac;
  const double aN = (i + 1 < n) ? H(ac, A[ij + n]) : ac;
  const double aS = (i > 0) ? H(ac, A[ij - n]) : ac;
  const double xc = X[ij];
  const double xE = (j + 1 < n) ? (double)X[ij + 1] : 0.0;
  const double xW = (j > 0) ? (double)X[ij - 1] : 0.0;
  const double xN = (i + 1 < n) ? (double)X[ij + n] : 0.0;
  const double xS = (i > 0) ? (double)X[ij - n] : 0.0;
  const double ih = (double)(n + 1), ih2 = ih * ih;
  const double bx = bvec[2 * b], by = bvec[2 * b + 1];
  const double bxp = bx > 0 ? bx : 0, bxm = bx < 0 ? bx : 0;
  const double byp = by > 0 ? by : 0, bym = by < 0 ? by : 0;
  const double v = ((aE + aW + aN + aS) * xc - aE * xE - aW * xW - aN * xN - aS * xS) * ih2 +
                   (bxp * (xc - xW) + bxm * (xE - xc) + byp * (xc - xS) + bym * (xN - xc)) * ih;
  y[base + ij] = (float)v;
}

void launch_apply_A(const float* a, const float* b, const float* x, float* y, int n, int B,
                    const int* active, hipStream_t st) {
  const int tx = (n + 63) / 64, ty = (n + 3) / 4;
  hipLaunchKernelGGL(apply_A_kernel, dim3(tx * ty * B), dim3(256), 0, st, a, b, x, y, n, tx, tx * ty,
                     active);
}

// partial[b][blk][i] = sum over the block's elements of w[b][k] * V_i[b][k], i < cnt.
// Each block covers KR_CHUNK consecutive elements of one problem.
constexpr int KR_CHUNK = 8192;
constexpr int KR_MAXV = 64;

int krylov_blocks(int n) { return (int)(((size_t)n * n + KR_CHUNK - 1) / KR_CHUNK); }

__global__ __launch_bounds__(256) void dots_kernel(const float* __restrict__ w,
                                                   const float* __restrict__ V, size_t vstride,
                                                   int cnt, size_t nn, int blocks,
                                                   double* __restrict__ partial,
                                                   const int* __restrict__ active) {
  const int b = blockIdx.x / blocks, blk = blockIdx.x % blocks;
  if (active != nullptr && active[b] == 0) return;
  const size_t k0 = (size_t)blk * KR_CHUNK;
  const size_t k1 = (k0 + KR_CHUNK < nn) ? k0 + KR_CHUNK : nn;
  const float* W = w + (size_t)b * nn;
  for (int i = 0; i < cnt; ++i) {
    const float* Vi = V + (size_t)i * vstride + (size_t)b * nn;
    double s = 0.0;
    for (size_t k = k0 + threadIdx.x; k < k1; k += 256) s += (double)W[k] * (double)Vi[k];
    s = block_sum_256(s);
    if (threadIdx.x == 0) partial[((size_t)b * blocks + blk) * KR_MAXV + i] = s;
  }
}

__global__ void dots_reduce_kernel(const double* __restrict__ partial, int blocks, int cnt, int B,
                                   double* __restrict__ out, const int* __restrict__ active) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= B * cnt) return;
  const int b = id / cnt, i = id % cnt;
  if (active != nullptr && active[b] == 0) { out[b * KR_MAXV + i] = 0.0; return; }
  double s = 0.0;
  for (int k = 0; k < blocks; ++k) s += partial[((size_t)b * blocks + k) * KR_MAXV + i];
  out[b * KR_MAXV + i] = s;
}

void launch_dots(const float* w, const float* V, size_t vstride, int cnt, int n, int B,
                 double* partial, double* out, const int* active, hipStream_t st) {
  const size_t nn = (size_t)n * n;
  const int blocks = krylov_blocks(n);
  hipLaunchKernelGGL(dots_kernel, dim3(blocks * B), dim3(256), 0, st, w, V, vstride, cnt, nn, blocks,
                     partial, active);
  hipLaunchKernelGGL(dots_reduce_kernel, dim3((B * cnt + 255) / 256), dim3(256), 0, st, partial,
                     blocks, cnt, B, out, active);
}

// w[b] -= sum_{i<cnt} h[b][i] V_i[b]
__global__ void orth_update_kernel(float* __restrict__ w, const float* __restrict__ V,
                                   size_t vstride, int cnt, size_t nn, int B,
                                   const double* __restrict__ h, const int* __restrict__ active) {
  const size_t total = nn * (size_t)B;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(k / nn);
    if (active != nullptr && active[b] == 0) continue;
    double acc = w[k];
    for (int i = 0; i < cnt; ++i) acc -= h[b * KR_MAXV + i] * (double)V[(size_t)i * vstride + k];
    w[k] = (float)acc;
  }
}

void launch_orth_update(float* w, const float* V, size_t vstride, int cnt, int n, int B,
                        const double* h, const int* active, hipStream_t st) {
  const size_t total = (size_t)n * n * B;
  size_t blocks = (total + 255) / 256;
  if (blocks > 131072) blocks = 131072;
  hipLaunchKernelGGL(orth_update_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, V, vstride, cnt,
                     (size_t)n * n, B, h, active);
}

// x[b] *= s[b]
__global__ void scale_kernel(float* __restrict__ x, size_t nn, int B, const double* __restrict__ s,
                             const int* __restrict__ active) {
  const size_t total = nn * (size_t)B;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(k / nn);
    if (active != nullptr && active[b] == 0) continue;
    x[k] = (float)((double)x[k] * s[b]);
  }
}

void launch_scale(float* x, int n, int B, const double* s, const int* active, hipStream_t st) {
  const size_t total = (size_t)n * n * B;
  size_t blocks = (total + 255) / 256;
  if (blocks > 131072) blocks = 131072;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, (size_t)n * n, B, s,
                     active);
}

// u[b] += sum_{j<cnt} y[b][j] Z_j[b]
template <typename UT>
__global__ void combine_kernel(UT* __restrict__ u, const float* __restrict__ Z, size_t zstride,
                               int cnt, size_t nn, int B, const double* __restrict__ y,
                               const int* __restrict__ active) {
  const size_t total = nn * (size_t)B;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(k / nn);
    if (active != nullptr && active[b] == 0) continue;
    double acc = 0.0;
    for (int j = 0; j < cnt; ++j) acc += y[b * KR_MAXV + j] * (double)Z[(size_t)j * zstride + k];
    u[k] = (UT)((double)u[k] + acc);
  }
}

void launch_combine(void* u, bool u_f64, const float* Z, size_t zstride, int cnt, int n, int B,
                    const double* y, const int* active, hipStream_t st) {
  const size_t total = (size_t)n * n * B;
  size_t blocks = (total + 255) / 256;
  if (blocks > 131072) blocks = 131072;
  if (u_f64)
    hipLaunchKernelGGL(combine_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, (double*)u, Z,
                       zstride, cnt, (size_t)n * n, B, y, active);
  else
    hipLaunchKernelGGL(combine_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (float*)u, Z,
                       zstride, cnt, (size_t)n * n, B, y, active);
}

}  // namespace mg
