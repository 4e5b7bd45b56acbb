// Batched vector kernels of preconditioned conjugate gradients (the short-recurrence Krylov
// method for a symmetric operator with a symmetric preconditioner: the V-cycle, or the
// symmetric variant of the network, Sec. 3.3, as preconditioner of a Krylov method, Sec. 2.2).
//
// Every vector is [B][n][n] float32 (u float32 or float64) and every kernel covers the problems
// of a compact list: blockIdx.y indexes the list, blockIdx.x a chunk of PCG_CHUNK nodes of that
// problem.  Inner products are accumulated in f64: per thread, then across the wavefront by
// shuffles and across the workgroup in LDS, one partial per workgroup, stored by problem (so that
// groups of problems launched from different lists share one buffer); pcg_reduce_kernel sums the
// partials of a problem in a fixed order, so results do not depend on timing.
#include "mgcnn_device.h"
#include "mgcnn_internal.h"
#include "mgcnn_pcg.h"

namespace mg {

constexpr int PCG_THREADS = 256;
constexpr int PCG_PER_THREAD = 4;
constexpr int PCG_CHUNK = PCG_THREADS * PCG_PER_THREAD;

int pcg_blocks(int n) { return (int)(((size_t)n * n + PCG_CHUNK - 1) / PCG_CHUNK); }

__device__ __forceinline__ double pcg_block_sum(double v) {
  __shared__ double sh[PCG_THREADS / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < PCG_THREADS / 64; ++w) s += sh[w];
  return s;
}

// MODE PCG_UPDATE: u += alpha p, r -= alpha q, then rt = r * dsc and partial |r|^2
// MODE PCG_PREP:   rt = r * dsc and partial |r|^2
template <typename UT, int MODE>
__global__ __launch_bounds__(PCG_THREADS) void pcg_step_kernel(UT* __restrict__ u, const float* __restrict__ p,
                                                               float* __restrict__ r, const float* __restrict__ q,
                                                               const float* __restrict__ dsc, float* __restrict__ rt,
                                                               const double* __restrict__ coef,
                                                               double* __restrict__ partial, int nn, int nblk,
                                                               const int* __restrict__ list) {
  const int b = list[blockIdx.y];
  const size_t base = (size_t)b * nn;
  const double al = MODE != PCG_PREP ? coef[2 * b] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < PCG_PER_THREAD; ++k) {
    const int i = blockIdx.x * PCG_CHUNK + k * PCG_THREADS + threadIdx.x;
    if (i >= nn) break;
    const size_t g = base + i;
    float ri = r[g];
    if constexpr (MODE == PCG_UPDATE) {
      u[g] = (UT)((double)u[g] + al * (double)p[g]);
      ri = (float)((double)ri - al * (double)q[g]);
      r[g] = ri;
    }
    rt[g] = ri * dsc[g];
    acc += (double)ri * (double)ri;
  }
  const double s = pcg_block_sum(acc);
  if (threadIdx.x == 0) partial[((size_t)b * nblk + blockIdx.x) * 2 + 0] = s;
}

// SCALE: z *= dsc in place (the output half of D^-1/2 B(D^-1/2 r)); partial slot 1 = (r, z)
template <bool SCALE>
__global__ __launch_bounds__(PCG_THREADS) void pcg_rz_kernel(float* __restrict__ z, const float* __restrict__ r,
                                                             const float* __restrict__ dsc,
                                                             double* __restrict__ partial, int nn, int nblk,
                                                             const int* __restrict__ list) {
  const int b = list[blockIdx.y];
  const size_t base = (size_t)b * nn;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < PCG_PER_THREAD; ++k) {
    const int i = blockIdx.x * PCG_CHUNK + k * PCG_THREADS + threadIdx.x;
    if (i >= nn) break;
    const size_t g = base + i;
    float zi = z[g];
    if constexpr (SCALE) {
      zi *= dsc[g];
      z[g] = zi;
    }
    acc += (double)r[g] * (double)zi;
  }
  const double s = pcg_block_sum(acc);
  if (threadIdx.x == 0) partial[((size_t)b * nblk + blockIdx.x) * 2 + 1] = s;
}

// p = z + beta p (beta = coef[2b + 1]; p = z when beta is 0, whatever p held)
__global__ __launch_bounds__(PCG_THREADS) void pcg_dir_kernel(float* __restrict__ p, const float* __restrict__ z,
                                                              const double* __restrict__ coef, int nn,
                                                              const int* __restrict__ list) {
  const int b = list[blockIdx.y];
  const size_t base = (size_t)b * nn;
  const double be = coef[2 * b + 1];
#pragma unroll
  for (int k = 0; k < PCG_PER_THREAD; ++k) {
    const int i = blockIdx.x * PCG_CHUNK + k * PCG_THREADS + threadIdx.x;
    if (i >= nn) break;
    const size_t g = base + i;
    p[g] = be == 0.0 ? z[g] : (float)((double)z[g] + be * (double)p[g]);
  }
}

// partial slot 0 = (x, y)
__global__ __launch_bounds__(PCG_THREADS) void pcg_dot_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                              double* __restrict__ partial, int nn, int nblk,
                                                              const int* __restrict__ list) {
  const int b = list[blockIdx.y];
  const size_t base = (size_t)b * nn;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < PCG_PER_THREAD; ++k) {
    const int i = blockIdx.x * PCG_CHUNK + k * PCG_THREADS + threadIdx.x;
    if (i >= nn) break;
    acc += (double)x[base + i] * (double)y[base + i];
  }
  const double s = pcg_block_sum(acc);
  if (threadIdx.x == 0) partial[((size_t)b * nblk + blockIdx.x) * 2 + 0] = s;
}

// out[2 b + s] = sum of the problem's partials in slot s (s < nslot), one workgroup per problem
__global__ __launch_bounds__(PCG_THREADS) void pcg_reduce_kernel(const double* __restrict__ partial, int nblk,
                                                                 int nslot, double* __restrict__ out,
                                                                 const int* __restrict__ list) {
  const int b = list[blockIdx.x];
  for (int s = 0; s < nslot; ++s) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < nblk; k += PCG_THREADS)
      acc += partial[((size_t)b * nblk + k) * 2 + s];
    const double t = pcg_block_sum(acc);
    if (threadIdx.x == 0) out[2 * b + s] = t;
    __syncthreads();   // the LDS of pcg_block_sum is reused by the next slot
  }
}

__global__ __launch_bounds__(PCG_THREADS) void pcg_fill_kernel(float* __restrict__ x, float v, size_t len) {
  const size_t i = (size_t)blockIdx.x * PCG_THREADS + threadIdx.x;
  if (i < len) x[i] = v;
}

__global__ __launch_bounds__(PCG_THREADS) void pcg_sqrt_kernel(float* __restrict__ x, size_t len) {
  const size_t i = (size_t)blockIdx.x * PCG_THREADS + threadIdx.x;
  if (i < len) x[i] = sqrtf(x[i]);
}

static dim3 pcg_grid(int n, int count) { return dim3(pcg_blocks(n), count); }

void launch_pcg_step(int mode, void* u, bool u_f64, const float* p, float* r, const float* q, const float* dsc,
                     float* rt, const double* coef, double* partial, int n, int count, const int* list,
                     hipStream_t st) {
  const int nn = n * n, nblk = pcg_blocks(n);
  const dim3 g = pcg_grid(n, count), blk(PCG_THREADS);
#define PCG_STEP(UT, M)                                                                             \
  hipLaunchKernelGGL((pcg_step_kernel<UT, M>), g, blk, 0, st, (UT*)u, p, r, q, dsc, rt, coef, partial, nn, \
                     nblk, list)
  if (u_f64) {
    if (mode == PCG_UPDATE) PCG_STEP(double, PCG_UPDATE);
    else PCG_STEP(double, PCG_PREP);
  } else {
    if (mode == PCG_UPDATE) PCG_STEP(float, PCG_UPDATE);
    else PCG_STEP(float, PCG_PREP);
  }
#undef PCG_STEP
}

void launch_pcg_rz(bool scale, float* z, const float* r, const float* dsc, double* partial, int n, int count,
                   const int* list, hipStream_t st) {
  const int nn = n * n, nblk = pcg_blocks(n);
  if (scale)
    hipLaunchKernelGGL((pcg_rz_kernel<true>), pcg_grid(n, count), dim3(PCG_THREADS), 0, st, z, r, dsc, partial,
                       nn, nblk, list);
  else
    hipLaunchKernelGGL((pcg_rz_kernel<false>), pcg_grid(n, count), dim3(PCG_THREADS), 0, st, z, r, dsc, partial,
                       nn, nblk, list);
}

void launch_pcg_dir(float* p, const float* z, const double* coef, int n, int count, const int* list,
                    hipStream_t st) {
  hipLaunchKernelGGL(pcg_dir_kernel, pcg_grid(n, count), dim3(PCG_THREADS), 0, st, p, z, coef, n * n, list);
}

void launch_pcg_dot(const float* x, const float* y, double* partial, int n, int count, const int* list,
                    hipStream_t st) {
  hipLaunchKernelGGL(pcg_dot_kernel, pcg_grid(n, count), dim3(PCG_THREADS), 0, st, x, y, partial, n * n,
                     pcg_blocks(n), list);
}

void launch_pcg_reduce(const double* partial, int nslot, double* out, int n, int count, const int* list,
                       hipStream_t st) {
  hipLaunchKernelGGL(pcg_reduce_kernel, dim3(count), dim3(PCG_THREADS), 0, st, partial, pcg_blocks(n), nslot,
                     out, list);
}

void launch_pcg_fill(float* x, float v, size_t len, hipStream_t st) {
  if (len == 0) return;
  hipLaunchKernelGGL(pcg_fill_kernel, dim3((unsigned)((len + PCG_THREADS - 1) / PCG_THREADS)),
                     dim3(PCG_THREADS), 0, st, x, v, len);
}

void launch_pcg_sqrt(float* x, size_t len, hipStream_t st) {
  if (len == 0) return;
  hipLaunchKernelGGL(pcg_sqrt_kernel, dim3((unsigned)((len + PCG_THREADS - 1) / PCG_THREADS)),
                     dim3(PCG_THREADS), 0, st, x, len);
}

}  // namespace mg
