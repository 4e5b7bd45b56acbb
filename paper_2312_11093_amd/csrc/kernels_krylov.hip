// Batched vector kernels for the Krylov (FGMRES) solve with the MGCNN network as a fixed
// right preconditioner (Sec. 2.2: the network is linear in its input, so it can precondition
// a Krylov method).  Every kernel handles a batch of independent problems; problems whose flag
// not in the `active` list are left out of the grid.
//
// Layout: Arnoldi vectors are [B][vpad] float32 with vpad = n*n rounded up to 512; the
// padding is zero from allocation on and no kernel writes it with anything but zero, so the
// Gram-Schmidt kernels run without bounds checks.  Preconditioned vectors Z and the rhs / u
// keep the [B][n][n] layout of the rest of the library.
#include "mgcnn_device.h"
#include "mgcnn_internal.h"
#include "mgcnn_krylov.h"

namespace mg {

constexpr int KR_LD = KRYLOV_LD;
constexpr int KG_THREADS = 256;
constexpr int KG_ELEMS = 2 * KG_THREADS;    // elements per group (two per thread)
constexpr int KG_ITERS = 1;                 // groups per workgroup (more adds register pressure)

size_t krylov_vpad(int n) {
  const size_t nn = (size_t)n * n, q = (size_t)KG_ELEMS * KG_ITERS;
  return (nn + q - 1) / q * q;
}
int krylov_blocks(int n) { return (int)(krylov_vpad(n) / ((size_t)KG_ELEMS * KG_ITERS)); }

// ---- stencil passes ----------------------------------------------------------------------------
// Divergence-form 5-point diffusion with harmonic face means plus first-order upwind convection,
// f64 arithmetic.  Tiles of 256 columns x KW_ROWS rows; each thread walks one column, keeping the
// rows above, at and below in registers, so every vertical face coefficient is formed once and
// every value comes from HBM once.  In full tiles all loads of the walk are issued before the
// arithmetic (a loop with an exit test per row keeps only one row in flight per thread).
// Reciprocals: hardware estimate refined by two Newton steps.
//   KW_APPLY:     y[b][ystride] = A x                      (x f32 [B][n][n])
//   KW_RESIDUAL:  y[b][ystride] = f - A u                  (u f32 or f64 [B][n][n])
//   KW_NORMALIZE: v[b][ystride] *= s[b];  rt = v / D       (rt [B][n][n])
//   KW_INNER:     rt = (v[b][ystride] - A x) / D           (x f32, rt [B][n][n])
constexpr int KW_ROWS = 8;
enum KwMode : int { KW_APPLY = 0, KW_RESIDUAL = 1, KW_NORMALIZE = 2, KW_INNER = 3 };

__device__ __forceinline__ double krcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double kharm(double p, double q) { return (2.0 * p * q) * krcp(p + q); }

template <typename XT, int MODE>
__global__ __launch_bounds__(256) void kwalk_kernel(const float* __restrict__ a,
                                                    const float* __restrict__ bvec,
                                                    const float* __restrict__ f,
                                                    const XT* __restrict__ x,
                                                    float* __restrict__ y, size_t ystride,
                                                    float* __restrict__ rt,
                                                    const double* __restrict__ sc, int n,
                                                    int tiles_x, int tiles_per_prob,
                                                    const int* __restrict__ active, int form) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  const int j = (tile % tiles_x) * 256 + threadIdx.x;
  const int i0 = (tile / tiles_x) * KW_ROWS;
  if (j >= n) return;
  const size_t base = (size_t)b * n * n;
  const float* A = a + base;
  const double ih = (double)(n + 1), ih2 = ih * ih;
  const double bx = bvec[2 * b], by = bvec[2 * b + 1];
  const double bxp = bx > 0 ? bx : 0, bxm = bx < 0 ? bx : 0;
  const double byp = by > 0 ? by : 0, bym = by < 0 ? by : 0;
  const double conv_diag = (bxp - bxm + byp - bym) * ih;
  const bool hasE = j + 1 < n, hasW = j > 0;
  const int dE = hasE ? 1 : 0, dW = hasW ? 1 : 0;          // clamped offsets: branch-free loads
  const XT* X = (MODE == KW_NORMALIZE) ? nullptr : x + base;
  double ac = A[i0 * n + j];
  double aS = (i0 > 0 && !form) ? kharm(ac, (double)A[(i0 - 1) * n + j]) : ac;
  double xc = 0.0, xs = 0.0;
  if constexpr (MODE != KW_NORMALIZE) {
    xc = X[i0 * n + j];
    xs = (i0 > 0) ? (double)X[(i0 - 1) * n + j] : 0.0;
  }
  const double sb = (MODE == KW_NORMALIZE) ? sc[(size_t)b * KR_LD] : 0.0;
  if (i0 + KW_ROWS < n) {
    // full tile, every row has a north neighbour: issue all loads of the walk first, so that
    // the rows' loads are in flight together, then run the recurrence over the registers
    float an_[KW_ROWS], ae_[KW_ROWS], aw_[KW_ROWS], v_[KW_ROWS];
    XT xn_[KW_ROWS], xe_[KW_ROWS], xw_[KW_ROWS];
#pragma unroll
    for (int r = 0; r < KW_ROWS; ++r) {
      const int ij = (i0 + r) * n + j;
      an_[r] = A[ij + n];
      ae_[r] = A[ij + dE];
      aw_[r] = A[ij - dW];
      if constexpr (MODE != KW_NORMALIZE) {
        xn_[r] = X[ij + n];
        xe_[r] = X[ij + dE];
        xw_[r] = X[ij - dW];
      }
      if constexpr (MODE == KW_NORMALIZE || MODE == KW_INNER) v_[r] = y[(size_t)b * ystride + ij];
      if constexpr (MODE == KW_RESIDUAL) v_[r] = f[base + ij];
    }
#pragma unroll
    for (int r = 0; r < KW_ROWS; ++r) {
      const int ij = (i0 + r) * n + j;
      const double an = an_[r];
      const double aN = !form ? kharm(ac, an) : ac;
      const double aE = (hasE && !form) ? kharm(ac, (double)ae_[r]) : ac;
      const double aW = (hasW && !form) ? kharm(ac, (double)aw_[r]) : ac;
      const double sa = aE + aW + aN + aS;
      if constexpr (MODE == KW_NORMALIZE) {
        const double v = (double)v_[r] * sb;
        y[(size_t)b * ystride + ij] = (float)v;
        rt[base + ij] = (float)(v * krcp(sa * ih2 + conv_diag));
      } else {
        const double xn = (double)xn_[r];
        const double xE = hasE ? (double)xe_[r] : 0.0;
        const double xW = hasW ? (double)xw_[r] : 0.0;
        const double Ax = (sa * xc - aE * xE - aW * xW - aN * xn - aS * xs) * ih2 +
                          (bxp * (xc - xW) + bxm * (xE - xc) + byp * (xc - xs) + bym * (xn - xc)) * ih;
        if constexpr (MODE == KW_INNER)
          rt[base + ij] = (float)(((double)v_[r] - Ax) * krcp(sa * ih2 + conv_diag));
        else
          y[(size_t)b * ystride + ij] = (MODE == KW_RESIDUAL) ? (float)((double)v_[r] - Ax) : (float)Ax;
        xs = xc; xc = xn;
      }
      ac = an; aS = form ? an : aN;
    }
    return;
  }
#pragma unroll 2
  for (int r = 0; r < KW_ROWS; ++r) {
    const int i = i0 + r;
    if (i >= n) break;
    const int ij = i * n + j;
    const bool hasN = i + 1 < n;
    const int dN = hasN ? n : 0;
    const double an = A[ij + dN];
    const double aN = (hasN && !form) ? kharm(ac, an) : ac;
    const double aE = (hasE && !form) ? kharm(ac, (double)A[ij + dE]) : ac;
    const double aW = (hasW && !form) ? kharm(ac, (double)A[ij - dW]) : ac;
    const double sa = aE + aW + aN + aS;
    if constexpr (MODE == KW_NORMALIZE) {
      float* vp = y + (size_t)b * ystride + ij;
      const double v = (double)*vp * sb;
      *vp = (float)v;
      rt[base + ij] = (float)(v * krcp(sa * ih2 + conv_diag));
    } else {
      const double xn = hasN ? (double)X[ij + dN] : 0.0;
      const double xE = hasE ? (double)X[ij + dE] : 0.0;
      const double xW = hasW ? (double)X[ij - dW] : 0.0;
      const double Ax = (sa * xc - aE * xE - aW * xW - aN * xn - aS * xs) * ih2 +
                        (bxp * (xc - xW) + bxm * (xE - xc) + byp * (xc - xs) + bym * (xn - xc)) * ih;
      if constexpr (MODE == KW_INNER)
        rt[base + ij] = (float)(((double)y[(size_t)b * ystride + ij] - Ax) * krcp(sa * ih2 + conv_diag));
      else
        y[(size_t)b * ystride + ij] = (MODE == KW_RESIDUAL) ? (float)((double)f[base + ij] - Ax) : (float)Ax;
      xs = xc; xc = xn;
    }
    ac = an; aS = form ? an : aN;   // next row's south face (own node value when form = 1)
  }
}

static void kwalk_grid(int n, int B, dim3& grid, int& tx, int& tpp) {
  tx = (n + 255) / 256;
  tpp = tx * ((n + KW_ROWS - 1) / KW_ROWS);
  grid = dim3(tpp * B);
}

void launch_apply_A(const float* a, const float* b, const float* x, float* y, size_t ystride, int n,
                    int B, const int* active, int form, hipStream_t st) {
  dim3 grid; int tx, tpp;
  kwalk_grid(n, B, grid, tx, tpp);
  hipLaunchKernelGGL((kwalk_kernel<float, KW_APPLY>), grid, dim3(256), 0, st, a, b, (const float*)nullptr,
                     x, y, ystride, (float*)nullptr, (const double*)nullptr, n, tx, tpp, active, form);
}

void launch_krylov_residual(const float* a, const float* b, const float* f, const void* u, bool u_f64,
                            float* r, size_t rstride, int n, int B, const int* active, int form,
                            hipStream_t st) {
  dim3 grid; int tx, tpp;
  kwalk_grid(n, B, grid, tx, tpp);
  if (u_f64)
    hipLaunchKernelGGL((kwalk_kernel<double, KW_RESIDUAL>), grid, dim3(256), 0, st, a, b, f,
                       (const double*)u, r, rstride, (float*)nullptr, (const double*)nullptr, n, tx, tpp,
                       active, form);
  else
    hipLaunchKernelGGL((kwalk_kernel<float, KW_RESIDUAL>), grid, dim3(256), 0, st, a, b, f,
                       (const float*)u, r, rstride, (float*)nullptr, (const double*)nullptr, n, tx, tpp,
                       active, form);
}

void launch_inner_residual(const float* a, const float* b, const float* v, const float* x, float* rt, int n,
                           int B, const int* active, int form, hipStream_t st) {
  dim3 grid; int tx, tpp;
  kwalk_grid(n, B, grid, tx, tpp);
  hipLaunchKernelGGL((kwalk_kernel<float, KW_INNER>), grid, dim3(256), 0, st, a, b, (const float*)nullptr,
                     x, (float*)v, krylov_vpad(n), rt, (const double*)nullptr, n, tx, tpp, active, form);
}

void launch_normalize_diag(const float* a, const float* b, float* v, float* rt, const double* s, int n,
                           int B, const int* active, int form, hipStream_t st) {
  dim3 grid; int tx, tpp;
  kwalk_grid(n, B, grid, tx, tpp);
  hipLaunchKernelGGL((kwalk_kernel<float, KW_NORMALIZE>), grid, dim3(256), 0, st, a, b,
                     (const float*)nullptr, (const float*)nullptr, v, krylov_vpad(n), rt, s, n, tx, tpp,
                     active, form);
}

// ---- Gram-Schmidt passes -----------------------------------------------------------------------
// c ? y : x on values, written as a bit blend so that the compiler cannot turn it into a
// select of addresses (which would keep register arrays out of registers).
__device__ __forceinline__ float blend(bool c, float x, float y) {
  const unsigned m = 0u - (unsigned)c;
  return __uint_as_float((__float_as_uint(x) & ~m) | (__float_as_uint(y) & m));
}

// Reduce-scatter over the 64 lanes of a wave: on entry every lane holds S partial values (S a
// power of two <= 64); on exit the lanes whose low 6 - log2(S) bits are clear hold in a[0] the
// wave total of slot (lane >> (6 - log2(S))).  S - 1 + 6 - log2(S) shuffles instead of 6 S.
template <int S>
__device__ __forceinline__ void wave_reduce_scatter(float (&a)[S]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int step = S / 2, bit = 32; step >= 1; step >>= 1, bit >>= 1) {
    const bool hi = (lane & bit) != 0;
#pragma unroll
    for (int k = 0; k < step; ++k) {
      const float lo_v = a[k], hi_v = a[k + step];
      const float keep = blend(hi, lo_v, hi_v);
      const float send = blend(hi, hi_v, lo_v);
      a[k] = keep + __shfl_xor(send, bit, 64);
    }
  }
#pragma unroll
  for (int b2 = 32 / S; b2 >= 1; b2 >>= 1) a[0] += __shfl_xor(a[0], b2, 64);
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <int S>
__device__ __forceinline__ int slot_of_lane(int lane) {
  return lane >> (6 - __builtin_ctz((unsigned)S));
}

template <int N>
struct Pow2Ceil { static constexpr int value = 2 * Pow2Ceil<(N + 1) / 2>::value; };
template <>
struct Pow2Ceil<1> { static constexpr int value = 1; };

enum KgMode : int { KG_DOTS = 0, KG_ORTH_DOTS = 1, KG_ORTH_NORM = 2 };

// One pass over w and the basis V_0..V_{cnt-1} of every live problem; each workgroup covers
// KG_ITERS groups of 512 elements of one problem:
//   KG_DOTS:      partial <- V_i . w (slots i < cnt) and w . w (slot cnt)
//   KG_ORTH_DOTS: w <- w - sum_i h_i V_i, then partial <- V_i . w (the group's basis values stay
//                 in registers between the two uses)
//   KG_ORTH_NORM: w <- w - sum_i h_i V_i, then partial <- w . w (slot 0)
// Per-thread products are float32 over the workgroup's 2 * KG_ITERS elements per thread, wave
// sums float32, workgroup and grid sums f64 in a fixed order.  partial layout: [b][slot][block].
template <int MODE, int MAXV>
__global__ __launch_bounds__(KG_THREADS) void kgs_kernel(float* __restrict__ w,
                                                         const float* __restrict__ V, size_t vstride,
                                                         size_t vpad, int cnt, int blocks,
                                                         const double* __restrict__ h,
                                                         double* __restrict__ partial,
                                                         const int* __restrict__ active) {
  constexpr int S = (MODE == KG_ORTH_NORM) ? 1 : Pow2Ceil<MAXV>::value;
  __shared__ double red[4][S];
  __shared__ double redn[4];
  __shared__ double hs[MAXV];
  const int slot = blockIdx.x / blocks, blk = blockIdx.x % blocks;
  const int b = active != nullptr ? active[slot] : slot;
  if (MODE != KG_DOTS) {
    if ((int)threadIdx.x < MAXV)
      hs[threadIdx.x] = (int)threadIdx.x < cnt ? h[(size_t)b * KR_LD + threadIdx.x] : 0.0;
    __syncthreads();
  }
  float acc[S];
#pragma unroll
  for (int i = 0; i < S; ++i) acc[i] = 0.f;
  float nrm = 0.f;
#pragma unroll 1
  for (int it = 0; it < KG_ITERS; ++it) {
    const size_t e = (size_t)b * vpad + ((size_t)blk * KG_ITERS + it) * KG_ELEMS + 2 * threadIdx.x;
    const float2 w2 = *reinterpret_cast<const float2*>(w + e);
    // all MAXV loads are issued unconditionally (slots past cnt re-read V_0, a cache hit) so
    // that none of them waits behind a branch; those slots are zeroed afterwards
    float2 v[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      v[i] = *reinterpret_cast<const float2*>(V + (size_t)(i < cnt ? i : 0) * vstride + e);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      v[i].x = blend(i >= cnt, v[i].x, 0.f);
      v[i].y = blend(i >= cnt, v[i].y, 0.f);
    }
    if (MODE == KG_DOTS) {
#pragma unroll
      for (int i = 0; i < MAXV; ++i) acc[i] = fmaf(v[i].x, w2.x, fmaf(v[i].y, w2.y, acc[i]));
      nrm = fmaf(w2.x, w2.x, fmaf(w2.y, w2.y, nrm));
    } else {
      double x0 = w2.x, x1 = w2.y;
#pragma unroll
      for (int i = 0; i < MAXV; ++i) {
        const double hi = hs[i];
        x0 -= hi * (double)v[i].x;
        x1 -= hi * (double)v[i].y;
      }
      const float2 xf = make_float2((float)x0, (float)x1);
      *reinterpret_cast<float2*>(w + e) = xf;
      if (MODE == KG_ORTH_DOTS) {
#pragma unroll
        for (int i = 0; i < MAXV; ++i) acc[i] = fmaf(v[i].x, xf.x, fmaf(v[i].y, xf.y, acc[i]));
      } else {
        nrm = fmaf(xf.x, xf.x, fmaf(xf.y, xf.y, nrm));
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (MODE != KG_ORTH_NORM) {
    wave_reduce_scatter<S>(acc);
    if ((lane & ((64 / S) - 1)) == 0) red[wv][slot_of_lane<S>(lane)] = (double)acc[0];
  }
  if (MODE != KG_ORTH_DOTS) {
    nrm = wave_sum(nrm);
    if (lane == 0) redn[wv] = (double)nrm;
  }
  __syncthreads();
  double* out = partial + (size_t)b * KR_LD * blocks + blk;
  if (MODE != KG_ORTH_NORM && (int)threadIdx.x < cnt)
    out[(size_t)threadIdx.x * blocks] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
  if (MODE != KG_ORTH_DOTS && threadIdx.x == 0)
    out[(size_t)(MODE == KG_DOTS ? cnt : 0) * blocks] = (redn[0] + redn[1]) + (redn[2] + redn[3]);
}

// out[b][i] = sum over blocks of partial[b][i][block], one wave per (b, i), fixed order.
__global__ __launch_bounds__(256) void kgs_reduce_kernel(const double* __restrict__ partial, int blocks,
                                                         int total, int B, double* __restrict__ out,
                                                         const int* __restrict__ active) {
  const int id = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (id >= B * total) return;
  const int slot = id / total, i = id % total;
  const int b = active != nullptr ? active[slot] : slot;
  const double* p = partial + ((size_t)b * KR_LD + i) * blocks;
  double s = 0.0;
  for (int k = lane; k < blocks; k += 64) s += p[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[(size_t)b * KR_LD + i] = s;
}

template <int MODE, int MAXV>
static void launch_kgs_one(float* w, const float* V, size_t vstride, size_t vpad, int cnt, int blocks,
                           int B, const double* h, double* partial, const int* active, hipStream_t st) {
  hipLaunchKernelGGL((kgs_kernel<MODE, MAXV>), dim3(blocks * B), dim3(KG_THREADS), 0, st, w, V, vstride,
                     vpad, cnt, blocks, h, partial, active);
}

// Register-held basis slice: the instance with the smallest multiple of 8 >= cnt.
template <int MODE>
static void launch_kgs_mode(float* w, const float* V, size_t vstride, size_t vpad, int cnt, int blocks,
                            int B, const double* h, double* partial, const int* active, hipStream_t st) {
  switch ((cnt + 7) / 8) {
    case 0:
    case 1: launch_kgs_one<MODE, 8>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    case 2: launch_kgs_one<MODE, 16>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    case 3: launch_kgs_one<MODE, 24>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    case 4: launch_kgs_one<MODE, 32>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    case 5: launch_kgs_one<MODE, 40>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    case 6: launch_kgs_one<MODE, 48>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    case 7: launch_kgs_one<MODE, 56>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
    default: launch_kgs_one<MODE, 64>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st); break;
  }
}

int launch_gs_pass(int mode, float* w, const float* V, size_t vstride, int cnt, int n, int B,
                   const double* h, double* partial, double* out, const int* active, hipStream_t st) {
  const size_t vpad = krylov_vpad(n);
  const int blocks = krylov_blocks(n);
  if (cnt < 0 || cnt > KRYLOV_MAX_BASIS || (mode != KG_DOTS && cnt < 1)) return -1;
  const int total = (mode == KG_DOTS) ? cnt + 1 : (mode == KG_ORTH_DOTS ? cnt : 1);
  if (mode == KG_DOTS)
    launch_kgs_mode<KG_DOTS>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st);
  else if (mode == KG_ORTH_DOTS)
    launch_kgs_mode<KG_ORTH_DOTS>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st);
  else
    launch_kgs_mode<KG_ORTH_NORM>(w, V, vstride, vpad, cnt, blocks, B, h, partial, active, st);
  const int waves = B * total;
  hipLaunchKernelGGL(kgs_reduce_kernel, dim3((waves + 3) / 4), dim3(256), 0, st, partial, blocks, total,
                     B, out, active);
  return 0;
}

// In-place change of basis: each thread reads element e of all the problem's input vectors and
// writes element e of the k outputs (so overwriting inputs 0..k-1 is safe).  Coefficients are
// wave-uniform (scalar loads).
constexpr int KB_MAX = KRYLOV_MAX_DEFLATE;
__global__ __launch_bounds__(256) void basis_combine_kernel(float* __restrict__ X, size_t stride,
                                                            size_t plen, int k,
                                                            const double* __restrict__ C,
                                                            size_t cstride, int blocks_per_prob,
                                                            const int* __restrict__ active) {
  const int slot = blockIdx.x / blocks_per_prob, blk = blockIdx.x % blocks_per_prob;
  const int b = active != nullptr ? active[slot] : slot;
  const size_t e = (size_t)blk * 256 + threadIdx.x;
  if (e >= plen) return;
  const double* Cb = C + (size_t)b * cstride;
  const int count = (int)Cb[cstride - 1];
  float acc[KB_MAX];
#pragma unroll
  for (int i = 0; i < KB_MAX; ++i) acc[i] = 0.f;
  float* Xb = X + (size_t)b * plen + e;
  for (int j = 0; j < count; ++j) {
    const float x = Xb[(size_t)j * stride];
#pragma unroll
    for (int i = 0; i < KB_MAX; ++i)
      if (i < k) acc[i] = fmaf((float)Cb[(size_t)j * k + i], x, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < KB_MAX; ++i)
    if (i < k) Xb[(size_t)i * stride] = acc[i];
}

void launch_basis_combine(float* X, size_t stride, size_t plen, int cnt, int k, const double* C,
                          size_t cstride, int B, const int* active, hipStream_t st) {
  (void)cnt;
  const int bpp = (int)((plen + 255) / 256);
  hipLaunchKernelGGL(basis_combine_kernel, dim3(bpp * B), dim3(256), 0, st, X, stride, plen, k, C,
                     cstride, bpp, active);
}

// u[b] += sum_{j<cnt} y[b][j] Z_j[b] for the listed problems (terms with y = 0 are skipped:
// their Z_j may be stale)
template <typename UT>
__global__ void combine_kernel(UT* __restrict__ u, const float* __restrict__ Z, size_t zstride,
                               int cnt, size_t nn, int B, const double* __restrict__ y,
                               const int* __restrict__ active) {
  const size_t total = nn * (size_t)B;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const int slot = (int)(k / nn);
    const int b = active != nullptr ? active[slot] : slot;
    const size_t e = (size_t)b * nn + (k - (size_t)slot * nn);
    double acc = 0.0;
    for (int j = 0; j < cnt; ++j) {
      const double yj = y[(size_t)b * KR_LD + j];
      if (yj != 0.0) acc += yj * (double)Z[(size_t)j * zstride + e];
    }
    u[e] = (UT)((double)u[e] + acc);
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
