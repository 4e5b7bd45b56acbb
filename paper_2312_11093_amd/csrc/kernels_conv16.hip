// 16 -> 16 channel 3x3 convolutions of the MGCNN networks on CDNA4 matrix cores.
//
// Every 16->16 conv is an implicit GEMM per output pixel segment:
//     D[o][px] = sum_tap sum_c W[o][c][tap] * Z[c][px + off(tap)]
// with M = 16 output channels, N = 16 pixels of one row segment and K = 9 taps x 16
// channels.  The input tile (with halo) is staged once in LDS, channel-last with a
// padded pixel stride (20 x 4 B for f32, 20 x 2 B for bf16) so that the 16 lanes of
// one operand row read 16 consecutive pixels without bank conflicts.  Each tap is
// then 4 v_mfma_f32_16x16x4f32 (f32 state) or 1 v_mfma_f32_16x16x16bf16 (bf16 state,
// f32 accumulation).  The accumulator layout gives each lane four consecutive output
// channels of one pixel, so the epilogue stores 16 B (f32) / 8 B (bf16) per lane and a
// wave writes one contiguous 1 KB / 512 B row segment.
//
// Kernels:
//   conv16_same    : smoother  y = x + W * (s . x)          (Alg. 3, Eqs. (17)-(18))
//                    setup layer y = x + tanh(W * x + beta)  (Alg. 2, Eq. (6))
//   conv16_restrict: y = W *_{stride 2, no padding} x       (RCNN, Sec. 2.4)
//   prolong_add    : y += W^T-conv_{stride 2} x              (TCNN, Sec. 2.4, Eq. (3))
#include "mgcnn_internal.h"
#include "mgcnn_device.h"

namespace mg {

constexpr int PS = 20;   // LDS pixel stride in elements (16 channels + 4 pad)

// ------------------------------------------------------------------------------------------
// operand helpers
// ------------------------------------------------------------------------------------------
template <int ST>
struct Frag;

// f32 state: per tap 4 MFMA 16x16x4; lane l supplies A[o = l%16][k = l/16] and
// B[k = l/16][px = l%16]; instruction s uses channel c = 4*(l/16) + s, so one 16 B LDS read
// feeds all four instructions of a tap.
template <>
struct Frag<ST_F32> {
  typedef float elem;
  float w[9][4];
  __device__ void load_w(const float* W, bool transposed) {
    const int l = threadIdx.x & 63;
    const int o = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int c = 4 * g + s;
        w[t][s] = transposed ? W[(c * C + o) * 9 + t] : W[(o * C + c) * 9 + t];
      }
  }
  __device__ __forceinline__ f4v mma(int t, const elem* lds_px, f4v acc) const {
    const int g = (threadIdx.x & 63) >> 4;
    const float4 z = *reinterpret_cast<const float4*>(lds_px + 4 * g);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[t][0], z.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[t][1], z.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[t][2], z.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[t][3], z.w, acc, 0, 0, 0);
    return acc;
  }
};

// bf16 state: one MFMA 16x16x16 per tap; lane l supplies A[o = l%16][k = 4*(l/16) + e] and
// B[k = 4*(l/16) + e][px = l%16], e = 0..3, i.e. four consecutive channels (8 B).
template <>
struct Frag<ST_BF16> {
  typedef uint16_t elem;
  s4v w[9];
  __device__ void load_w(const float* W, bool transposed) {
    const int l = threadIdx.x & 63;
    const int o = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 4 * g + e;
        const float v = transposed ? W[(c * C + o) * 9 + t] : W[(o * C + c) * 9 + t];
        w[t][e] = (short)f32_to_bf16_rne(v);
      }
  }
  __device__ __forceinline__ f4v mma(int t, const elem* lds_px, f4v acc) const {
    const int g = (threadIdx.x & 63) >> 4;
    const uint2 z = *reinterpret_cast<const uint2*>(lds_px + 4 * g);
    s4v b;
    b[0] = (short)(z.x & 0xffffu); b[1] = (short)(z.x >> 16);
    b[2] = (short)(z.y & 0xffffu); b[3] = (short)(z.y >> 16);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[t], b, acc, 0, 0, 0);
  }
};

// Load 4 consecutive channels (group g) of pixel `pix` of a channel-last tensor as floats.
__device__ __forceinline__ float4 ld4(const float* X, int pix, int g) {
  return reinterpret_cast<const float4*>(X)[pix * 4 + g];
}
__device__ __forceinline__ float4 ld4(const uint16_t* X, int pix, int g) {
  const uint2 z = reinterpret_cast<const uint2*>(X)[pix * 4 + g];
  return make_float4(__uint_as_float(z.x << 16), __uint_as_float(z.x & 0xffff0000u),
                     __uint_as_float(z.y << 16), __uint_as_float(z.y & 0xffff0000u));
}
__device__ __forceinline__ void st4_lds(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
__device__ __forceinline__ void st4_lds(uint16_t* p, float4 v) {
  *reinterpret_cast<uint2*>(p) = make_uint2(pack_bf16x2(v.x, v.y), pack_bf16x2(v.z, v.w));
}
__device__ __forceinline__ void st4(float* X, int pix, int g, float4 v) {
  reinterpret_cast<float4*>(X)[pix * 4 + g] = v;
}
__device__ __forceinline__ void st4(uint16_t* X, int pix, int g, float4 v) {
  reinterpret_cast<uint2*>(X)[pix * 4 + g] = make_uint2(pack_bf16x2(v.x, v.y), pack_bf16x2(v.z, v.w));
}

// 16-byte staging chunks: 4 f32 channels or 8 bf16 channels of one pixel.  All chunks of a
// tile are loaded into registers first (many loads in flight per lane), then combined and
// written to LDS.
template <int ST>
struct Chunk;
template <>
struct Chunk<ST_F32> {
  static constexpr int CPP = 4;   // chunks per pixel
  typedef float4 T;
  static __device__ __forceinline__ T load(const float* X, int pix, int h) {
    return reinterpret_cast<const float4*>(X)[pix * 4 + h];
  }
  static __device__ __forceinline__ T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ T mul(T a, T b) {
    return make_float4(a.x * b.x, a.y * b.y, a.z * b.z, a.w * b.w);
  }
  static __device__ __forceinline__ void to_lds(float* px, int h, T v) {
    *reinterpret_cast<float4*>(px + 4 * h) = v;
  }
};
template <>
struct Chunk<ST_BF16> {
  static constexpr int CPP = 2;
  typedef uint4 T;
  static __device__ __forceinline__ T load(const uint16_t* X, int pix, int h) {
    return reinterpret_cast<const uint4*>(X)[pix * 2 + h];
  }
  static __device__ __forceinline__ T zero() { return make_uint4(0u, 0u, 0u, 0u); }
  static __device__ __forceinline__ uint32_t mul2(uint32_t a, uint32_t b) {
    const float lo = __uint_as_float(a << 16) * __uint_as_float(b << 16);
    const float hi = __uint_as_float(a & 0xffff0000u) * __uint_as_float(b & 0xffff0000u);
    return pack_bf16x2(lo, hi);
  }
  static __device__ __forceinline__ T mul(T a, T b) {
    return make_uint4(mul2(a.x, b.x), mul2(a.y, b.y), mul2(a.z, b.z), mul2(a.w, b.w));
  }
  static __device__ __forceinline__ void to_lds(uint16_t* px, int h, T v) {
    *reinterpret_cast<uint2*>(px + 8 * h) = make_uint2(v.x, v.y);
    *reinterpret_cast<uint2*>(px + 8 * h + 4) = make_uint2(v.z, v.w);
  }
};

// ------------------------------------------------------------------------------------------
// same-size conv: smoother (s given) or tanh ResNet layer (bias given)
// Tile: 8 output rows x TW columns (TW = 32 for f32, 64 for bf16); each wave owns two rows.
// ------------------------------------------------------------------------------------------
template <int ST>
struct SameCfg {
  static constexpr int TH = 8, TW = (ST == ST_F32) ? 32 : 64;
  static constexpr int IR = TH + 2, IC = TW + 2, NPIX = IR * IC;
  static constexpr int NCHUNK = NPIX * Chunk<ST>::CPP, NPT = (NCHUNK + 255) / 256;
  static constexpr int NSEG = TW / 16, NTASK = TH * NSEG, TPW = NTASK / 4;
};

template <int ST, int MODE>
__global__ __launch_bounds__(256) void conv16_same_kernel(
    const typename Frag<ST>::elem* __restrict__ x, const typename Frag<ST>::elem* __restrict__ s,
    const float* __restrict__ W, const float* __restrict__ bias,
    typename Frag<ST>::elem* __restrict__ y, int m, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef SameCfg<ST> K;
  typedef Chunk<ST> CK;
  __shared__ __attribute__((aligned(16))) E lds[K::NPIX * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int row0 = (tile / tiles_x) * K::TH, col0 = (tile % tiles_x) * K::TW;
  const size_t pbase = (size_t)b * m * m * C;     // problem offset in elements
  const E* Xb = x + pbase;
  const E* Sb = (MODE == CM_SMOOTH) ? s + pbase : nullptr;
  E* Yb = y + pbase;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  // 1. issue every staging load of this thread (x and s with a one-pixel halo)
  typename CK::T xv[K::NPT], sv[K::NPT];
#pragma unroll
  for (int r = 0; r < K::NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    const int pix = k / CK::CPP, h = k % CK::CPP;
    const int lr = pix / K::IC, lc = pix - lr * K::IC;
    const int gi = row0 + lr - 1, gj = col0 + lc - 1;
    const bool ok = k < K::NCHUNK && gi >= 0 && gi < m && gj >= 0 && gj < m;
    const int gp = ok ? gi * m + gj : 0;
    xv[r] = ok ? CK::load(Xb, gp, h) : CK::zero();
    if constexpr (MODE == CM_SMOOTH) sv[r] = ok ? CK::load(Sb, gp, h) : CK::zero();
  }
  // 2. prefetch the skip operand (centre pixels) of this wave's output segments
  float4 xc[K::TPW];
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int gi = row0 + task / K::NSEG, gj = col0 + (task % K::NSEG) * 16 + px;
    xc[tt] = (gi < m && gj < m) ? ld4(Xb, gi * m + gj, g) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  Frag<ST> fr;
  fr.load_w(W, false);
  // 3. z = s . x (smoother) or x (tanh layer) into LDS
#pragma unroll
  for (int r = 0; r < K::NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    if (k < K::NCHUNK) {
      const int pix = k / CK::CPP, h = k % CK::CPP;
      typename CK::T v = xv[r];
      if constexpr (MODE == CM_SMOOTH) v = CK::mul(v, sv[r]);
      CK::to_lds(&lds[pix * PS], h, v);
    }
  }
  __syncthreads();
  // 4. implicit GEMM per 16-pixel segment, then y = x + acc (or x + tanh(acc + bias))
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int orow = task / K::NSEG, seg = task % K::NSEG;
    const int gi = row0 + orow;
    if (gi >= m || col0 + seg * 16 >= m) continue;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((orow + p) * K::IC + seg * 16 + px + q) * PS], acc);
    const int gj = col0 + seg * 16 + px;
    if (gj < m) {
      const float4 c = xc[tt];
      float4 o;
      if constexpr (MODE == CM_TANH) {
        o.x = c.x + tanhf(acc[0] + bias[4 * g + 0]);
        o.y = c.y + tanhf(acc[1] + bias[4 * g + 1]);
        o.z = c.z + tanhf(acc[2] + bias[4 * g + 2]);
        o.w = c.w + tanhf(acc[3] + bias[4 * g + 3]);
      } else {
        o.x = c.x + acc[0]; o.y = c.y + acc[1]; o.z = c.z + acc[2]; o.w = c.w + acc[3];
      }
      st4(Yb, gi * m + gj, g, o);
    }
  }
}

// ------------------------------------------------------------------------------------------
// stride-2 restriction conv, no padding: m -> mo = (m-1)/2
// Tile: TH coarse rows (4 for f32, 8 for bf16) x 32 coarse columns.  Columns of the staged
// fine tile are de-interleaved by parity so that the stride-2 operand reads stay consecutive.
// ------------------------------------------------------------------------------------------
template <int ST>
struct RsCfg {
  static constexpr int TH = (ST == ST_F32) ? 4 : 8, TW = 32;
  static constexpr int IR = 2 * TH + 1, IC = 2 * TW + 1, HALF = TW + 1, ROW = 2 * HALF;
  static constexpr int NPIX = IR * IC, NCHUNK = NPIX * Chunk<ST>::CPP, NPT = (NCHUNK + 255) / 256;
  static constexpr int NSEG = TW / 16, NTASK = TH * NSEG, TPW = NTASK / 4;
};

template <int HALF>
__device__ __forceinline__ int rs_slot(int lc) { return (lc & 1) ? HALF + (lc >> 1) : (lc >> 1); }

template <int ST>
__global__ __launch_bounds__(256) void conv16_restrict_kernel(
    const typename Frag<ST>::elem* __restrict__ x, const float* __restrict__ W,
    typename Frag<ST>::elem* __restrict__ y, int m, int mo, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef RsCfg<ST> K;
  typedef Chunk<ST> CK;
  __shared__ __attribute__((aligned(16))) E lds[K::IR * K::ROW * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int orow0 = (tile / tiles_x) * K::TH, ocol0 = (tile % tiles_x) * K::TW;
  const int frow0 = 2 * orow0, fcol0 = 2 * ocol0;
  const E* Xb = x + (size_t)b * m * m * C;
  E* Yb = y + (size_t)b * mo * mo * C;
  typename CK::T xv[K::NPT];
#pragma unroll
  for (int r = 0; r < K::NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    const int pix = k / CK::CPP, h = k % CK::CPP;
    const int lr = pix / K::IC, lc = pix - lr * K::IC;
    const int gi = frow0 + lr, gj = fcol0 + lc;
    const bool ok = k < K::NCHUNK && gi < m && gj < m;
    xv[r] = ok ? CK::load(Xb, gi * m + gj, h) : CK::zero();
  }
  Frag<ST> fr;
  fr.load_w(W, false);
#pragma unroll
  for (int r = 0; r < K::NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    if (k < K::NCHUNK) {
      const int pix = k / CK::CPP, h = k % CK::CPP;
      const int lr = pix / K::IC, lc = pix - lr * K::IC;
      CK::to_lds(&lds[(lr * K::ROW + rs_slot<K::HALF>(lc)) * PS], h, xv[r]);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int orow = task / K::NSEG, seg = task % K::NSEG;
    const int gi = orow0 + orow;
    if (gi >= mo || ocol0 + seg * 16 >= mo) continue;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    const int jj = seg * 16 + px;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((2 * orow + p) * K::ROW + rs_slot<K::HALF>(2 * jj + q)) * PS], acc);
    const int gj = ocol0 + jj;
    if (gj < mo) st4(Yb, gi * mo + gj, g, make_float4(acc[0], acc[1], acc[2], acc[3]));
  }
}

// ------------------------------------------------------------------------------------------
// prolongation: y_fine += convT_{stride 2}(W_T, x_coarse), fine side m = 2 mc + 1.
// Fine pixel (i, j) receives coarse (I, J) through tap (p, q) with 2I + p = i, 2J + q = j:
// odd i uses p = 1 only, even i uses p = 0 (I = i/2) and p = 2 (I = i/2 - 1); same for j.
// Work is split into row segments of 16 fine pixels of equal column parity, so every lane
// of one MFMA uses the same tap.  Tile: 4 x 32 coarse pixels = 8 x 64 fine pixels.
// ------------------------------------------------------------------------------------------
constexpr int PL_CH = 4, PL_CW = 32;                  // coarse tile
constexpr int PL_IR = PL_CH + 1, PL_IC = PL_CW + 1;   // staged coarse rows/cols (one halo)

template <int ST>
__global__ __launch_bounds__(256) void prolong_add_kernel(
    const typename Frag<ST>::elem* __restrict__ xc, const float* __restrict__ WT,
    typename Frag<ST>::elem* __restrict__ yf, int mc, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef Chunk<ST> CK;
  constexpr int NPIX = PL_IR * PL_IC, NCHUNK = NPIX * CK::CPP, NPT = (NCHUNK + 255) / 256;
  __shared__ __attribute__((aligned(16))) E lds[NPIX * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int m = 2 * mc + 1;
  const int I0 = (tile / tiles_x) * PL_CH, J0 = (tile % tiles_x) * PL_CW;
  const E* Cb = xc + (size_t)b * mc * mc * C;
  E* Fb = yf + (size_t)b * m * m * C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  // fine read-modify-write operands of this wave's 8 segments, fetched first
  float4 yv[8];
#pragma unroll
  for (int task = 0; task < 8; ++task) {
    const int fr_local = wave * 2 + (task >> 2), par = (task >> 1) & 1, jb = task & 1;
    const int i = 2 * I0 + fr_local, j = 2 * (J0 + jb * 16 + px) + par;
    yv[task] = (i < m && j < m) ? ld4(Fb, i * m + j, g) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  typename CK::T cv[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    const int pix = k / CK::CPP, h = k % CK::CPP;
    const int lr = pix / PL_IC, lc = pix - lr * PL_IC;
    const int I = I0 - 1 + lr, J = J0 - 1 + lc;
    const bool ok = k < NCHUNK && I >= 0 && I < mc && J >= 0 && J < mc;
    cv[r] = ok ? CK::load(Cb, I * mc + J, h) : CK::zero();
  }
  Frag<ST> fr;
  fr.load_w(WT, true);
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    if (k < NCHUNK) CK::to_lds(&lds[(k / CK::CPP) * PS], k % CK::CPP, cv[r]);
  }
  __syncthreads();
#pragma unroll
  for (int task = 0; task < 8; ++task) {
    const int fr_local = wave * 2 + (task >> 2);   // fine row within the 8-row tile
    const int par = (task >> 1) & 1;                // fine column parity
    const int jb = task & 1;                        // 16-wide block of coarse columns
    const int i = 2 * I0 + fr_local;
    if (i >= m) continue;
    const int jc = jb * 16 + px;                    // coarse column within the tile
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    const int np = (fr_local & 1) ? 1 : 2;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      if (rt >= np) break;
      int p, lr;
      if (fr_local & 1) { p = 1; lr = (fr_local - 1) / 2 + 1; }
      else if (rt == 0) { p = 0; lr = fr_local / 2 + 1; }
      else { p = 2; lr = fr_local / 2; }
      if (par) {
        acc = fr.mma(p * 3 + 1, &lds[(lr * PL_IC + jc + 1) * PS], acc);
      } else {
        acc = fr.mma(p * 3 + 0, &lds[(lr * PL_IC + jc + 1) * PS], acc);
        acc = fr.mma(p * 3 + 2, &lds[(lr * PL_IC + jc) * PS], acc);
      }
    }
    const int j = 2 * (J0 + jc) + par;
    if (j < m) {
      float4 o = yv[task];
      o.x += acc[0]; o.y += acc[1]; o.z += acc[2]; o.w += acc[3];
      st4(Fb, i * m + j, g, o);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Finest level, down smoother with the reChannel-in conv folded in:
//   x1 = W_in * rt  (1 -> 16, zero padding),  y = x1 + W_dn * (s . x1).
// x1 is computed on the staged tile (one-pixel halo, zero outside the grid) from an LDS copy of
// rt with a two-pixel halo, so x1 never travels through HBM.
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void smooth_in_kernel(
    const float* __restrict__ rt, const typename Frag<ST>::elem* __restrict__ s,
    const float* __restrict__ Win, const float* __restrict__ W,
    typename Frag<ST>::elem* __restrict__ y, int m, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef SameCfg<ST> K;
  constexpr int RR = K::IR + 2, RC = K::IC + 2;          // rt tile (two-pixel halo)
  constexpr int PPT = (K::NPIX + 255) / 256;             // staged pixels per thread
  __shared__ __attribute__((aligned(16))) E lds[K::NPIX * PS];     // z = s . x1
  __shared__ __attribute__((aligned(16))) E lx[K::TH * K::TW * PS];  // x1 at the output pixels
  __shared__ float lrt[RR * RC];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int row0 = (tile / tiles_x) * K::TH, col0 = (tile % tiles_x) * K::TW;
  const size_t pbase = (size_t)b * m * m;
  const E* Sb = s + pbase * C;
  E* Yb = y + pbase * C;
  const float* Rb = rt + pbase;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  // s for the staged pixels (one thread = one whole pixel, 16 channels)
  float sv[PPT][C];
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = threadIdx.x + 256 * r;
    const int lr = pix / K::IC, lc = pix - lr * K::IC;
    const int gi = row0 + lr - 1, gj = col0 + lc - 1;
    const bool ok = pix < K::NPIX && gi >= 0 && gi < m && gj >= 0 && gj < m;
    if (ok) {
      load16(Sb + (size_t)(gi * m + gj) * C, sv[r]);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) sv[r][c] = 0.f;
    }
  }
  for (int k = threadIdx.x; k < RR * RC; k += 256) {
    const int lr = k / RC, lc = k - lr * RC;
    const int gi = row0 + lr - 2, gj = col0 + lc - 2;
    lrt[k] = (gi >= 0 && gi < m && gj >= 0 && gj < m) ? Rb[gi * m + gj] : 0.f;
  }
  Frag<ST> fr;
  fr.load_w(W, false);
  __syncthreads();
  // x1 = W_in * rt on the staged tile (weights are wave-uniform: scalar loads), z = s . x1
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = threadIdx.x + 256 * r;
    if (pix >= K::NPIX) continue;
    const int lr = pix / K::IC, lc = pix - lr * K::IC;
    const int gi = row0 + lr - 1, gj = col0 + lc - 1;
    const bool in = gi >= 0 && gi < m && gj >= 0 && gj < m;
    float nb[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) nb[p * 3 + q] = lrt[(lr + p) * RC + lc + q];
    float x1[C], z[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc = fmaf(Win[c * 9 + k], nb[k], acc);
      acc = in ? acc : 0.f;
      if constexpr (ST == ST_BF16) acc = bf16_to_f32(f32_to_bf16_rne(acc));   // stored-state rounding
      x1[c] = acc;
      z[c] = acc * sv[r][c];
    }
    store16(&lds[pix * PS], z);
    if (lr >= 1 && lr <= K::TH && lc >= 1 && lc <= K::TW) store16(&lx[((lr - 1) * K::TW + lc - 1) * PS], x1);
  }
  __syncthreads();
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int orow = task / K::NSEG, seg = task % K::NSEG;
    const int gi = row0 + orow;
    if (gi >= m || col0 + seg * 16 >= m) continue;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((orow + p) * K::IC + seg * 16 + px + q) * PS], acc);
    const int gj = col0 + seg * 16 + px;
    if (gj < m) {
      const E* xp = &lx[(orow * K::TW + seg * 16 + px) * PS + 4 * g];
      float4 xo;
      if constexpr (ST == ST_F32) {
        xo = *reinterpret_cast<const float4*>(xp);
      } else {
        const uint2 zz = *reinterpret_cast<const uint2*>(xp);
        xo = make_float4(__uint_as_float(zz.x << 16), __uint_as_float(zz.x & 0xffff0000u),
                         __uint_as_float(zz.y << 16), __uint_as_float(zz.y & 0xffff0000u));
      }
      st4(Yb, gi * m + gj, g, make_float4(xo.x + acc[0], xo.y + acc[1], xo.z + acc[2], xo.w + acc[3]));
    }
  }
}

// ------------------------------------------------------------------------------------------
// Finest level, up smoother with the reChannel-out conv and the update folded in:
//   y = v + W_up * (s . v)  on the output tile plus a one-pixel ring (kept in LDS, zero outside
//   the grid), then u += W_out * y on the output tile.  y never travels through HBM.
// Output tile: (TH - 2) x (TW - 2); the MFMA region is TH x TW, staged v region (TH+2)x(TW+2).
// ------------------------------------------------------------------------------------------
template <int ST, typename UT>
__global__ __launch_bounds__(256) void smooth_out_kernel(
    const typename Frag<ST>::elem* __restrict__ v, const typename Frag<ST>::elem* __restrict__ s,
    const float* __restrict__ W, const float* __restrict__ Wout, UT* __restrict__ u, int m,
    int tiles_x, int tiles_per_prob, const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef SameCfg<ST> K;
  typedef Chunk<ST> CK;
  constexpr int OH = K::TH - 2, OW = K::TW - 2;         // output tile
  __shared__ __attribute__((aligned(16))) E lds[K::NPIX * PS];
  __shared__ __attribute__((aligned(16))) E ly[K::TH * K::TW * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  // origin of the MFMA (y) region; the output tile starts one pixel further in
  const int yr0 = (tile / tiles_x) * OH - 1, yc0 = (tile % tiles_x) * OW - 1;
  const size_t pbase = (size_t)b * m * m;
  const E* Vb = v + pbase * C;
  const E* Sb = s + pbase * C;
  UT* Ub = u + pbase;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  typename CK::T xv[K::NPT], sv[K::NPT];
#pragma unroll
  for (int r = 0; r < K::NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    const int pix = k / CK::CPP, h = k % CK::CPP;
    const int lr = pix / K::IC, lc = pix - lr * K::IC;
    const int gi = yr0 + lr - 1, gj = yc0 + lc - 1;
    const bool ok = k < K::NCHUNK && gi >= 0 && gi < m && gj >= 0 && gj < m;
    const int gp = ok ? gi * m + gj : 0;
    xv[r] = ok ? CK::load(Vb, gp, h) : CK::zero();
    sv[r] = ok ? CK::load(Sb, gp, h) : CK::zero();
  }
  float4 xc[K::TPW];
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int gi = yr0 + task / K::NSEG, gj = yc0 + (task % K::NSEG) * 16 + px;
    const bool ok = gi >= 0 && gi < m && gj >= 0 && gj < m;
    xc[tt] = ok ? ld4(Vb, gi * m + gj, g) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  Frag<ST> fr;
  fr.load_w(W, false);
#pragma unroll
  for (int r = 0; r < K::NPT; ++r) {
    const int k = threadIdx.x + 256 * r;
    if (k < K::NCHUNK) CK::to_lds(&lds[(k / CK::CPP) * PS], k % CK::CPP, CK::mul(xv[r], sv[r]));
  }
  __syncthreads();
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int orow = task / K::NSEG, seg = task % K::NSEG;
    const int gi = yr0 + orow;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((orow + p) * K::IC + seg * 16 + px + q) * PS], acc);
    const int gj = yc0 + seg * 16 + px;
    const bool in = gi >= 0 && gi < m && gj >= 0 && gj < m;
    const float4 c = xc[tt];
    // the up-smoothed state (zero outside the grid: padding of the reChannel-out conv)
    st4_lds(&ly[(orow * K::TW + seg * 16 + px) * PS + 4 * g],
            in ? make_float4(c.x + acc[0], c.y + acc[1], c.z + acc[2], c.w + acc[3])
               : make_float4(0.f, 0.f, 0.f, 0.f));
  }
  __syncthreads();
  // u += W_out * y on the output tile (weights wave-uniform: scalar loads)
  for (int k = threadIdx.x; k < OH * OW; k += 256) {
    const int orr = k / OW, occ = k - orr * OW;
    const int gi = yr0 + 1 + orr, gj = yc0 + 1 + occ;
    if (gi >= m || gj >= m) continue;
    float acc = 0.f;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float yv[C];
        load16(&ly[((orr + p) * K::TW + occ + q) * PS], yv);
#pragma unroll
        for (int c2 = 0; c2 < C; ++c2) acc = fmaf(Wout[c2 * 9 + p * 3 + q], yv[c2], acc);
      }
    UT* U = Ub + gi * m + gj;
    *U = *U + (UT)acc;
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
void launch_conv16(ConvMode mode, StateType st_, const void* x, const void* s, const float* W,
                   const float* bias, void* y, int m, int B, const int* active, hipStream_t st) {
  if (mode == CM_RESTRICT) {
    const int mo = (m - 1) / 2;
    const int TW = 32, TH = (st_ == ST_F32) ? RsCfg<ST_F32>::TH : RsCfg<ST_BF16>::TH;
    const int tx = (mo + TW - 1) / TW, ty = (mo + TH - 1) / TH;
    const dim3 grid(tx * ty * B), blk(256);
    if (st_ == ST_F32)
      hipLaunchKernelGGL(conv16_restrict_kernel<ST_F32>, grid, blk, 0, st, (const float*)x, W,
                         (float*)y, m, mo, tx, tx * ty, active);
    else
      hipLaunchKernelGGL(conv16_restrict_kernel<ST_BF16>, grid, blk, 0, st, (const uint16_t*)x, W,
                         (uint16_t*)y, m, mo, tx, tx * ty, active);
    return;
  }
  const int TW = (st_ == ST_F32 || mode == CM_TANH) ? SameCfg<ST_F32>::TW : SameCfg<ST_BF16>::TW;
  const int TH = SameCfg<ST_F32>::TH;
  const int tx = (m + TW - 1) / TW, ty = (m + TH - 1) / TH;
  const dim3 grid(tx * ty * B), blk(256);
  if (mode == CM_SMOOTH) {
    if (st_ == ST_F32)
      hipLaunchKernelGGL((conv16_same_kernel<ST_F32, CM_SMOOTH>), grid, blk, 0, st,
                         (const float*)x, (const float*)s, W, bias, (float*)y, m, tx, tx * ty,
                         active);
    else
      hipLaunchKernelGGL((conv16_same_kernel<ST_BF16, CM_SMOOTH>), grid, blk, 0, st,
                         (const uint16_t*)x, (const uint16_t*)s, W, bias, (uint16_t*)y, m, tx,
                         tx * ty, active);
  } else {
    hipLaunchKernelGGL((conv16_same_kernel<ST_F32, CM_TANH>), grid, blk, 0, st, (const float*)x,
                       (const float*)nullptr, W, bias, (float*)y, m, tx, tx * ty, active);
  }
}

void launch_smooth_in(StateType st_, const float* rt, const void* s, const float* Win, const float* W,
                      void* y, int m, int B, const int* active, hipStream_t st) {
  if (st_ == ST_F32) {
    typedef SameCfg<ST_F32> K;
    const int tx = (m + K::TW - 1) / K::TW, ty = (m + K::TH - 1) / K::TH;
    hipLaunchKernelGGL(smooth_in_kernel<ST_F32>, dim3(tx * ty * B), dim3(256), 0, st, rt,
                       (const float*)s, Win, W, (float*)y, m, tx, tx * ty, active);
  } else {
    typedef SameCfg<ST_BF16> K;
    const int tx = (m + K::TW - 1) / K::TW, ty = (m + K::TH - 1) / K::TH;
    hipLaunchKernelGGL(smooth_in_kernel<ST_BF16>, dim3(tx * ty * B), dim3(256), 0, st, rt,
                       (const uint16_t*)s, Win, W, (uint16_t*)y, m, tx, tx * ty, active);
  }
}

template <int ST, typename UT>
static void smooth_out_launch(const void* v, const void* s, const float* W, const float* Wout, void* u,
                              int m, int B, const int* active, hipStream_t st) {
  typedef SameCfg<ST> K;
  typedef typename Frag<ST>::elem E;
  const int OH = K::TH - 2, OW = K::TW - 2;
  const int tx = (m + OW - 1) / OW, ty = (m + OH - 1) / OH;
  hipLaunchKernelGGL((smooth_out_kernel<ST, UT>), dim3(tx * ty * B), dim3(256), 0, st, (const E*)v,
                     (const E*)s, W, Wout, (UT*)u, m, tx, tx * ty, active);
}

void launch_smooth_out(StateType st_, const void* v, const void* s, const float* W, const float* Wout,
                       void* u, bool u_f64, int m, int B, const int* active, hipStream_t st) {
  if (st_ == ST_F32) {
    if (u_f64) smooth_out_launch<ST_F32, double>(v, s, W, Wout, u, m, B, active, st);
    else smooth_out_launch<ST_F32, float>(v, s, W, Wout, u, m, B, active, st);
  } else {
    if (u_f64) smooth_out_launch<ST_BF16, double>(v, s, W, Wout, u, m, B, active, st);
    else smooth_out_launch<ST_BF16, float>(v, s, W, Wout, u, m, B, active, st);
  }
}

void launch_prolong_add(StateType st_, const void* xc, const float* WT, void* yf, int mc, int B,
                        const int* active, hipStream_t st) {
  const int tx = (mc + PL_CW - 1) / PL_CW + 1, ty = (mc + PL_CH - 1) / PL_CH + 1;
  const dim3 grid(tx * ty * B), blk(256);
  if (st_ == ST_F32)
    hipLaunchKernelGGL(prolong_add_kernel<ST_F32>, grid, blk, 0, st, (const float*)xc, WT,
                       (float*)yf, mc, tx, tx * ty, active);
  else
    hipLaunchKernelGGL(prolong_add_kernel<ST_BF16>, grid, blk, 0, st, (const uint16_t*)xc, WT,
                       (uint16_t*)yf, mc, tx, tx * ty, active);
}

}  // namespace mg
