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
#include <type_traits>

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
  typedef float lds_t;
  static constexpr int PLANES = 1;
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
  __device__ __forceinline__ f4v mma(int t, const lds_t* lds_px, f4v acc, int) const {
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
  typedef uint16_t lds_t;
  static constexpr int PLANES = 1;
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
  __device__ __forceinline__ f4v mma(int t, const lds_t* lds_px, f4v acc, int) const {
    const int g = (threadIdx.x & 63) >> 4;
    const uint2 z = *reinterpret_cast<const uint2*>(lds_px + 4 * g);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[t], __builtin_bit_cast(s4v, z), acc, 0, 0, 0);
  }
};

// Three-way bf16 split of float32: x = hi + mid + lo exactly up to the rounding of lo
// (|error| <= 2^-26 |x|); each difference below is exact in float32.
__device__ __forceinline__ void split3_2(float x0, float x1, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = pack_bf16x2(x0, x1);
  const float r0 = x0 - __uint_as_float(h << 16), r1 = x1 - __uint_as_float(h & 0xffff0000u);
  m = pack_bf16x2(r0, r1);
  const float q0 = r0 - __uint_as_float(m << 16), q1 = r1 - __uint_as_float(m & 0xffff0000u);
  l = pack_bf16x2(q0, q1);
}
__device__ __forceinline__ void split3_4(float4 v, uint2& H, uint2& M, uint2& L) {
  split3_2(v.x, v.y, H.x, M.x, L.x);
  split3_2(v.z, v.w, H.y, M.y, L.y);
}

// f32 state on bf16 matrix cores: the staged operand is kept in LDS as three bf16 planes
// (hi, mid, lo) and the weights as three bf16 fragments; per tap six 16x16x16 MFMAs form
// hi.hi + hi.mid + mid.hi + hi.lo + lo.hi + mid.mid (dropped terms < 2^-24 relative), i.e.
// float32-level products at the bf16 matrix rate.  Lane layout as in the bf16 case.
template <>
struct Frag<ST_F32X> {
  typedef float elem;
  typedef uint16_t lds_t;
  static constexpr int PLANES = 3;
  s4v wh[9], wm[9], wl[9];
  __device__ void load_w(const float* W, bool transposed) {
    const int l = threadIdx.x & 63;
    const int o = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 4 * g + e;
        v[e] = transposed ? W[(c * C + o) * 9 + t] : W[(o * C + c) * 9 + t];
      }
      uint2 H, M, L;
      split3_4(make_float4(v[0], v[1], v[2], v[3]), H, M, L);
      wh[t] = __builtin_bit_cast(s4v, H);
      wm[t] = __builtin_bit_cast(s4v, M);
      wl[t] = __builtin_bit_cast(s4v, L);
    }
  }
  __device__ __forceinline__ f4v mma(int t, const lds_t* lds_px, f4v acc, int pstride) const {
    const int g = (threadIdx.x & 63) >> 4;
    const s4v bh = __builtin_bit_cast(s4v, *reinterpret_cast<const uint2*>(lds_px + 4 * g));
    const s4v bm = __builtin_bit_cast(s4v, *reinterpret_cast<const uint2*>(lds_px + pstride + 4 * g));
    const s4v bl = __builtin_bit_cast(s4v, *reinterpret_cast<const uint2*>(lds_px + 2 * pstride + 4 * g));
    // small terms first
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wm[t], bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wh[t], bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wl[t], bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wh[t], bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wm[t], bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wh[t], bh, acc, 0, 0, 0);
    return acc;
  }
};

// Two-way bf16 split: x = hi + lo + e with |e| <= 2^-17 |x| (hi rounded to nearest, the
// difference exact in float32, lo its bf16 rounding).
__device__ __forceinline__ void split2_4(float4 v, uint2& H, uint2& L) {
  H = make_uint2(pack_bf16x2(v.x, v.y), pack_bf16x2(v.z, v.w));
  L = make_uint2(pack_bf16x2(v.x - __uint_as_float(H.x << 16), v.y - __uint_as_float(H.x & 0xffff0000u)),
                 pack_bf16x2(v.z - __uint_as_float(H.y << 16), v.w - __uint_as_float(H.y & 0xffff0000u)));
}

// f32 state on bf16 matrix cores with a two-way split: two bf16 LDS planes (hi, lo: the bytes
// of one float32 plane, so the tile and the occupancy of the f32 path are kept) and per tap
// three 16x16x16 MFMAs hi.lo + lo.hi + hi.hi.  The dropped lo.lo term and the lo roundings
// leave each product within about 2^-16 of float32: enough for a preconditioner, whose
// rounding a flexible Krylov method absorbs, at about half the matrix time of f32 MFMA.
template <>
struct Frag<ST_F32X2> {
  typedef float elem;
  typedef uint16_t lds_t;
  static constexpr int PLANES = 2;
  s4v wh[9], wl[9];
  __device__ void load_w(const float* W, bool transposed) {
    const int l = threadIdx.x & 63;
    const int o = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 4 * g + e;
        v[e] = transposed ? W[(c * C + o) * 9 + t] : W[(o * C + c) * 9 + t];
      }
      uint2 H, L;
      split2_4(make_float4(v[0], v[1], v[2], v[3]), H, L);
      wh[t] = __builtin_bit_cast(s4v, H);
      wl[t] = __builtin_bit_cast(s4v, L);
    }
  }
  __device__ __forceinline__ f4v mma(int t, const lds_t* lds_px, f4v acc, int pstride) const {
    const int g = (threadIdx.x & 63) >> 4;
    const s4v bh = __builtin_bit_cast(s4v, *reinterpret_cast<const uint2*>(lds_px + 4 * g));
    const s4v bl = __builtin_bit_cast(s4v, *reinterpret_cast<const uint2*>(lds_px + pstride + 4 * g));
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wh[t], bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wl[t], bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wh[t], bh, acc, 0, 0, 0);
    return acc;
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
  static __device__ __forceinline__ void to_lds(float* px, int h, T v, int) {
    *reinterpret_cast<float4*>(px + 4 * h) = v;
  }
};
template <>
struct Chunk<ST_F32X> : Chunk<ST_F32> {
  static __device__ __forceinline__ void to_lds(uint16_t* px, int h, T v, int pstride) {
    uint2 H, M, L;
    split3_4(v, H, M, L);
    *reinterpret_cast<uint2*>(px + 4 * h) = H;
    *reinterpret_cast<uint2*>(px + pstride + 4 * h) = M;
    *reinterpret_cast<uint2*>(px + 2 * pstride + 4 * h) = L;
  }
};
template <>
struct Chunk<ST_F32X2> : Chunk<ST_F32> {
  static __device__ __forceinline__ void to_lds(uint16_t* px, int h, T v, int pstride) {
    uint2 H, L;
    split2_4(v, H, L);
    *reinterpret_cast<uint2*>(px + 4 * h) = H;
    *reinterpret_cast<uint2*>(px + pstride + 4 * h) = L;
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
  static __device__ __forceinline__ void to_lds(uint16_t* px, int h, T v, int) {
    *reinterpret_cast<uint2*>(px + 8 * h) = make_uint2(v.x, v.y);
    *reinterpret_cast<uint2*>(px + 8 * h + 4) = make_uint2(v.z, v.w);
  }
};

// ------------------------------------------------------------------------------------------
// same-size conv: smoother (s given) or tanh ResNet layer (bias given)
// Tile: TH output rows (8 by default; 4 or 16 as tile variants) x TW columns (TW = 32 for f32,
// 64 for bf16); each wave owns TH / 4 rows.
// ------------------------------------------------------------------------------------------
template <int ST, int THV = 8>
struct SameCfg {
  static constexpr int TH = THV, TW = (ST == ST_BF16) ? 64 : 32;
  static constexpr int IR = TH + 2, IC = TW + 2, NPIX = IR * IC;
  static constexpr int NCHUNK = NPIX * Chunk<ST>::CPP, NPT = (NCHUNK + 255) / 256;
  static constexpr int NSEG = TW / 16, NTASK = TH * NSEG, TPW = NTASK / 4;
};

// One output tile of the same-size conv: problem b, tile index `tile` of a grid of side m.
// SBF: s stored as bf16 while the state is f32 (f32 storage only; the bf16 state has bf16 s).
template <int ST, int MODE, bool SBF, int TH>
__device__ __forceinline__ void conv16_same_tile(
    const typename Frag<ST>::elem* __restrict__ x, const void* __restrict__ s,
    const float* __restrict__ W, const float* __restrict__ bias,
    typename Frag<ST>::elem* __restrict__ y, int m, int tiles_x, int b, int tile) {
  typedef typename Frag<ST>::elem E;
  typedef SameCfg<ST, TH> K;
  typedef Chunk<ST> CK;
  constexpr int PSTR = K::NPIX * PS;                  // LDS plane stride
  __shared__ __attribute__((aligned(16))) typename Frag<ST>::lds_t lds[Frag<ST>::PLANES * PSTR];
  const int row0 = (tile / tiles_x) * K::TH, col0 = (tile % tiles_x) * K::TW;
  const size_t pbase = (size_t)b * m * m * C;     // problem offset in elements
  const E* Xb = x + pbase;
  constexpr bool HAS_S = MODE == CM_SMOOTH || MODE == CM_SMOOTH_POST;
  const E* Sb = (HAS_S && !SBF) ? (const E*)s + pbase : nullptr;
  const uint16_t* Sh = (HAS_S && SBF) ? (const uint16_t*)s + pbase : nullptr;
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
    if constexpr (MODE == CM_SMOOTH && !SBF) sv[r] = ok ? CK::load(Sb, gp, h) : CK::zero();
    if constexpr (MODE == CM_SMOOTH && SBF) sv[r] = ok ? ld4(Sh, gp, h) : CK::zero();   // 4 bf16 channels
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
      CK::to_lds(&lds[pix * PS], h, v, PSTR);
    }
  }
  __syncthreads();
  // 4. implicit GEMM per 16-pixel segment, then y = x + acc (or x + tanh(acc + bias))
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int orow = task / K::NSEG, seg = task % K::NSEG;
    const int gi = row0 + orow;   // segments past the grid are computed (zero staged tile), not stored
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((orow + p) * K::IC + seg * 16 + px + q) * PS], acc, PSTR);
    const int gj = col0 + seg * 16 + px;
    if (gi < m && gj < m) {
      const float4 c = xc[tt];
      float4 o;
      if constexpr (MODE == CM_TANH) {
        o.x = c.x + mg_tanh(acc[0] + bias[4 * g + 0]);
        o.y = c.y + mg_tanh(acc[1] + bias[4 * g + 1]);
        o.z = c.z + mg_tanh(acc[2] + bias[4 * g + 2]);
        o.w = c.w + mg_tanh(acc[3] + bias[4 * g + 3]);
      } else if constexpr (MODE == CM_SMOOTH_POST) {
        // s of the output pixel's four channels multiplies the convolution (adjoint form)
        float4 so;
        if constexpr (SBF) so = ld4(Sh, gi * m + gj, g);
        else so = ld4(Sb, gi * m + gj, g);
        o.x = c.x + so.x * acc[0]; o.y = c.y + so.y * acc[1];
        o.z = c.z + so.z * acc[2]; o.w = c.w + so.w * acc[3];
      } else {
        o.x = c.x + acc[0]; o.y = c.y + acc[1]; o.z = c.z + acc[2]; o.w = c.w + acc[3];
      }
      st4(Yb, gi * m + gj, g, o);
    }
  }
}

template <int ST, int MODE, bool SBF = false, int TH = 8>
__global__ __launch_bounds__(256) void conv16_same_kernel(
    const typename Frag<ST>::elem* __restrict__ x, const void* __restrict__ s,
    const float* __restrict__ W, const float* __restrict__ bias,
    typename Frag<ST>::elem* __restrict__ y, int m, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  conv16_same_tile<ST, MODE, SBF, TH>(x, s, W, bias, y, m, tiles_x, b, tile);
}

// One tanh layer of the setup network on every level at once (Alg. 2, Setup2: the levels do not
// depend on each other once the restricted coefficient tensors exist): workgroup t belongs to
// the level whose tile range [start_l, start_{l+1}) contains it.
struct SetupLevels {
  const float* x[MAX_LEVELS];
  float* y[MAX_LEVELS];
  int m[MAX_LEVELS], tiles_x[MAX_LEVELS], tiles_per_prob[MAX_LEVELS], start[MAX_LEVELS + 1];
  int L;
};

template <int ST, int TH>
__global__ __launch_bounds__(256) void conv16_tanh_levels_kernel(SetupLevels lv, const float* __restrict__ W,
                                                                 const float* __restrict__ bias) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  int l = 0;
  while (l + 1 < lv.L && t >= lv.start[l + 1]) ++l;
  const int u = t - lv.start[l];
  const int slot = u / lv.tiles_per_prob[l], tile = u % lv.tiles_per_prob[l];
  conv16_same_tile<ST, CM_TANH, false, TH>(lv.x[l], nullptr, W, bias, lv.y[l], lv.m[l], lv.tiles_x[l], slot, tile);
}

// ------------------------------------------------------------------------------------------
// stride-2 restriction conv, no padding: m -> mo = (m-1)/2
// Tile: TH coarse rows (4 for f32, 8 for bf16) x 32 coarse columns.  Columns of the staged
// fine tile are de-interleaved by parity so that the stride-2 operand reads stay consecutive.
// ------------------------------------------------------------------------------------------
template <int ST, int THV = 0>
struct RsCfg {
  static constexpr int TH = THV ? THV : ((ST == ST_BF16) ? 8 : 4), TW = 32;
  static constexpr int IR = 2 * TH + 1, IC = 2 * TW + 1, HALF = TW + 1, ROW = 2 * HALF;
  static constexpr int NPIX = IR * IC, NCHUNK = NPIX * Chunk<ST>::CPP, NPT = (NCHUNK + 255) / 256;
  static constexpr int NSEG = TW / 16, NTASK = TH * NSEG, TPW = NTASK / 4;
};

template <int HALF>
__device__ __forceinline__ int rs_slot(int lc) { return (lc & 1) ? HALF + (lc >> 1) : (lc >> 1); }

template <int ST, int TH = 0>
__global__ __launch_bounds__(256) void conv16_restrict_kernel(
    const typename Frag<ST>::elem* __restrict__ x, const float* __restrict__ W,
    typename Frag<ST>::elem* __restrict__ y, int m, int mo, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef RsCfg<ST, TH> K;
  typedef Chunk<ST> CK;
  constexpr int PSTR = K::IR * K::ROW * PS;           // LDS plane stride
  __shared__ __attribute__((aligned(16))) typename Frag<ST>::lds_t lds[Frag<ST>::PLANES * PSTR];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
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
      CK::to_lds(&lds[(lr * K::ROW + rs_slot<K::HALF>(lc)) * PS], h, xv[r], PSTR);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  // tap-major over the wave's segments: independent accumulation chains (the staged tile is
  // zero outside the grid, so every segment may be computed; only the stores are guarded)
  f4v accs[K::TPW];
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) accs[tt] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int tt = 0; tt < K::TPW; ++tt) {
        const int task = wave * K::TPW + tt;
        const int orow = task / K::NSEG, jj = (task % K::NSEG) * 16 + px;
        accs[tt] = fr.mma(p * 3 + q, &lds[((2 * orow + p) * K::ROW + rs_slot<K::HALF>(2 * jj + q)) * PS],
                          accs[tt], PSTR);
      }
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int gi = orow0 + task / K::NSEG, gj = ocol0 + (task % K::NSEG) * 16 + px;
    const f4v acc = accs[tt];
    if (gi < mo && gj < mo) st4(Yb, gi * mo + gj, g, make_float4(acc[0], acc[1], acc[2], acc[3]));
  }
}

// ------------------------------------------------------------------------------------------
// prolongation: y_fine += convT_{stride 2}(W_T, x_coarse), fine side m = 2 mc + 1.
// Fine pixel (i, j) receives coarse (I, J) through tap (p, q) with 2I + p = i, 2J + q = j:
// odd i uses p = 1 only, even i uses p = 0 (I = i/2) and p = 2 (I = i/2 - 1); same for j.
// Work is split into row segments of 16 fine pixels of equal column parity, so every lane
// of one MFMA uses the same tap.  Tile: PL_CH x 32 coarse pixels = 2 PL_CH x 64 fine pixels
// (PL_CH = 4 by default; 2 or 8 as tile variants); each wave owns PL_CH / 2 fine rows.
// ------------------------------------------------------------------------------------------
constexpr int PL_CW = 32;                             // coarse tile columns

template <int ST, int PL_CH = 4>
__global__ __launch_bounds__(256) void prolong_add_kernel(
    const typename Frag<ST>::elem* __restrict__ xc, const float* __restrict__ WT,
    typename Frag<ST>::elem* __restrict__ yf, int mc, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef Chunk<ST> CK;
  constexpr int PL_IR = PL_CH + 1, PL_IC = PL_CW + 1;   // staged coarse rows/cols (one halo)
  constexpr int FRW = PL_CH / 2, NT = 4 * FRW;          // fine rows and segments per wave
  constexpr int NPIX = PL_IR * PL_IC, NCHUNK = NPIX * CK::CPP, NPT = (NCHUNK + 255) / 256;
  constexpr int PSTR = NPIX * PS;                     // LDS plane stride
  __shared__ __attribute__((aligned(16))) typename Frag<ST>::lds_t lds[Frag<ST>::PLANES * PSTR];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  const int m = 2 * mc + 1;
  const int I0 = (tile / tiles_x) * PL_CH, J0 = (tile % tiles_x) * PL_CW;
  const E* Cb = xc + (size_t)b * mc * mc * C;
  E* Fb = yf + (size_t)b * m * m * C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  // fine read-modify-write operands of this wave's segments, fetched first
  float4 yv[NT];
#pragma unroll
  for (int task = 0; task < NT; ++task) {
    const int fr_local = wave * FRW + (task >> 2), par = (task >> 1) & 1, jb = task & 1;
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
    if (k < NCHUNK) CK::to_lds(&lds[(k / CK::CPP) * PS], k % CK::CPP, cv[r], PSTR);
  }
  __syncthreads();
#pragma unroll
  for (int task = 0; task < NT; ++task) {
    const int fr_local = wave * FRW + (task >> 2);  // fine row within the tile
    const int par = (task >> 1) & 1;                // fine column parity
    const int jb = task & 1;                        // 16-wide block of coarse columns
    const int i = 2 * I0 + fr_local;   // rows past the grid are computed too (the staged coarse
                                       // tile is zero there) and not stored, so the segments'
                                       // loads and MFMAs can be scheduled together
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
        acc = fr.mma(p * 3 + 1, &lds[(lr * PL_IC + jc + 1) * PS], acc, PSTR);
      } else {
        acc = fr.mma(p * 3 + 0, &lds[(lr * PL_IC + jc + 1) * PS], acc, PSTR);
        acc = fr.mma(p * 3 + 2, &lds[(lr * PL_IC + jc) * PS], acc, PSTR);
      }
    }
    const int j = 2 * (J0 + jc) + par;
    if (i < m && j < m) {
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
// rt with a two-pixel halo, so x1 never travels through HBM.  The skip term x1 at the output
// pixels is, with f32 state, three more 16x16x4 MFMAs per segment into the same accumulator
// (W_in as a 16 x 12 matrix, taps 9..11 zero, against the nine rt values around each pixel);
// with bf16 state it is the rounded stored x1, kept in LDS.
// PAIR (packed pairs of problems, networks of at most 8 hidden channels): slot b carries problem
// 2b in channels 0..7 and problem 2b + 1 in channels 8..15; rt holds 2 x slots planes, and each
// half of x1 comes from its own plane with the first eight rows of W_in.
// ------------------------------------------------------------------------------------------
template <int ST, bool SBF = false, int TH = 8, bool PAIR = false>
__global__ __launch_bounds__(256) void smooth_in_kernel(
    const float* __restrict__ rt, const void* __restrict__ s,
    const float* __restrict__ Win, const float* __restrict__ W,
    typename Frag<ST>::elem* __restrict__ y, int m, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  typedef SameCfg<ST, TH> K;
  constexpr int RR = K::IR + 2, RC = K::IC + 2;          // rt tile (two-pixel halo)
  constexpr int PPT = (K::NPIX + 255) / 256;             // staged pixels per thread
  constexpr int RPT = (RR * RC + 255) / 256;             // rt values per thread
  constexpr int PSTR = K::NPIX * PS;                     // LDS plane stride
  constexpr int NRT = PAIR ? 2 : 1;                      // rt planes
  __shared__ __attribute__((aligned(16))) typename Frag<ST>::lds_t lds[Frag<ST>::PLANES * PSTR];  // z = s . x1
  constexpr bool SKIP_MMA = ST == ST_F32 || ST == ST_F32X2;   // skip term on the matrix cores
  __shared__ __attribute__((aligned(16))) E lx[SKIP_MMA ? 4 : K::TH * K::TW * PS];  // x1 at the outputs
  __shared__ float lrt[NRT][RR * RC];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  const int row0 = (tile / tiles_x) * K::TH, col0 = (tile % tiles_x) * K::TW;
  const size_t pbase = (size_t)b * m * m;
  typedef typename std::conditional<SBF, uint16_t, E>::type SE;   // storage type of s
  const SE* Sb = (const SE*)s + pbase * C;
  E* Yb = y + pbase * C;
  const float* Rb = rt + (PAIR ? 2 * pbase : pbase);     // plane h of the slot at Rb + h m^2
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  // 1. every global load of this thread first: the rt tile, then s of the staged pixels
  float rv[NRT][RPT];
#pragma unroll
  for (int h = 0; h < NRT; ++h)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int k = threadIdx.x + 256 * r;
      const int lr = k / RC, lc = k - lr * RC;
      const int gi = row0 + lr - 2, gj = col0 + lc - 2;
      rv[h][r] = (k < RR * RC && gi >= 0 && gi < m && gj >= 0 && gj < m) ? Rb[(size_t)h * m * m + gi * m + gj]
                                                                       : 0.f;
    }
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
#pragma unroll
  for (int h = 0; h < NRT; ++h)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int k = threadIdx.x + 256 * r;
      if (k < RR * RC) lrt[h][k] = rv[h][r];
    }
  Frag<ST> fr;
  fr.load_w(W, false);
  __syncthreads();
  // 2. x1 = W_in * rt on the staged tile (weights are wave-uniform: scalar loads), z = s . x1
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = threadIdx.x + 256 * r;
    if (pix >= K::NPIX) continue;
    const int lr = pix / K::IC, lc = pix - lr * K::IC;
    const int gi = row0 + lr - 1, gj = col0 + lc - 1;
    const bool in = gi >= 0 && gi < m && gj >= 0 && gj < m;
    float nb[NRT][9];
#pragma unroll
    for (int h = 0; h < NRT; ++h)
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) nb[h][p * 3 + q] = lrt[h][(lr + p) * RC + lc + q];
    float x1[C], z[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int h = PAIR ? c / 8 : 0, cw = PAIR ? c % 8 : c;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc = fmaf(Win[cw * 9 + k], nb[h][k], acc);
      acc = in ? acc : 0.f;
      if constexpr (ST == ST_BF16) acc = bf16_to_f32(f32_to_bf16_rne(acc));   // stored-state rounding
      x1[c] = acc;
      z[c] = acc * sv[r][c];
    }
    if constexpr (ST == ST_F32X || ST == ST_F32X2) {
#pragma unroll
      for (int h = 0; h < 4; ++h)
        Chunk<ST>::to_lds(&lds[pix * PS], h, make_float4(z[4 * h], z[4 * h + 1], z[4 * h + 2], z[4 * h + 3]),
                          PSTR);
    } else {
      store16(&lds[pix * PS], z);
    }
    if constexpr (!SKIP_MMA)
      if (lr >= 1 && lr <= K::TH && lc >= 1 && lc <= K::TW) store16(&lx[((lr - 1) * K::TW + lc - 1) * PS], x1);
  }
  // A operand of the skip MFMAs: lane (px, g) holds W_in[channel px][k = 4 s + g] for instruction s,
  // k running over the nine taps of each rt plane (PAIR: channel px reads plane px / 8 only)
  constexpr int NSK = PAIR ? 6 : 3;
  float wsk[NSK];
#pragma unroll
  for (int s3 = 0; s3 < NSK; ++s3) {
    const int kk = 4 * s3 + g, h = kk / 9, tap = kk % 9;
    const bool use = SKIP_MMA && kk < 9 * NRT && (!PAIR || h == px / 8);
    wsk[s3] = use ? Win[(PAIR ? px % 8 : px) * 9 + tap] : 0.f;
  }
  __syncthreads();
  // 3. implicit GEMM per 16-pixel segment, y = x1 + acc
#pragma unroll
  for (int tt = 0; tt < K::TPW; ++tt) {
    const int task = wave * K::TPW + tt;
    const int orow = task / K::NSEG, seg = task % K::NSEG;
    const int gi = row0 + orow;   // segments past the grid are computed (zero staged tile), not stored
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (SKIP_MMA) {
      // x1 at the output pixel: B[k = g][px] = rt of plane k / 9 at tap k % 9, k = 4 s + g (zero
      // past the last plane)
#pragma unroll
      for (int s3 = 0; s3 < NSK; ++s3) {
        const int kk = 4 * s3 + g;
        const bool in = kk < 9 * NRT;
        const int h = in ? kk / 9 : 0, tp = in ? kk % 9 : 0;
        const float rb = lrt[h][(orow + 1 + tp / 3) * RC + seg * 16 + px + 1 + tp % 3];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wsk[s3], in ? rb : 0.f, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((orow + p) * K::IC + seg * 16 + px + q) * PS], acc, PSTR);
    const int gj = col0 + seg * 16 + px;
    if (gi < m && gj < m) {
      float4 xo;
      if constexpr (SKIP_MMA) {
        xo = make_float4(0.f, 0.f, 0.f, 0.f);
      } else if constexpr (ST != ST_BF16) {
        xo = *reinterpret_cast<const float4*>(&lx[(orow * K::TW + seg * 16 + px) * PS + 4 * g]);
      } else {
        const E* xp = &lx[(orow * K::TW + seg * 16 + px) * PS + 4 * g];
        const uint2 zz = *reinterpret_cast<const uint2*>(xp);
        xo = make_float4(__uint_as_float(zz.x << 16), __uint_as_float(zz.x & 0xffff0000u),
                         __uint_as_float(zz.y << 16), __uint_as_float(zz.y & 0xffff0000u));
      }
      st4(Yb, gi * m + gj, g, make_float4(xo.x + acc[0], xo.y + acc[1], xo.z + acc[2], xo.w + acc[3]));
    }
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
// ---- tile variants (autotuning) ----------------------------------------------------------
// Rows of the output tile per variant: variant 0 is the default shape.  Variant tables per
// (operation, storage, level side) are set through mgcnn_set_tile_variant (process-wide); the
// per-pixel arithmetic and its order do not depend on the tile, so every variant gives the same
// results bit for bit.
// The same-size convs (and the finest down smoother) have five variants; the restriction and the
// prolongation three (rows 0 = no such variant).
constexpr int SAME_ROWS[TILE_VARIANTS] = {8, 4, 16, 10, 12};
constexpr int PROLONG_ROWS[TILE_VARIANTS] = {8, 4, 16, 0, 0};   // fine rows (2 x coarse rows)
constexpr int RS_ROWS_F32[TILE_VARIANTS] = {4, 2, 8, 0, 0};
constexpr int RS_ROWS_BF16[TILE_VARIANTS] = {8, 4, 16, 0, 0};
static int g_tile_variant[TILE_OPS][2][13] = {};     // [op][bf16 storage][log2(m + 1)]

static int lg2p1(int m) {
  int p = 0;
  while ((1 << p) < m + 1 && p < 12) ++p;
  return p;
}

int tile_variant_rows(int op, bool bf16, int v) {
  if (v < 0 || v >= TILE_VARIANTS) return 0;
  if (op == TILE_RESTRICT) return bf16 ? RS_ROWS_BF16[v] : RS_ROWS_F32[v];
  if (op == TILE_PROLONG) return PROLONG_ROWS[v];
  return SAME_ROWS[v];
}
int get_tile_variant(int op, bool bf16, int m) { return g_tile_variant[op][bf16 ? 1 : 0][lg2p1(m)]; }
void set_tile_variant(int op, bool bf16, int m, int v) { g_tile_variant[op][bf16 ? 1 : 0][lg2p1(m)] = v; }

template <int ST, int MODE, bool SBF, int TH>
static void same_launch(const void* x, const void* s, const float* W, const float* bias, void* y, int m,
                        int B, const int* active, hipStream_t st) {
  typedef typename Frag<ST>::elem E;
  typedef SameCfg<ST, TH> K;
  const int tx = (m + K::TW - 1) / K::TW, ty = (m + K::TH - 1) / K::TH;
  hipLaunchKernelGGL((conv16_same_kernel<ST, MODE, SBF, TH>), dim3(tx * ty * B), dim3(256), 0, st,
                     (const E*)x, s, W, bias, (E*)y, m, tx, tx * ty, active);
}

template <int ST, int MODE, bool SBF>
static void same_variant(int v, const void* x, const void* s, const float* W, const float* bias, void* y,
                         int m, int B, const int* active, hipStream_t st) {
  if (v == 1) same_launch<ST, MODE, SBF, 4>(x, s, W, bias, y, m, B, active, st);
  else if (v == 2) same_launch<ST, MODE, SBF, 16>(x, s, W, bias, y, m, B, active, st);
  else if (v == 3) same_launch<ST, MODE, SBF, 10>(x, s, W, bias, y, m, B, active, st);
  else if (v == 4) same_launch<ST, MODE, SBF, 12>(x, s, W, bias, y, m, B, active, st);
  else same_launch<ST, MODE, SBF, 8>(x, s, W, bias, y, m, B, active, st);
}

template <int ST, int TH>
static void restrict_launch(const void* x, const float* W, void* y, int m, int B, const int* active,
                            hipStream_t st) {
  typedef typename Frag<ST>::elem E;
  typedef RsCfg<ST, TH> K;
  const int mo = (m - 1) / 2;
  const int tx = (mo + K::TW - 1) / K::TW, ty = (mo + K::TH - 1) / K::TH;
  hipLaunchKernelGGL((conv16_restrict_kernel<ST, TH>), dim3(tx * ty * B), dim3(256), 0, st, (const E*)x, W,
                     (E*)y, m, mo, tx, tx * ty, active);
}

template <int ST, bool SBF = false>
static void conv16_launch(ConvMode mode, const void* x, const void* s, const float* W, const float* bias,
                          void* y, int m, int B, const int* active, hipStream_t st) {
  constexpr bool BF = ST == ST_BF16;
  if (mode == CM_RESTRICT) {
    const int v = get_tile_variant(TILE_RESTRICT, BF, m);
    constexpr int R1 = BF ? RS_ROWS_BF16[1] : RS_ROWS_F32[1], R2 = BF ? RS_ROWS_BF16[2] : RS_ROWS_F32[2];
    if (v == 1) restrict_launch<ST, R1>(x, W, y, m, B, active, st);
    else if (v == 2) restrict_launch<ST, R2>(x, W, y, m, B, active, st);
    else restrict_launch<ST, 0>(x, W, y, m, B, active, st);
    return;
  }
  if (mode == CM_SMOOTH)
    same_variant<ST, CM_SMOOTH, SBF>(get_tile_variant(TILE_SMOOTHER, BF, m), x, s, W, bias, y, m, B, active, st);
  else if (mode == CM_SMOOTH_POST)
    same_variant<ST, CM_SMOOTH_POST, SBF>(get_tile_variant(TILE_SMOOTHER, BF, m), x, s, W, bias, y, m, B,
                                          active, st);
  else if constexpr (ST != ST_BF16 && !SBF)
    same_variant<ST, CM_TANH, false>(get_tile_variant(TILE_SETUP, BF, m), x, nullptr, W, bias, y, m, B,
                                     active, st);
}

template <int ST, int TH>
static void tanh_levels_launch(const float* const* x, float* const* y, const int* m, const int* B, int L,
                               const float* W, const float* bias, hipStream_t st) {
  typedef SameCfg<ST, TH> K;
  SetupLevels lv{};
  lv.L = L;
  lv.start[0] = 0;
  for (int l = 0; l < L; ++l) {
    lv.x[l] = x[l];
    lv.y[l] = y[l];
    lv.m[l] = m[l];
    lv.tiles_x[l] = (m[l] + K::TW - 1) / K::TW;
    lv.tiles_per_prob[l] = lv.tiles_x[l] * ((m[l] + K::TH - 1) / K::TH);
    lv.start[l + 1] = lv.start[l] + lv.tiles_per_prob[l] * B[l];
  }
  hipLaunchKernelGGL((conv16_tanh_levels_kernel<ST, TH>), dim3(lv.start[L]), dim3(256), 0, st, lv, W, bias);
}

void launch_tanh_levels(StateType t, const float* const* x, float* const* y, const int* m, const int* B,
                        int L, const float* W, const float* bias, hipStream_t st) {
  if (L < 1 || L > MAX_LEVELS) return;
  const int v = get_tile_variant(TILE_SETUP, false, m[0]);
  if (t == ST_F32X) {
    if (v == 1) tanh_levels_launch<ST_F32X, 4>(x, y, m, B, L, W, bias, st);
    else if (v == 2) tanh_levels_launch<ST_F32X, 16>(x, y, m, B, L, W, bias, st);
    else if (v == 3) tanh_levels_launch<ST_F32X, 10>(x, y, m, B, L, W, bias, st);
    else if (v == 4) tanh_levels_launch<ST_F32X, 12>(x, y, m, B, L, W, bias, st);
    else tanh_levels_launch<ST_F32X, 8>(x, y, m, B, L, W, bias, st);
  } else if (t == ST_F32X2) {
    if (v == 1) tanh_levels_launch<ST_F32X2, 4>(x, y, m, B, L, W, bias, st);
    else if (v == 2) tanh_levels_launch<ST_F32X2, 16>(x, y, m, B, L, W, bias, st);
    else if (v == 3) tanh_levels_launch<ST_F32X2, 10>(x, y, m, B, L, W, bias, st);
    else if (v == 4) tanh_levels_launch<ST_F32X2, 12>(x, y, m, B, L, W, bias, st);
    else tanh_levels_launch<ST_F32X2, 8>(x, y, m, B, L, W, bias, st);
  } else {
    if (v == 1) tanh_levels_launch<ST_F32, 4>(x, y, m, B, L, W, bias, st);
    else if (v == 2) tanh_levels_launch<ST_F32, 16>(x, y, m, B, L, W, bias, st);
    else if (v == 3) tanh_levels_launch<ST_F32, 10>(x, y, m, B, L, W, bias, st);
    else if (v == 4) tanh_levels_launch<ST_F32, 12>(x, y, m, B, L, W, bias, st);
    else tanh_levels_launch<ST_F32, 8>(x, y, m, B, L, W, bias, st);
  }
}

void launch_conv16(ConvMode mode, StateType st_, const void* x, const void* s, const float* W,
                   const float* bias, void* y, int m, int B, const int* active, hipStream_t st,
                   bool s_bf16) {
  // With f32 storage the same-size convs (smoothers and the setup network's tanh layers) use
  // the split when asked (measured faster there); the restriction keeps f32 MFMA (larger LDS
  // tile, lower occupancy with three planes).  bf16 storage has no tanh layers.
  const bool sb = s_bf16 && st_ != ST_BF16 && (mode == CM_SMOOTH || mode == CM_SMOOTH_POST);
  if (st_ == ST_F32 || (st_ == ST_F32X && mode == CM_RESTRICT)) {
    if (sb) conv16_launch<ST_F32, true>(mode, x, s, W, bias, y, m, B, active, st);
    else conv16_launch<ST_F32>(mode, x, s, W, bias, y, m, B, active, st);
  } else if (st_ == ST_F32X) {
    if (sb) conv16_launch<ST_F32X, true>(mode, x, s, W, bias, y, m, B, active, st);
    else conv16_launch<ST_F32X>(mode, x, s, W, bias, y, m, B, active, st);
  } else {
    conv16_launch<ST_BF16>(mode, x, s, W, bias, y, m, B, active, st);
  }
}

template <int ST, bool SBF, int TH, bool PAIR>
static void smooth_in_launch_th(const float* rt, const void* s, const float* Win, const float* W, void* y,
                                int m, int B, const int* active, hipStream_t st) {
  typedef SameCfg<ST, TH> K;
  typedef typename Frag<ST>::elem E;
  const int tx = (m + K::TW - 1) / K::TW, ty = (m + K::TH - 1) / K::TH;
  hipLaunchKernelGGL((smooth_in_kernel<ST, SBF, TH, PAIR>), dim3(tx * ty * B), dim3(256), 0, st, rt, s, Win,
                     W, (E*)y, m, tx, tx * ty, active);
}

template <int ST, bool SBF = false, bool PAIR = false>
static void smooth_in_launch(const float* rt, const void* s, const float* Win, const float* W, void* y,
                             int m, int B, const int* active, hipStream_t st) {
  const int v = get_tile_variant(TILE_SMOOTH_IN, ST == ST_BF16, m);
  if (v == 1) smooth_in_launch_th<ST, SBF, 4, PAIR>(rt, s, Win, W, y, m, B, active, st);
  else if (v == 2) smooth_in_launch_th<ST, SBF, 16, PAIR>(rt, s, Win, W, y, m, B, active, st);
  else if (v == 3) smooth_in_launch_th<ST, SBF, 10, PAIR>(rt, s, Win, W, y, m, B, active, st);
  else if (v == 4) smooth_in_launch_th<ST, SBF, 12, PAIR>(rt, s, Win, W, y, m, B, active, st);
  else smooth_in_launch_th<ST, SBF, 8, PAIR>(rt, s, Win, W, y, m, B, active, st);
}

void launch_smooth_in(StateType st_, const float* rt, const void* s, const float* Win, const float* W,
                      void* y, int m, int B, const int* active, hipStream_t st, bool s_bf16, bool pairs) {
  // f32 storage: f32 MFMA (the split variant measured slower: its three LDS planes halve the
  // occupancy of this kernel).  Packed pairs keep the setup tensors in the state's type.
  if (pairs) {
    if (st_ == ST_F32 || st_ == ST_F32X) smooth_in_launch<ST_F32, false, true>(rt, s, Win, W, y, m, B, active, st);
    else if (st_ == ST_F32X2) smooth_in_launch<ST_F32X2, false, true>(rt, s, Win, W, y, m, B, active, st);
    else smooth_in_launch<ST_BF16, false, true>(rt, s, Win, W, y, m, B, active, st);
    return;
  }
  if (st_ == ST_F32 || st_ == ST_F32X) {
    if (s_bf16) smooth_in_launch<ST_F32, true>(rt, s, Win, W, y, m, B, active, st);
    else smooth_in_launch<ST_F32>(rt, s, Win, W, y, m, B, active, st);
  } else if (st_ == ST_F32X2) {
    if (s_bf16) smooth_in_launch<ST_F32X2, true>(rt, s, Win, W, y, m, B, active, st);
    else smooth_in_launch<ST_F32X2>(rt, s, Win, W, y, m, B, active, st);
  } else {
    smooth_in_launch<ST_BF16>(rt, s, Win, W, y, m, B, active, st);
  }
}

template <int ST, int PL_CH>
static void prolong_launch_ch(const void* xc, const float* WT, void* yf, int mc, int B, const int* active,
                              hipStream_t st) {
  typedef typename Frag<ST>::elem E;
  const int tx = (mc + PL_CW - 1) / PL_CW + 1, ty = (mc + PL_CH - 1) / PL_CH + 1;
  hipLaunchKernelGGL((prolong_add_kernel<ST, PL_CH>), dim3(tx * ty * B), dim3(256), 0, st, (const E*)xc, WT,
                     (E*)yf, mc, tx, tx * ty, active);
}

template <int ST>
static void prolong_launch(const void* xc, const float* WT, void* yf, int mc, int B, const int* active,
                           hipStream_t st) {
  const int v = get_tile_variant(TILE_PROLONG, ST == ST_BF16, 2 * mc + 1);
  if (v == 1) prolong_launch_ch<ST, 2>(xc, WT, yf, mc, B, active, st);
  else if (v == 2) prolong_launch_ch<ST, 8>(xc, WT, yf, mc, B, active, st);
  else prolong_launch_ch<ST, 4>(xc, WT, yf, mc, B, active, st);
}

void launch_prolong_add(StateType st_, const void* xc, const float* WT, void* yf, int mc, int B,
                        const int* active, hipStream_t st) {
  if (st_ == ST_F32 || st_ == ST_F32X) prolong_launch<ST_F32>(xc, WT, yf, mc, B, active, st);
  else prolong_launch<ST_BF16>(xc, WT, yf, mc, B, active, st);
}

}  // namespace mg
