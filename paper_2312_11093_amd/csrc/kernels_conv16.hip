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

// Load 4 consecutive channels (chunk g) of pixel `pix` of a channel-last tensor as floats.
__device__ __forceinline__ float4 ld4(const float* X, size_t pix, int g) {
  return reinterpret_cast<const float4*>(X)[pix * 4 + g];
}
__device__ __forceinline__ float4 ld4(const uint16_t* X, size_t pix, int g) {
  const uint2 z = reinterpret_cast<const uint2*>(X)[pix * 4 + g];
  return make_float4(__uint_as_float(z.x << 16), __uint_as_float(z.x & 0xffff0000u),
                     __uint_as_float(z.y << 16), __uint_as_float(z.y & 0xffff0000u));
}
__device__ __forceinline__ void st4_lds(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
__device__ __forceinline__ void st4_lds(uint16_t* p, float4 v) {
  *reinterpret_cast<uint2*>(p) =
      make_uint2((uint32_t)f32_to_bf16_rne(v.x) | ((uint32_t)f32_to_bf16_rne(v.y) << 16),
                 (uint32_t)f32_to_bf16_rne(v.z) | ((uint32_t)f32_to_bf16_rne(v.w) << 16));
}
__device__ __forceinline__ void st4(float* X, size_t pix, int g, float4 v) {
  reinterpret_cast<float4*>(X)[pix * 4 + g] = v;
}
__device__ __forceinline__ void st4(uint16_t* X, size_t pix, int g, float4 v) {
  reinterpret_cast<uint2*>(X)[pix * 4 + g] =
      make_uint2((uint32_t)f32_to_bf16_rne(v.x) | ((uint32_t)f32_to_bf16_rne(v.y) << 16),
                 (uint32_t)f32_to_bf16_rne(v.z) | ((uint32_t)f32_to_bf16_rne(v.w) << 16));
}

// ------------------------------------------------------------------------------------------
// same-size conv: smoother (s given) or tanh ResNet layer (bias given)
// ------------------------------------------------------------------------------------------
constexpr int SAME_TH = 8, SAME_TW = 64;
constexpr int SAME_IR = SAME_TH + 2, SAME_IC = SAME_TW + 2;

template <int ST, int MODE>
__global__ __launch_bounds__(256) void conv16_same_kernel(
    const typename Frag<ST>::elem* __restrict__ x, const typename Frag<ST>::elem* __restrict__ s,
    const float* __restrict__ W, const float* __restrict__ bias,
    typename Frag<ST>::elem* __restrict__ y, int m, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  __shared__ __attribute__((aligned(16))) E lds[SAME_IR * SAME_IC * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int row0 = (tile / tiles_x) * SAME_TH, col0 = (tile % tiles_x) * SAME_TW;
  const size_t pbase = (size_t)b * m * m;
  const E* X = x;
  // stage z = s . x (smoother) or x (tanh layer) with a one-pixel halo, zero outside
  for (int k = threadIdx.x; k < SAME_IR * SAME_IC * 4; k += 256) {
    const int pix = k >> 2, g = k & 3;
    const int lr = pix / SAME_IC, lc = pix - lr * SAME_IC;
    const int gi = row0 + lr - 1, gj = col0 + lc - 1;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gi >= 0 && gi < m && gj >= 0 && gj < m) {
      const size_t gp = pbase + (size_t)gi * m + gj;
      v = ld4(X, gp, g);
      if constexpr (MODE == CM_SMOOTH) {
        const float4 sv = ld4(s, gp, g);
        v.x *= sv.x; v.y *= sv.y; v.z *= sv.z; v.w *= sv.w;
      }
    }
    st4_lds(&lds[pix * PS + 4 * g], v);
  }
  Frag<ST> fr;
  fr.load_w(W, false);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
#pragma unroll 1
  for (int task = 0; task < 8; ++task) {
    const int orow = wave * 2 + (task >> 2), seg = task & 3;
    const int gi = row0 + orow;
    if (gi >= m) continue;
    if (col0 + seg * 16 >= m) continue;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((orow + p) * SAME_IC + seg * 16 + px + q) * PS], acc);
    const int gj = col0 + seg * 16 + px;
    if (gj < m) {
      const size_t gp = pbase + (size_t)gi * m + gj;
      const float4 xc = ld4(X, gp, g);
      float4 o;
      if constexpr (MODE == CM_TANH) {
        o.x = xc.x + tanhf(acc[0] + bias[4 * g + 0]);
        o.y = xc.y + tanhf(acc[1] + bias[4 * g + 1]);
        o.z = xc.z + tanhf(acc[2] + bias[4 * g + 2]);
        o.w = xc.w + tanhf(acc[3] + bias[4 * g + 3]);
      } else {
        o.x = xc.x + acc[0]; o.y = xc.y + acc[1]; o.z = xc.z + acc[2]; o.w = xc.w + acc[3];
      }
      st4(y, gp, g, o);
    }
  }
}

// ------------------------------------------------------------------------------------------
// stride-2 restriction conv, no padding: m -> mo = (m-1)/2
// Columns of the staged fine tile are de-interleaved by parity so that the stride-2
// operand reads stay consecutive in LDS.
// ------------------------------------------------------------------------------------------
constexpr int RS_TH = 4, RS_TW = 32;
constexpr int RS_IR = 2 * RS_TH + 1, RS_IC = 2 * RS_TW + 1, RS_HALF = RS_TW + 1;
constexpr int RS_ROW = 2 * RS_HALF;   // slots per staged row

__device__ __forceinline__ int rs_slot(int lc) { return (lc & 1) ? RS_HALF + (lc >> 1) : (lc >> 1); }

template <int ST>
__global__ __launch_bounds__(256) void conv16_restrict_kernel(
    const typename Frag<ST>::elem* __restrict__ x, const float* __restrict__ W,
    typename Frag<ST>::elem* __restrict__ y, int m, int mo, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  __shared__ __attribute__((aligned(16))) E lds[RS_IR * RS_ROW * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int orow0 = (tile / tiles_x) * RS_TH, ocol0 = (tile % tiles_x) * RS_TW;
  const int frow0 = 2 * orow0, fcol0 = 2 * ocol0;
  const size_t pin = (size_t)b * m * m;
  for (int k = threadIdx.x; k < RS_IR * RS_IC * 4; k += 256) {
    const int pix = k >> 2, g = k & 3;
    const int lr = pix / RS_IC, lc = pix - lr * RS_IC;
    const int gi = frow0 + lr, gj = fcol0 + lc;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gi < m && gj < m) v = ld4(x, pin + (size_t)gi * m + gj, g);
    st4_lds(&lds[(lr * RS_ROW + rs_slot(lc)) * PS + 4 * g], v);
  }
  Frag<ST> fr;
  fr.load_w(W, false);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  const size_t pout = (size_t)b * mo * mo;
#pragma unroll 1
  for (int seg = 0; seg < RS_TW / 16; ++seg) {
    const int orow = wave;
    const int gi = orow0 + orow;
    if (gi >= mo || ocol0 + seg * 16 >= mo) continue;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    const int jj = seg * 16 + px;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc = fr.mma(p * 3 + q, &lds[((2 * orow + p) * RS_ROW + rs_slot(2 * jj + q)) * PS], acc);
    const int gj = ocol0 + jj;
    if (gj < mo) st4(y, pout + (size_t)gi * mo + gj, g, make_float4(acc[0], acc[1], acc[2], acc[3]));
  }
}

// ------------------------------------------------------------------------------------------
// prolongation: y_fine += convT_{stride 2}(W_T, x_coarse), fine side m = 2 mc + 1.
// Fine pixel (i, j) receives coarse (I, J) through tap (p, q) with 2I + p = i, 2J + q = j:
// odd i uses p = 1 only, even i uses p = 0 (I = i/2) and p = 2 (I = i/2 - 1); same for j.
// Work is split into row segments of 16 fine pixels of equal column parity, so every lane
// of one MFMA uses the same tap.
// ------------------------------------------------------------------------------------------
constexpr int PL_CH = 4, PL_CW = 32;                  // coarse tile
constexpr int PL_IR = PL_CH + 1, PL_IC = PL_CW + 1;   // staged coarse rows/cols (one halo)

template <int ST>
__global__ __launch_bounds__(256) void prolong_add_kernel(
    const typename Frag<ST>::elem* __restrict__ xc, const float* __restrict__ WT,
    typename Frag<ST>::elem* __restrict__ yf, int mc, int tiles_x, int tiles_per_prob,
    const int* __restrict__ active) {
  typedef typename Frag<ST>::elem E;
  __shared__ __attribute__((aligned(16))) E lds[PL_IR * PL_IC * PS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  if (active != nullptr && active[b] == 0) return;
  const int m = 2 * mc + 1;
  const int I0 = (tile / tiles_x) * PL_CH, J0 = (tile % tiles_x) * PL_CW;
  const size_t pc = (size_t)b * mc * mc;
  for (int k = threadIdx.x; k < PL_IR * PL_IC * 4; k += 256) {
    const int pix = k >> 2, g = k & 3;
    const int lr = pix / PL_IC, lc = pix - lr * PL_IC;
    const int I = I0 - 1 + lr, J = J0 - 1 + lc;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (I >= 0 && I < mc && J >= 0 && J < mc) v = ld4(xc, pc + (size_t)I * mc + J, g);
    st4_lds(&lds[pix * PS + 4 * g], v);
  }
  Frag<ST> fr;
  fr.load_w(WT, true);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  const size_t pf = (size_t)b * m * m;
#pragma unroll 1
  for (int task = 0; task < 8; ++task) {
    const int fr_local = wave * 2 + (task >> 2);   // fine row within the 8-row tile
    const int par = (task >> 1) & 1;                // fine column parity
    const int jb = task & 1;                        // 16-wide block of coarse columns
    const int i = 2 * I0 + fr_local;
    if (i >= m) continue;
    const int jc = jb * 16 + px;                    // coarse column within the tile
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    // row taps
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
      const size_t gp = pf + (size_t)i * m + j;
      float4 o = ld4(yf, gp, g);
      o.x += acc[0]; o.y += acc[1]; o.z += acc[2]; o.w += acc[3];
      st4(yf, gp, g, o);
    }
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
void launch_conv16(ConvMode mode, StateType st_, const void* x, const void* s, const float* W,
                   const float* bias, void* y, int m, int B, const int* active, hipStream_t st) {
  if (mode == CM_RESTRICT) {
    const int mo = (m - 1) / 2;
    const int tx = (mo + RS_TW - 1) / RS_TW, ty = (mo + RS_TH - 1) / RS_TH;
    const dim3 grid(tx * ty * B), blk(256);
    if (st_ == ST_F32)
      hipLaunchKernelGGL(conv16_restrict_kernel<ST_F32>, grid, blk, 0, st, (const float*)x, W,
                         (float*)y, m, mo, tx, tx * ty, active);
    else
      hipLaunchKernelGGL(conv16_restrict_kernel<ST_BF16>, grid, blk, 0, st, (const uint16_t*)x, W,
                         (uint16_t*)y, m, mo, tx, tx * ty, active);
    return;
  }
  const int tx = (m + SAME_TW - 1) / SAME_TW, ty = (m + SAME_TH - 1) / SAME_TH;
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
