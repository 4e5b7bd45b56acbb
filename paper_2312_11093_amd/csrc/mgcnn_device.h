// Device-side helpers shared by the MGCNN kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mg {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w runs on XCD w % 8).
// Remap so that every XCD receives one contiguous range of logical tiles: neighbouring
// tiles, which share halo rows, then hit the same L2.
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
  const int q = nwg >> 3, r = nwg & 7;
  const int xcd = wg & 7, local = wg >> 3;
  return (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Sum over a 256-thread workgroup (4 waves); deterministic order; valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// tanh of the setup network's layers (Eq. (6)).  |x| <= 1/4: the Taylor series
//   x - x^3/3 + 2x^5/15 - 17x^7/315 + 62x^9/2835 - 1382x^11/155925 + 21844x^13/6081075,
// whose first omitted term is below 1e-10 |x| there; |x| > 1/4: 1 - 2 / (exp(2|x|) + 1) with the
// sign of x, where tanh >= 0.24 keeps the cancellation below a factor 4, so the error stays
// within a few float32 ulps of the exponential's (about 1e-6 relative at worst).
__device__ __forceinline__ float mg_tanh(float x) {
  const float ax = fabsf(x);
  if (ax <= 0.25f) {
    const float x2 = x * x;
    float p = 21844.f / 6081075.f;
    p = fmaf(p, x2, -1382.f / 155925.f);
    p = fmaf(p, x2, 62.f / 2835.f);
    p = fmaf(p, x2, -17.f / 315.f);
    p = fmaf(p, x2, 2.f / 15.f);
    p = fmaf(p, x2, -1.f / 3.f);
    return fmaf(x * x2, p, x);
  }
  const float e = __expf(2.f * ax);
  return copysignf(1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f), x);
}

// bf16 conversion: the hardware packed convert (round to nearest even) of gfx950.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// 16 contiguous channels of one pixel.
__device__ __forceinline__ void load16(const float* p, float* v) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float4 z = q[k];
    v[4 * k] = z.x; v[4 * k + 1] = z.y; v[4 * k + 2] = z.z; v[4 * k + 3] = z.w;
  }
}
__device__ __forceinline__ void load16(const uint16_t* p, float* v) {
  const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    uint4 z = q[k];
    const uint32_t w[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[8 * k + 2 * e] = __uint_as_float(w[e] << 16);
      v[8 * k + 2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
    }
  }
}
__device__ __forceinline__ void store16(float* p, const float* v) {
  float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}
__device__ __forceinline__ void store16(uint16_t* p, const float* v) {
  uint4* q = reinterpret_cast<uint4*>(p);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = pack_bf16x2(v[8 * k + 2 * e], v[8 * k + 2 * e + 1]);
    q[k] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

}  // namespace mg
