// Geometric multigrid baseline on CDNA4 (gfx950): the V-cycle of Sec. 2.3 (Alg. 1 applied
// recursively) with the settings of Sec. 4.1: the PDE rediscretised on every coarse grid
// (coefficient injected to the coarse nodes, h doubled), bilinear prolongation P, full-weighting
// restriction R = P^T / 4, weighted-Jacobi sweeps before and after the coarse correction, and an
// exact solve on the coarsest grid (at most 15 x 15).
//
// Every level is HBM-bound scalar work (no contraction), so each level is two fused kernels
// with temporal blocking in LDS:
//   down: all pre-sweeps from zero, the residual and its full-weighting restriction, per
//         32 x 32 output tile -- a and the right-hand side are read once, e and the coarse
//         right-hand side written once;
//   up:   prolong-add of the coarse correction and all post-sweeps, writing the level's final
//         correction (on the finest level straight into u or z).
// The halo of a tile grows by one node per sweep; the sweeps are recomputed on the overlap
// instead of exchanged.  The stencil of every node (the four neighbour weights of D^-1 A and
// D) is formed once per kernel in registers from a staged in LDS.
//
// Layouts: scalar fields [B][m][m] (x fastest), problem index from the compact list.
#include <algorithm>

#include "mgcnn_internal.h"
#include "mgcnn_device.h"
#include "mgcnn_gmg.h"

namespace mg {

constexpr int GT = 32;          // output tile side (fine nodes); 16 x 16 coarse nodes

// v_rcp_f32 (1 ulp): the preconditioner's stencil needs no correctly rounded division
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float harmf(float p, float q) { return (2.f * p * q) * rcpf(p + q); }

// Stencil of node (i, j) of an m x m grid from the coefficient staged in LDS around it (la at
// the node; +-1 and +-P its neighbours; face coefficients per the operator form).  q = rhs / D
// (or rhs itself when already scaled).
struct Node {
  float D, wW, wE, wS, wN, q;
};
__device__ __forceinline__ Node make_node(const float* la, int c, int P, int i, int j, int m,
                                          float ih, float ih2, float bxp, float bxm, float byp,
                                          float bym, float rhs, bool scaled, int form) {
  Node s;
  const float ac = la[c];
  const float aE = (j + 1 < m && !form) ? harmf(ac, la[c + 1]) : ac;
  const float aW = (j > 0 && !form) ? harmf(ac, la[c - 1]) : ac;
  const float aN = (i + 1 < m && !form) ? harmf(ac, la[c + P]) : ac;
  const float aS = (i > 0 && !form) ? harmf(ac, la[c - P]) : ac;
  s.D = (aE + aW + aN + aS) * ih2 + (bxp - bxm + byp - bym) * ih;
  const float iD = rcpf(s.D);
  s.wW = (j > 0) ? (aW * ih2 + bxp * ih) * iD : 0.f;
  s.wE = (j + 1 < m) ? (aE * ih2 - bxm * ih) * iD : 0.f;
  s.wS = (i > 0) ? (aS * ih2 + byp * ih) * iD : 0.f;
  s.wN = (i + 1 < m) ? (aN * ih2 - bym * ih) * iD : 0.f;
  s.q = scaled ? rhs : rhs * iD;
  return s;
}

// Zero the padding ring of the two e buffers (every region node is written before it is read).
template <int P>
__device__ __forceinline__ void zero_ring(float* e0, float* e1, int tid) {
  for (int t = tid; t < 4 * P; t += 256) {
    const int side = t / P, r = t % P;
    const int idx = side == 0 ? r : side == 1 ? (P - 1) * P + r : side == 2 ? r * P : r * P + P - 1;
    e0[idx] = 0.f;
    e1[idx] = 0.f;
  }
}

// Tile geometry: the e-region of side RS around the tile, padded by one ring (P = RS + 2) that
// holds the coefficient halo in `la` and zeros in the e buffers.
template <int RS>
struct Geo {
  static constexpr int P = RS + 2;
  static constexpr int PTS = (RS * RS + 255) / 256;   // region nodes per thread
};

// ------------------------------------------------------------------------------------------
// down: e = S^NU(0; r) on the tile; rc = R (r - A e) on the 16 x 16 coarse nodes of the tile.
// ------------------------------------------------------------------------------------------
template <int NU>
__global__ __launch_bounds__(256) void gmg_down_kernel(const float* __restrict__ a,
                                                       const float* __restrict__ bvec,
                                                       const float* __restrict__ rhs, int scaled,
                                                       float omega, float* __restrict__ e_out,
                                                       float* __restrict__ rc_out, int m,
                                                       int tiles_x, int tiles_per_prob,
                                                       const int* __restrict__ active, int form) {
  constexpr int RS = GT + 1 + 2 * NU;      // region: tile rows y0 - NU .. y0 + GT + NU
  using G = Geo<RS>;
  constexpr int P = G::P;
  __shared__ float la[P * P];
  __shared__ float le[2][P * P];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;
  const int y0 = (tile / tiles_x) * GT, x0 = (tile % tiles_x) * GT;
  const int oy = y0 - NU, ox = x0 - NU;    // grid coordinates of region node (0, 0)
  const size_t base = (size_t)b * m * m;
  const int tid = threadIdx.x;
  // every global load of the tile is issued before the first barrier: the coefficient with its
  // halo into LDS, the right-hand side of the tile's region nodes into registers
  float rv[G::PTS];
#pragma unroll
  for (int k = 0; k < G::PTS; ++k) {
    const int p = tid + 256 * k;
    const int i = oy + p / RS, j = ox + p % RS;
    rv[k] = (p < RS * RS && i >= 0 && i < m && j >= 0 && j < m) ? rhs[base + (size_t)i * m + j] : 0.f;
  }
  for (int idx = tid; idx < P * P; idx += 256) {
    const int gi = oy - 1 + idx / P, gj = ox - 1 + idx % P;
    const bool in = gi >= 0 && gi < m && gj >= 0 && gj < m;
    la[idx] = in ? a[base + (size_t)gi * m + gj] : 0.f;
  }
  zero_ring<P>(le[0], le[1], tid);
  const float ih = (float)(m + 1), ih2 = ih * ih;
  const float bx = bvec[2 * b], by = bvec[2 * b + 1];
  const float bxp = bx > 0.f ? bx : 0.f, bxm = bx < 0.f ? bx : 0.f;
  const float byp = by > 0.f ? by : 0.f, bym = by < 0.f ? by : 0.f;
  __syncthreads();
  Node nd[G::PTS];
  float ev[G::PTS];
#pragma unroll
  for (int k = 0; k < G::PTS; ++k) {
    const int p = tid + 256 * k;
    const int ry = p / RS, rx = p % RS;
    const int i = oy + ry, j = ox + rx;
    const bool in = p < RS * RS && i >= 0 && i < m && j >= 0 && j < m;
    const int c = (ry + 1) * P + rx + 1;
    if (in) {
      nd[k] = make_node(la, c, P, i, j, m, ih, ih2, bxp, bxm, byp, bym, rv[k], scaled != 0, form);
      ev[k] = omega * nd[k].q;                       // first sweep from zero
    } else {
      nd[k] = Node{1.f, 0.f, 0.f, 0.f, 0.f, 0.f};    // outside the grid: e stays 0
      ev[k] = 0.f;
    }
    if (p < RS * RS) le[0][c] = ev[k];
  }
  __syncthreads();
  const float om1 = 1.f - omega;
#pragma unroll
  for (int s = 1; s < NU; ++s) {
    const float* cur = le[(s - 1) & 1];
    float* nxt = le[s & 1];
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
      const int p = tid + 256 * k;
      if (p < RS * RS) {
        const int c = (p / RS + 1) * P + p % RS + 1;
        const Node& q = nd[k];
        const float v = om1 * ev[k] +
                        omega * (q.q + q.wW * cur[c - 1] + q.wE * cur[c + 1] + q.wS * cur[c - P] +
                                 q.wN * cur[c + P]);
        ev[k] = v;
        nxt[c] = v;
      }
    }
    __syncthreads();
  }
  // residual r - A e = D (q - e + sum w e_nb) on the restriction footprint (region rows and
  // columns NU .. NU + GT), into the free buffer
  {
    const float* cur = le[(NU - 1) & 1];
    float* res = le[NU & 1];
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
      const int p = tid + 256 * k;
      const int ry = p / RS, rx = p % RS;
      if (p < RS * RS && ry >= NU && ry <= NU + GT && rx >= NU && rx <= NU + GT) {
        const int c = (ry + 1) * P + rx + 1;
        const Node& q = nd[k];
        res[c] = q.D * (q.q - ev[k] + q.wW * cur[c - 1] + q.wE * cur[c + 1] + q.wS * cur[c - P] +
                        q.wN * cur[c + P]);
      }
    }
  }
  // final e of the tile's own nodes
#pragma unroll
  for (int k = 0; k < G::PTS; ++k) {
    const int p = tid + 256 * k;
    const int ry = p / RS, rx = p % RS;
    const int i = oy + ry, j = ox + rx;
    if (p < RS * RS && ry >= NU && ry < NU + GT && rx >= NU && rx < NU + GT && i < m && j < m)
      e_out[base + (size_t)i * m + j] = ev[k];
  }
  __syncthreads();
  // full weighting onto the coarse nodes (I, J) = (y0/2 + tid/16, x0/2 + tid%16)
  const int mc = (m - 1) / 2;
  const int I = y0 / 2 + tid / 16, J = x0 / 2 + tid % 16;
  if (I < mc && J < mc) {
    const float* res = le[NU & 1];
    const int c = (2 * I + 1 - oy + 1) * P + (2 * J + 1 - ox + 1);
    const float v = 4.f * res[c] + 2.f * (res[c - 1] + res[c + 1] + res[c - P] + res[c + P]) +
                    (res[c - P - 1] + res[c - P + 1] + res[c + P - 1] + res[c + P + 1]);
    rc_out[(size_t)b * mc * mc + (size_t)I * mc + J] = v * 0.0625f;
  }
}

// ------------------------------------------------------------------------------------------
// up: e = S^NU(e_pre + P ec; r) on the tile, written per `mode` (f32 / f64, store / add).
// ------------------------------------------------------------------------------------------
template <int NU>
__global__ __launch_bounds__(256) void gmg_up_kernel(const float* __restrict__ a,
                                                     const float* __restrict__ bvec,
                                                     const float* __restrict__ rhs, int scaled,
                                                     float omega, const float* __restrict__ e_pre,
                                                     const float* __restrict__ ec, void* out,
                                                     int mode, const int* __restrict__ flags,
                                                     int m, int tiles_x, int tiles_per_prob,
                                                     const int* __restrict__ active, int form) {
  constexpr int RS = GT + 2 * NU;          // region: tile rows y0 - NU .. y0 + GT + NU - 1
  using G = Geo<RS>;
  constexpr int P = G::P;
  constexpr int CS = GT / 2 + NU + 3;      // side of the staged coarse patch
  __shared__ float la[P * P];
  __shared__ float le[2][P * P];
  __shared__ float lc[CS * CS];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;
  const int y0 = (tile / tiles_x) * GT, x0 = (tile % tiles_x) * GT;
  const int oy = y0 - NU, ox = x0 - NU;
  const size_t base = (size_t)b * m * m;
  const int mc = (m - 1) / 2;
  const size_t cbase = (size_t)b * mc * mc;
  const int cy = (oy - 1) >> 1, cx = (ox - 1) >> 1;    // coarse patch origin (may be -1)
  const int tid = threadIdx.x;
  // global loads first: right-hand side and pre-smoothed e of the region nodes into registers,
  // the coefficient with its halo and the coarse patch into LDS
  float rv[G::PTS], pv[G::PTS];
#pragma unroll
  for (int k = 0; k < G::PTS; ++k) {
    const int p = tid + 256 * k;
    const int i = oy + p / RS, j = ox + p % RS;
    const bool in = p < RS * RS && i >= 0 && i < m && j >= 0 && j < m;
    const size_t g = base + (size_t)(in ? i : 0) * m + (in ? j : 0);
    rv[k] = in ? rhs[g] : 0.f;
    pv[k] = in ? e_pre[g] : 0.f;
  }
  for (int idx = tid; idx < P * P; idx += 256) {
    const int gi = oy - 1 + idx / P, gj = ox - 1 + idx % P;
    const bool in = gi >= 0 && gi < m && gj >= 0 && gj < m;
    la[idx] = in ? a[base + (size_t)gi * m + gj] : 0.f;
  }
  for (int idx = tid; idx < CS * CS; idx += 256) {
    const int I = cy + idx / CS, J = cx + idx % CS;
    lc[idx] = (I >= 0 && I < mc && J >= 0 && J < mc) ? ec[cbase + (size_t)I * mc + J] : 0.f;
  }
  zero_ring<P>(le[0], le[1], tid);
  const float ih = (float)(m + 1), ih2 = ih * ih;
  const float bx = bvec[2 * b], by = bvec[2 * b + 1];
  const float bxp = bx > 0.f ? bx : 0.f, bxm = bx < 0.f ? bx : 0.f;
  const float byp = by > 0.f ? by : 0.f, bym = by < 0.f ? by : 0.f;
  __syncthreads();
  Node nd[G::PTS];
  float ev[G::PTS];
#pragma unroll
  for (int k = 0; k < G::PTS; ++k) {
    const int p = tid + 256 * k;
    const int ry = p / RS, rx = p % RS;
    const int i = oy + ry, j = ox + rx;
    const bool in = p < RS * RS && i >= 0 && i < m && j >= 0 && j < m;
    const int c = (ry + 1) * P + rx + 1;
    if (in) {
      nd[k] = make_node(la, c, P, i, j, m, ih, ih2, bxp, bxm, byp, bym, rv[k], scaled != 0, form);
      // bilinear interpolation: fine i lies between coarse rows (i-1)>>1 and i>>1 (the same
      // row when i is odd); the four-term average gives weights 1, 1/2 and 1/4
      const int i0 = ((i - 1) >> 1) - cy, i1 = (i >> 1) - cy;
      const int j0 = ((j - 1) >> 1) - cx, j1 = (j >> 1) - cx;
      const float pe = 0.25f * ((lc[i0 * CS + j0] + lc[i0 * CS + j1]) +
                                (lc[i1 * CS + j0] + lc[i1 * CS + j1]));
      ev[k] = pv[k] + pe;
    } else {
      nd[k] = Node{1.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      ev[k] = 0.f;
    }
    if (p < RS * RS) le[0][c] = ev[k];
  }
  __syncthreads();
  const float om1 = 1.f - omega;
#pragma unroll
  for (int s = 0; s < NU; ++s) {
    const float* cur = le[s & 1];
    float* nxt = le[(s + 1) & 1];
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
      const int p = tid + 256 * k;
      if (p < RS * RS) {
        const int c = (p / RS + 1) * P + p % RS + 1;
        const Node& q = nd[k];
        const float v = om1 * ev[k] +
                        omega * (q.q + q.wW * cur[c - 1] + q.wE * cur[c + 1] + q.wS * cur[c - P] +
                                 q.wN * cur[c + P]);
        ev[k] = v;
        if (s + 1 < NU) nxt[c] = v;
      }
    }
    if (s + 1 < NU) __syncthreads();
  }
  if (flags != nullptr && flags[b] == 0) return;
#pragma unroll
  for (int k = 0; k < G::PTS; ++k) {
    const int p = tid + 256 * k;
    const int ry = p / RS, rx = p % RS;
    const int i = oy + ry, j = ox + rx;
    if (p < RS * RS && ry >= NU && ry < NU + GT && rx >= NU && rx < NU + GT && i < m && j < m) {
      const size_t g = base + (size_t)i * m + j;
      switch (mode) {
        case GMG_OUT_F32: static_cast<float*>(out)[g] = ev[k]; break;
        case GMG_OUT_F32_ADD: static_cast<float*>(out)[g] += ev[k]; break;
        case GMG_OUT_F64: static_cast<double*>(out)[g] = (double)ev[k]; break;
        default: static_cast<double*>(out)[g] += (double)ev[k]; break;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// coarsest grid: exact solve with the inverse formed at setup (f64).
// ------------------------------------------------------------------------------------------
// Inverse of the rediscretised operator on an mc x mc grid (row index i*mc + j), one
// workgroup per problem.  A is an M-matrix with bandwidth mc (couplings at +-1 and +-mc), so an
// LU factorisation without pivoting is stable and stays inside the band: the band (at most
// 225 rows x 31 diagonals, f64) is assembled and factorised in LDS, then thread t solves
// A x = e_t (forward then backward substitution, the last 16 values in a register window) and
// writes x, column t of A^-1, as row t of inv.  So inv = (A^-1)^T, what the apply kernel wants:
// for each k, the threads read consecutive entries.
constexpr int GMG_BAND = GMG_MAX_COARSE_SIDE;            // largest bandwidth
constexpr int GMG_BW = 2 * GMG_BAND + 1;                 // stored diagonals per row
constexpr int GMG_WIN = 16;                              // register window >= GMG_BAND

__global__ __launch_bounds__(256) void gmg_coarse_inverse_kernel(const float* __restrict__ a,
                                                                 const float* __restrict__ bvec,
                                                                 double* __restrict__ inv, int mc,
                                                                 int form) {
  const int b = blockIdx.x;
  const int N = mc * mc;
  const int tid = threadIdx.x;
  const float* A = a + (size_t)b * N;
  __shared__ double band[GMG_MAX_COARSE * GMG_BW];       // band[p][q - p + GMG_BAND] = A[p][q]
  auto at = [&](int p, int q) -> double& { return band[p * GMG_BW + (q - p + GMG_BAND)]; };
  for (int idx = tid; idx < GMG_MAX_COARSE * GMG_BW; idx += 256) band[idx] = 0.0;
  __syncthreads();
  const double ih = (double)(mc + 1), ih2 = ih * ih;
  const double bx = bvec[2 * b], by = bvec[2 * b + 1];
  const double bxp = bx > 0 ? bx : 0, bxm = bx < 0 ? bx : 0;
  const double byp = by > 0 ? by : 0, bym = by < 0 ? by : 0;
  auto hm = [](double p, double q) { return 2.0 * p * q / (p + q); };
  for (int p = tid; p < N; p += 256) {
    const int i = p / mc, j = p % mc;
    const double ac = A[p];
    const double aE = (j + 1 < mc && !form) ? hm(ac, A[p + 1]) : ac;
    const double aW = (j > 0 && !form) ? hm(ac, A[p - 1]) : ac;
    const double aN = (i + 1 < mc && !form) ? hm(ac, A[p + mc]) : ac;
    const double aS = (i > 0 && !form) ? hm(ac, A[p - mc]) : ac;
    at(p, p) = (aE + aW + aN + aS) * ih2 + (bxp - bxm + byp - bym) * ih;
    if (j + 1 < mc) at(p, p + 1) = -aE * ih2 + bxm * ih;
    if (j > 0) at(p, p - 1) = -aW * ih2 - bxp * ih;
    if (i + 1 < mc) at(p, p + mc) = -aN * ih2 + bym * ih;
    if (i > 0) at(p, p - mc) = -aS * ih2 - byp * ih;
  }
  __syncthreads();
  // Doolittle LU in the band: step k updates rows and columns k+1 .. k+mc (one entry per thread),
  // then stores the multipliers of column k
  const int W = mc;
  for (int k = 0; k < N; ++k) {
    if (tid < W * W) {
      const int i = k + 1 + tid / W, j = k + 1 + tid % W;
      if (i < N && j < N) at(i, j) -= at(i, k) / at(k, k) * at(k, j);
    }
    __syncthreads();
    if (tid < W && k + 1 + tid < N) at(k + 1 + tid, k) /= at(k, k);
    __syncthreads();
  }
  if (tid >= N) return;
  double* X = inv + (size_t)b * N * N + (size_t)tid * N;
  // forward: y = L^-1 e_t (unit lower); win[GMG_WIN - d] = y_{i-d}
  double win[GMG_WIN];
#pragma unroll
  for (int d = 0; d < GMG_WIN; ++d) win[d] = 0.0;
  for (int i = 0; i < N; ++i) {
    double y = (i == tid) ? 1.0 : 0.0;
#pragma unroll
    for (int d = 1; d <= GMG_BAND; ++d)
      if (i - d >= 0) y -= band[i * GMG_BW + (GMG_BAND - d)] * win[GMG_WIN - d];
#pragma unroll
    for (int d = 0; d < GMG_WIN - 1; ++d) win[d] = win[d + 1];
    win[GMG_WIN - 1] = y;
    X[i] = y;
  }
  // backward: x = U^-1 y; win[GMG_WIN - d] = x_{i+d}
#pragma unroll
  for (int d = 0; d < GMG_WIN; ++d) win[d] = 0.0;
  for (int i = N - 1; i >= 0; --i) {
    double x = X[i];
#pragma unroll
    for (int d = 1; d <= GMG_BAND; ++d)
      if (i + d < N) x -= band[i * GMG_BW + (GMG_BAND + d)] * win[GMG_WIN - d];
    x /= band[i * GMG_BW + GMG_BAND];
#pragma unroll
    for (int d = 0; d < GMG_WIN - 1; ++d) win[d] = win[d + 1];
    win[GMG_WIN - 1] = x;
    X[i] = x;
  }
}

// e = A^-1 r on the coarsest grid, one workgroup per problem.  `scaled`: r is given as r / D
// (only when the coarsest grid is the finest one).
__global__ __launch_bounds__(256) void gmg_coarse_solve_kernel(const double* __restrict__ inv,
                                                               const float* __restrict__ a,
                                                               const float* __restrict__ bvec,
                                                               const float* __restrict__ rhs,
                                                               int scaled, void* out, int mode,
                                                               const int* __restrict__ flags,
                                                               int mc, const int* __restrict__ active,
                                                               int form) {
  const int b = active != nullptr ? active[blockIdx.x] : blockIdx.x;
  const int N = mc * mc;
  const int tid = threadIdx.x;
  __shared__ double lr[GMG_MAX_COARSE];
  const size_t base = (size_t)b * N;
  if (tid < N) {
    double r = rhs[base + tid];
    if (scaled) {
      const float* A = a + base;
      const int i = tid / mc, j = tid % mc;
      const double ih = (double)(mc + 1), ih2 = ih * ih;
      const double ac = A[tid];
      auto hm = [](double p, double q) { return 2.0 * p * q / (p + q); };
      const double aE = (j + 1 < mc && !form) ? hm(ac, A[tid + 1]) : ac;
      const double aW = (j > 0 && !form) ? hm(ac, A[tid - 1]) : ac;
      const double aN = (i + 1 < mc && !form) ? hm(ac, A[tid + mc]) : ac;
      const double aS = (i > 0 && !form) ? hm(ac, A[tid - mc]) : ac;
      const double bx = bvec[2 * b], by = bvec[2 * b + 1];
      r *= (aE + aW + aN + aS) * ih2 + (fabs(bx) + fabs(by)) * ih;
    }
    lr[tid] = r;
  }
  __syncthreads();
  if (tid >= N) return;
  const double* M = inv + (size_t)b * N * N;
  double acc = 0.0;
  for (int k = 0; k < N; ++k) acc += M[(size_t)k * N + tid] * lr[k];
  if (flags != nullptr && flags[b] == 0) return;
  switch (mode) {
    case GMG_OUT_F32: static_cast<float*>(out)[base + tid] = (float)acc; break;
    case GMG_OUT_F32_ADD: static_cast<float*>(out)[base + tid] += (float)acc; break;
    case GMG_OUT_F64: static_cast<double*>(out)[base + tid] = acc; break;
    default: static_cast<double*>(out)[base + tid] += acc; break;
  }
}

// coefficient on the next coarser grid: a_c[I][J] = a[2I+1][2J+1]
__global__ __launch_bounds__(256) void gmg_inject_kernel(const float* __restrict__ a,
                                                         float* __restrict__ ac, int m, int B) {
  const int mc = (m - 1) / 2;
  const size_t total = (size_t)B * mc * mc;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * 256) {
    const size_t b = idx / ((size_t)mc * mc);
    const int r = (int)(idx % ((size_t)mc * mc));
    const int I = r / mc, J = r % mc;
    ac[idx] = a[b * m * m + (size_t)(2 * I + 1) * m + 2 * J + 1];
  }
}

// ---- launchers ---------------------------------------------------------------------------
static inline int tiles_1d(int m) { return (m + GT - 1) / GT; }

void launch_gmg_down(int nu, const float* a, const float* b, const float* rhs, bool scaled,
                     float omega, float* e, float* rc, int m, int B, const int* active, int form,
                     hipStream_t st) {
  const int tx = tiles_1d(m), tp = tx * tx;
  const dim3 grid(tp * B), block(256);
  switch (nu) {
    case 1: hipLaunchKernelGGL(gmg_down_kernel<1>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e, rc, m, tx, tp, active, form); break;
    case 2: hipLaunchKernelGGL(gmg_down_kernel<2>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e, rc, m, tx, tp, active, form); break;
    case 3: hipLaunchKernelGGL(gmg_down_kernel<3>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e, rc, m, tx, tp, active, form); break;
    default: hipLaunchKernelGGL(gmg_down_kernel<4>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e, rc, m, tx, tp, active, form); break;
  }
}

void launch_gmg_up(int nu, const float* a, const float* b, const float* rhs, bool scaled,
                   float omega, const float* e_pre, const float* ec, void* out, int mode,
                   const int* flags, int m, int B, const int* active, int form, hipStream_t st) {
  const int tx = tiles_1d(m), tp = tx * tx;
  const dim3 grid(tp * B), block(256);
  switch (nu) {
    case 1: hipLaunchKernelGGL(gmg_up_kernel<1>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e_pre, ec, out, mode, flags, m, tx, tp, active, form); break;
    case 2: hipLaunchKernelGGL(gmg_up_kernel<2>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e_pre, ec, out, mode, flags, m, tx, tp, active, form); break;
    case 3: hipLaunchKernelGGL(gmg_up_kernel<3>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e_pre, ec, out, mode, flags, m, tx, tp, active, form); break;
    default: hipLaunchKernelGGL(gmg_up_kernel<4>, grid, block, 0, st, a, b, rhs, (int)scaled, omega, e_pre, ec, out, mode, flags, m, tx, tp, active, form); break;
  }
}

void launch_gmg_coarse_inverse(const float* a, const float* b, double* inv, int mc, int B,
                               int form, hipStream_t st) {
  hipLaunchKernelGGL(gmg_coarse_inverse_kernel, dim3(B), dim3(256), 0, st, a, b, inv, mc, form);
}

void launch_gmg_coarse_solve(const double* inv, const float* a, const float* b, const float* rhs,
                             bool scaled, void* out, int mode, const int* flags, int mc, int B,
                             const int* active, int form, hipStream_t st) {
  hipLaunchKernelGGL(gmg_coarse_solve_kernel, dim3(B), dim3(256), 0, st, inv, a, b, rhs,
                     (int)scaled, out, mode, flags, mc, active, form);
}

void launch_gmg_inject(const float* a, float* ac, int m, int B, hipStream_t st) {
  const int mc = (m - 1) / 2;
  const size_t total = (size_t)B * mc * mc;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(gmg_inject_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, a, ac, m, B);
}

}  // namespace mg
