// Point-wise and 5-point stencil kernels of the MGCNN solver on CDNA4 (gfx950):
// setup features, residual + norm partials, stopping test, reChannel convolutions
// (1 -> 16, 4 -> 16, 16 -> 1) and small utilities.
//
// Layouts: scalar fields [B][n][n] (x fastest); channel-last tensors [B][n][n][C].
#include "mgcnn_internal.h"
#include "mgcnn_device.h"

namespace mg {

// ------------------------------------------------------------------------------------------
// Operator helpers (harmonic face coefficients in the divergence form, the row's own node
// value in the non-divergence form; first-order upwind convection).
// The discrete operator follows Sec. 2.5: 5-point diffusion (Eq. (8)) written for the
// divergence form of Eq. (12), upwind convection split by the sign of the velocity
// (Eqs. (9)-(11)); zero Dirichlet values outside the grid; a boundary face uses the
// interior node's coefficient.
// ------------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R harm(R p, R q) { return (R(2) * p * q) / (p + q); }

// ------------------------------------------------------------------------------------------
// features: F = [-A_W, -A_E, -A_S, -A_N] / D, zero where the neighbour is outside.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void features_kernel(const float* __restrict__ a,
                                                       const float* __restrict__ bvec,
                                                       float* __restrict__ F, int n, int tiles_x,
                                                       int tiles_per_prob, int form) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int j = (tile % tiles_x) * 64 + (threadIdx.x & 63);
  const int i = (tile / tiles_x) * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const float* A = a + (size_t)b * n * n;
  const double ac = A[(size_t)i * n + j];
  const double aE = (j + 1 < n) ? (form ? ac : harm<double>(ac, A[(size_t)i * n + j + 1])) : ac;
  const double aW = (j > 0) ? (form ? ac : harm<double>(ac, A[(size_t)i * n + j - 1])) : ac;
  const double aN = (i + 1 < n) ? (form ? ac : harm<double>(ac, A[(size_t)(i + 1) * n + j])) : ac;
  const double aS = (i > 0) ? (form ? ac : harm<double>(ac, A[(size_t)(i - 1) * n + j])) : ac;
  const double ih = (double)(n + 1), ih2 = ih * ih;
  const double bx = bvec[2 * b], by = bvec[2 * b + 1];
  const double bxp = bx > 0 ? bx : 0, bxm = bx < 0 ? bx : 0;
  const double byp = by > 0 ? by : 0, bym = by < 0 ? by : 0;
  const double D = (aE + aW + aN + aS) * ih2 + (fabs(bx) + fabs(by)) * ih;
  float4 o;
  o.x = (j > 0) ? (float)((aW * ih2 + bxp * ih) / D) : 0.f;
  o.y = (j + 1 < n) ? (float)((aE * ih2 - bxm * ih) / D) : 0.f;
  o.z = (i > 0) ? (float)((aS * ih2 + byp * ih) / D) : 0.f;
  o.w = (i + 1 < n) ? (float)((aN * ih2 - bym * ih) / D) : 0.f;
  reinterpret_cast<float4*>(F)[((size_t)b * n + i) * n + j] = o;
}

void launch_features(const float* a, const float* b, float* F, int n, int B, int form, hipStream_t st) {
  const int tx = (n + 63) / 64, ty = (n + 3) / 4;
  hipLaunchKernelGGL(features_kernel, dim3(tx * ty * B), dim3(256), 0, st, a, b, F, n, tx, tx * ty,
                     form);
}

// ------------------------------------------------------------------------------------------
// residual: r = f - A u ; rt = r / D ; per-workgroup partial sum of r^2 in f64.
// ------------------------------------------------------------------------------------------
// Tiles of 256 columns x RES_ROWS rows; each thread walks one column of its tile, keeping the
// row above, the current row and the row below in registers, so every vertical face
// coefficient is formed once and every value of a and u comes from HBM once.
constexpr int RES_ROWS = 8;
int residual_tiles(int n) { return ((n + 255) / 256) * ((n + RES_ROWS - 1) / RES_ROWS); }

// 1/x to full double precision: hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double rcp_full(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float rcp_full(float x) { return 1.0f / x; }
template <typename R>
__device__ __forceinline__ R harm_fast(R p, R q) { return (R(2) * p * q) * rcp_full(p + q); }

template <typename R, typename UT, bool HAS_U>
__global__ __launch_bounds__(256) void residual_kernel(const float* __restrict__ a,
                                                       const float* __restrict__ bvec,
                                                       const float* __restrict__ f,
                                                       const UT* __restrict__ u,
                                                       float* __restrict__ rt,
                                                       double* __restrict__ partial, int n,
                                                       int tiles_x, int tiles_per_prob,
                                                       const int* __restrict__ active, int form) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  const int j = (tile % tiles_x) * 256 + threadIdx.x;
  const int i0 = (tile / tiles_x) * RES_ROWS;
  const size_t base = (size_t)b * n * n;
  const float* A = a + base;
  const float* F = f + base;
  double r2 = 0.0;
  if (j < n) {
    if constexpr (HAS_U) {
      const UT* U = u + base;
      const R ih = (R)(n + 1), ih2 = ih * ih;
      const R bx = (R)bvec[2 * b], by = (R)bvec[2 * b + 1];
      const R bxp = bx > R(0) ? bx : R(0), bxm = bx < R(0) ? bx : R(0);
      const R byp = by > R(0) ? by : R(0), bym = by < R(0) ? by : R(0);
      const R conv_diag = (bxp - bxm + byp - bym) * ih;
      const bool hasE = j + 1 < n, hasW = j > 0;
      // rows i0 - 1 (south) and i0 (centre)
      R ac = (R)A[i0 * n + j];
      R uc = (R)U[i0 * n + j];
      R us = (i0 > 0) ? (R)U[(i0 - 1) * n + j] : R(0);
      R aS = (i0 > 0 && !form) ? harm_fast<R>(ac, (R)A[(i0 - 1) * n + j]) : ac;
      const int dE = hasE ? 1 : 0, dW = hasW ? 1 : 0;       // clamped offsets: branch-free loads
#pragma unroll 2
      for (int r = 0; r < RES_ROWS; ++r) {
        const int i = i0 + r;
        if (i >= n) break;
        const int ij = i * n + j;
        const bool hasN = i + 1 < n;
        const int dN = hasN ? n : 0;
        const R an_raw = (R)A[ij + dN], un_raw = (R)U[ij + dN];
        const R ae_raw = (R)A[ij + dE], aw_raw = (R)A[ij - dW];
        const R ue_raw = (R)U[ij + dE], uw_raw = (R)U[ij - dW];
        const R fv = (R)F[ij];
        const R an = an_raw;
        const R un = hasN ? un_raw : R(0);
        const R aN = (hasN && !form) ? harm_fast<R>(ac, an) : ac;
        const R aE = (hasE && !form) ? harm_fast<R>(ac, ae_raw) : ac;
        const R aW = (hasW && !form) ? harm_fast<R>(ac, aw_raw) : ac;
        const R uE = hasE ? ue_raw : R(0);
        const R uW = hasW ? uw_raw : R(0);
        const R sa = aE + aW + aN + aS;
        const R Au = (sa * uc - aE * uE - aW * uW - aN * un - aS * us) * ih2 +
                     (bxp * (uc - uW) + bxm * (uE - uc) + byp * (uc - us) + bym * (un - uc)) * ih;
        const R rr = fv - Au;
        if (rt != nullptr) {
          const R D = sa * ih2 + conv_diag;
          rt[base + ij] = (float)(rr * (R)__builtin_amdgcn_rcp((double)D));
        }
        r2 += (double)rr * (double)rr;
        // the next row's south face: the same face in the divergence form, the next node's own
        // value in the non-divergence form
        us = uc; uc = un; ac = an; aS = form ? an : aN;
      }
    } else {
      (void)a; (void)bvec; (void)u; (void)rt;
      for (int r = 0; r < RES_ROWS; ++r) {
        const int i = i0 + r;
        if (i >= n) break;
        const double v = (double)F[i * n + j];
        r2 += v * v;
      }
    }
  }
  r2 = block_sum_256(r2);
  if (threadIdx.x == 0) partial[(size_t)b * tiles_per_prob + tile] = r2;
}

void launch_residual(const float* a, const float* b, const float* f, const void* u, bool u_f64,
                     float* rt, double* partial, int n, int B, const int* active, int form,
                     hipStream_t st) {
  const int tx = (n + 255) / 256, ty = (n + RES_ROWS - 1) / RES_ROWS;
  const dim3 grid(tx * ty * B), blk(256);
  if (u == nullptr) {
    hipLaunchKernelGGL((residual_kernel<double, double, false>), grid, blk, 0, st, a, b, f,
                       (const double*)nullptr, rt, partial, n, tx, tx * ty, active, form);
  } else if (u_f64) {
    hipLaunchKernelGGL((residual_kernel<double, double, true>), grid, blk, 0, st, a, b, f,
                       (const double*)u, rt, partial, n, tx, tx * ty, active, form);
  } else {
    hipLaunchKernelGGL((residual_kernel<float, float, true>), grid, blk, 0, st, a, b, f,
                       (const float*)u, rt, partial, n, tx, tx * ty, active, form);
  }
}

// ------------------------------------------------------------------------------------------
// per-problem reductions and the stopping rule
// ------------------------------------------------------------------------------------------
__device__ double sum_partials_block(const double* p, int tiles) {
  double s = 0.0;
  for (int k = threadIdx.x; k < tiles; k += 256) s += p[k];
  return block_sum_256(s);
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial,
                                                           int tiles, double* __restrict__ out) {
  const int b = blockIdx.x;
  const double s = sum_partials_block(partial + (size_t)b * tiles, tiles);
  if (threadIdx.x == 0) out[b] = s;
}

void launch_sum_partials(const double* partial, int tiles, double* out, int B, hipStream_t st) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(B), dim3(256), 0, st, partial, tiles, out);
}

// relres[b] = ||r_b|| / ||f_b|| from the residual's partial sums and ||f_b||^2 (0 when f_b = 0).
__global__ __launch_bounds__(256) void relres_kernel(const double* __restrict__ partial, int tiles,
                                                     const double* __restrict__ nf2,
                                                     double* __restrict__ relres) {
  const int b = blockIdx.x;
  const double s = sum_partials_block(partial + (size_t)b * tiles, tiles);
  if (threadIdx.x == 0) relres[b] = nf2[b] > 0.0 ? sqrt(s) / sqrt(nf2[b]) : 0.0;
}

void launch_relres(const double* partial, int tiles, const double* nf2, double* relres, int B,
                   hipStream_t st) {
  hipLaunchKernelGGL(relres_kernel, dim3(B), dim3(256), 0, st, partial, tiles, nf2, relres);
}

// Stopping rule at iterate k = iters[b] (relative residual rho_k = ||r_k|| / ||f||):
//   rho_k <= tol          -> OK, stop (iters = k)
//   k == maxit            -> NOT_CONVERGED, stop
//   rho_k not finite or > 1e10 -> DIVERGED, stop
//   otherwise one more V-cycle is applied and iters becomes k + 1.
__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ partial,
                                                       int tiles, const double* __restrict__ nf2,
                                                       double tol, int maxit, int* active,
                                                       int* status, int* iters, double* relres,
                                                       long long* done_clock) {
  const int b = blockIdx.x;
  if (active[b] == 0) return;
  const double s = sum_partials_block(partial + (size_t)b * tiles, tiles);
  if (threadIdx.x != 0) return;
  const double rho = sqrt(s) / sqrt(nf2[b]);
  const int k = iters[b];
  relres[b] = rho;
  bool done = true;
  if (rho <= tol) {
    status[b] = 0;
  } else if (k >= maxit) {
    status[b] = 1;
  } else if (!(rho <= 1e10)) {
    status[b] = -6;
  } else {
    iters[b] = k + 1;
    done = false;
  }
  if (done) {
    active[b] = 0;
    if (done_clock != nullptr) done_clock[b] = wall_clock64();
  }
}

__global__ void clock_stamp_kernel(long long* out) {
  if (threadIdx.x == 0) out[0] = wall_clock64();
}

void launch_clock_stamp(long long* out, hipStream_t st) {
  hipLaunchKernelGGL(clock_stamp_kernel, dim3(1), dim3(64), 0, st, out);
}

void launch_finalize(const double* partial, int tiles, const double* nf2, double tol, int maxit,
                     int* active, int* status, int* iters, double* relres, int B, hipStream_t st,
                     long long* done_clock) {
  hipLaunchKernelGGL(finalize_kernel, dim3(B), dim3(256), 0, st, partial, tiles, nf2, tol, maxit,
                     active, status, iters, relres, done_clock);
}

__global__ void solve_init_kernel(const double* __restrict__ nf2, int* active, int* status,
                                  int* iters, double* relres, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const bool live = nf2[b] > 0.0;
  active[b] = live ? 1 : 0;
  status[b] = live ? 1 : 0;
  iters[b] = 0;
  relres[b] = live ? 1.0 : 0.0;
}

void launch_solve_init(const double* nf2, int* active, int* status, int* iters, double* relres,
                       int B, hipStream_t st) {
  hipLaunchKernelGGL(solve_init_kernel, dim3((B + 255) / 256), dim3(256), 0, st, nf2, active,
                     status, iters, relres, B);
}

// ------------------------------------------------------------------------------------------
// reChannel convolutions with few channels on one side (VALU direct conv).
// ------------------------------------------------------------------------------------------

// out[px][o] = sum_{c,p,q} W[o][c][p][q] in[px + (p-1, q-1)][c], CIN in {1, 4}.
// PAIR (packed pairs of problems, networks of at most 8 hidden channels): output slot b holds
// problem 2b in channels 0..7 and problem 2b + 1 in channels 8..15, each from its own input with
// the first eight rows of W (problem 2b + 1 absent when 2b + 1 = nprob: its channels are zero).
template <int CIN, typename OT, bool PAIR = false>
__global__ __launch_bounds__(256) void conv_in_kernel(const float* __restrict__ in,
                                                      const float* __restrict__ W,
                                                      OT* __restrict__ out, int n, int tiles_x,
                                                      int tiles_per_prob,
                                                      const int* __restrict__ active, int nprob) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  const int j = (tile % tiles_x) * 64 + (threadIdx.x & 63);
  const int i = (tile / tiles_x) * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  constexpr int NIN = PAIR ? 2 : 1;
  float v[NIN][9][CIN];
#pragma unroll
  for (int h = 0; h < NIN; ++h) {
    const int prob = PAIR ? 2 * b + h : b;
    const bool have = !PAIR || prob < nprob;
    const float* X = in + (size_t)(have ? prob : 0) * n * n * CIN;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int ii = i + p - 1, jj = j + q - 1;
        const bool ok = have && ii >= 0 && ii < n && jj >= 0 && jj < n;
        if constexpr (CIN == 4) {
          float4 z = ok ? reinterpret_cast<const float4*>(X)[(size_t)ii * n + jj]
                        : make_float4(0.f, 0.f, 0.f, 0.f);
          v[h][p * 3 + q][0] = z.x; v[h][p * 3 + q][1] = z.y; v[h][p * 3 + q][2] = z.z; v[h][p * 3 + q][3] = z.w;
        } else {
          v[h][p * 3 + q][0] = ok ? X[(size_t)ii * n + jj] : 0.f;
        }
      }
    }
  }
  float acc[C];
#pragma unroll
  for (int o = 0; o < C; ++o) {
    const int h = PAIR ? o / 8 : 0, oo = PAIR ? o % 8 : o;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CIN; ++c)
#pragma unroll
      for (int k = 0; k < 9; ++k) s = fmaf(W[(oo * CIN + c) * 9 + k], v[h][k][c], s);
    acc[o] = s;
  }
  store16(out + ((size_t)b * n * n + (size_t)i * n + j) * C, acc);
}

void launch_conv_in(int cin, const float* in, const float* W, void* out, StateType ot, int n,
                    int B, const int* active, hipStream_t st) {
  const int tx = (n + 63) / 64, ty = (n + 3) / 4;
  const dim3 grid(tx * ty * B), blk(256);
  if (cin == 1) {
    if (ot != ST_BF16)
      hipLaunchKernelGGL((conv_in_kernel<1, float>), grid, blk, 0, st, in, W, (float*)out, n, tx,
                         tx * ty, active, B);
    else
      hipLaunchKernelGGL((conv_in_kernel<1, bf16_t>), grid, blk, 0, st, in, W, (bf16_t*)out, n,
                         tx, tx * ty, active, B);
  } else {
    if (ot != ST_BF16)
      hipLaunchKernelGGL((conv_in_kernel<4, float>), grid, blk, 0, st, in, W, (float*)out, n, tx,
                         tx * ty, active, B);
    else
      hipLaunchKernelGGL((conv_in_kernel<4, bf16_t>), grid, blk, 0, st, in, W, (bf16_t*)out, n,
                         tx, tx * ty, active, B);
  }
}

void launch_conv_in_pairs(const float* in, const float* W, float* out, int n, int nprob, hipStream_t st) {
  const int tx = (n + 63) / 64, ty = (n + 3) / 4, slots = (nprob + 1) / 2;
  hipLaunchKernelGGL((conv_in_kernel<4, float, true>), dim3(tx * ty * slots), dim3(256), 0, st, in, W, out,
                     n, tx, tx * ty, (const int*)nullptr, nprob);
}

// u[px] += sum_{c,p,q} W[0][c][p][q] x[px + (p-1, q-1)][c]
//
// Each workgroup covers an OU_TH x OU_TW output tile.  Every pixel of the tile plus its one-pixel
// halo is read once (its 16 channels straight into registers) and reduced over the channels for
// all nine taps: y_t(q) = sum_c W[c][t] x[q][c].  The nine partial sums go to LDS and every output
// adds the nine values of its neighbours, u(p) += sum_t y_t(p - d_t).
constexpr int OU_TH = 8, OU_TW = 64;
constexpr int OU_SH = OU_TH + 2, OU_SW = OU_TW + 2;

// PAIR: slot b carries problem 2b in channels 0..7 and problem 2b + 1 in channels 8..15 (packed
// pairs); each is reduced with the first eight channels of W into its own u (absent problem
// 2b + 1 = nprob is skipped), and `flags` holds per-problem flags.
template <typename XT, typename UT, bool PAIR = false>
__global__ __launch_bounds__(256) void out_update_kernel(const XT* __restrict__ x,
                                                         const float* __restrict__ W,
                                                         UT* __restrict__ u, int n, int tiles_x,
                                                         int tiles_per_prob,
                                                         const int* __restrict__ active,
                                                         const int* __restrict__ flags,
                                                         int accumulate, int nprob) {
  constexpr int NO = PAIR ? 2 : 1;            // outputs per slot
  // tap partials of one problem at a time (packed pairs: the two problems of the slot in turn,
  // from the same staged values, so the LDS of a tile is that of one problem)
  __shared__ float Y[1][9][OU_SH * OU_SW];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int b = active != nullptr ? active[slot] : slot;   // compact list of the live problems
  bool live[NO];
  bool any = false;
#pragma unroll
  for (int h = 0; h < NO; ++h) {
    const int prob = PAIR ? 2 * b + h : b;
    live[h] = (!PAIR || prob < nprob) && (flags == nullptr || flags[prob] != 0);   // retired since the list was built
    any = any || live[h];
  }
  if (!any) return;
  const int i0 = (tile / tiles_x) * OU_TH - 1, j0 = (tile % tiles_x) * OU_TW - 1;
  const XT* X = x + (size_t)b * n * n * C;
  // output (r, cc) sits at staged (r + 1, cc + 1); tap (p, q) reads staged (r + p, cc + q)
  auto outputs = [&](int h) {
    const size_t ubase = (size_t)(PAIR ? 2 * b + h : b) * n * n;
    for (int o = threadIdx.x; o < OU_TH * OU_TW; o += 256) {
      const int r = o / OU_TW, cc = o % OU_TW;
      const int i = i0 + 1 + r, j = j0 + 1 + cc;
      if (i >= n || j >= n) continue;
      float acc = 0.f;
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += Y[0][p * 3 + q][(r + p) * OU_SW + cc + q];
      UT* U = u + ubase + (size_t)i * n + j;
      *U = accumulate ? *U + (UT)acc : (UT)acc;
    }
  };
  if constexpr (!PAIR) {
    for (int q = threadIdx.x; q < OU_SH * OU_SW; q += 256) {
      const int ii = i0 + q / OU_SW, jj = j0 + q % OU_SW;
      float y[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) y[k] = 0.f;
      if (ii >= 0 && ii < n && jj >= 0 && jj < n) {
        float v[C];
        load16(X + ((size_t)ii * n + jj) * C, v);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int k = 0; k < 9; ++k) y[k] = fmaf(W[c * 9 + k], v[c], y[k]);
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) Y[0][k][q] = y[k];
    }
    __syncthreads();
    if (live[0]) outputs(0);
  } else {
    // every staged pixel's sixteen channels are loaded once; the two halves then produce their
    // tap partials in turn
    constexpr int QPT = (OU_SH * OU_SW + 255) / 256;   // staged pixels per thread
    float v[QPT][C];
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
      const int q = threadIdx.x + 256 * r;
      const int ii = i0 + q / OU_SW, jj = j0 + q % OU_SW;
      if (q < OU_SH * OU_SW && ii >= 0 && ii < n && jj >= 0 && jj < n) {
        load16(X + ((size_t)ii * n + jj) * C, v[r]);
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) v[r][c] = 0.f;
      }
    }
#pragma unroll
    for (int h = 0; h < NO; ++h) {
      if (h > 0) __syncthreads();   // the previous problem's outputs have read Y
#pragma unroll
      for (int r = 0; r < QPT; ++r) {
        const int q = threadIdx.x + 256 * r;
        if (q >= OU_SH * OU_SW) continue;
        const int ii = i0 + q / OU_SW, jj = j0 + q % OU_SW;
        float y[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) y[k] = 0.f;
        if (ii >= 0 && ii < n && jj >= 0 && jj < n) {
#pragma unroll
          for (int cc = 0; cc < 8; ++cc)
#pragma unroll
            for (int k = 0; k < 9; ++k) y[k] = fmaf(W[cc * 9 + k], v[r][8 * h + cc], y[k]);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) Y[0][k][q] = y[k];
      }
      __syncthreads();
      if (live[h]) outputs(h);
    }
  }
}

template <bool PAIR>
static void out_update_launch(StateType t, const void* x, const float* Wout, void* u, bool u_f64, int n,
                              int slots, int nprob, const int* active, hipStream_t st, bool accumulate,
                              const int* flags) {
  const int tx = (n + OU_TW - 1) / OU_TW, ty = (n + OU_TH - 1) / OU_TH;
  const dim3 grid(tx * ty * slots), blk(256);
  const int acc = accumulate ? 1 : 0;
  if (t != ST_BF16) {
    if (u_f64)
      hipLaunchKernelGGL((out_update_kernel<float, double, PAIR>), grid, blk, 0, st, (const float*)x,
                         Wout, (double*)u, n, tx, tx * ty, active, flags, acc, nprob);
    else
      hipLaunchKernelGGL((out_update_kernel<float, float, PAIR>), grid, blk, 0, st, (const float*)x,
                         Wout, (float*)u, n, tx, tx * ty, active, flags, acc, nprob);
  } else {
    if (u_f64)
      hipLaunchKernelGGL((out_update_kernel<bf16_t, double, PAIR>), grid, blk, 0, st, (const bf16_t*)x,
                         Wout, (double*)u, n, tx, tx * ty, active, flags, acc, nprob);
    else
      hipLaunchKernelGGL((out_update_kernel<bf16_t, float, PAIR>), grid, blk, 0, st, (const bf16_t*)x,
                         Wout, (float*)u, n, tx, tx * ty, active, flags, acc, nprob);
  }
}

void launch_out_update(StateType t, const void* x, const float* Wout, void* u, bool u_f64, int n,
                       int B, const int* active, hipStream_t st, bool accumulate, const int* flags) {
  out_update_launch<false>(t, x, Wout, u, u_f64, n, B, B, active, st, accumulate, flags);
}

void launch_out_update_pairs(StateType t, const void* x, const float* Wout, void* u, bool u_f64, int n,
                             int slots, int nprob, const int* active, hipStream_t st, bool accumulate,
                             const int* flags) {
  out_update_launch<true>(t, x, Wout, u, u_f64, n, slots, nprob, active, st, accumulate, flags);
}

// ------------------------------------------------------------------------------------------
// utilities
// ------------------------------------------------------------------------------------------
__global__ void f32_to_bf16_kernel(const float* __restrict__ in, bf16_t* __restrict__ out,
                                   size_t count) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (size_t)gridDim.x * blockDim.x)
    out[k] = f32_to_bf16_rne(in[k]);
}

void launch_f32_to_bf16(const float* in, bf16_t* out, size_t count, hipStream_t st) {
  if (count == 0) return;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, out, count);
}

__global__ void zero_kernel(uint32_t* __restrict__ p, size_t words) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
       k += (size_t)gridDim.x * blockDim.x)
    p[k] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  if (words == 0) return;
  size_t blocks = (words + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, words);
}

__global__ void bf16_to_f32_kernel(const bf16_t* __restrict__ in, float* __restrict__ out,
                                   size_t count) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (size_t)gridDim.x * blockDim.x)
    out[k] = bf16_to_f32(in[k]);
}

void launch_bf16_to_f32(const bf16_t* in, float* out, size_t count, hipStream_t st) {
  if (count == 0) return;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(bf16_to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, out, count);
}

// u = 0 for every problem whose right-hand side is zero (its solution is exactly zero).
template <typename UT>
__global__ void zero_if_zero_rhs_kernel(UT* __restrict__ u, const double* __restrict__ nf2,
                                        size_t nn, int B) {
  const size_t total = nn * (size_t)B;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x)
    if (nf2[k / nn] == 0.0) u[k] = UT(0);
}

void launch_zero_if_zero_rhs(void* u, bool u_f64, const double* nf2, int n, int B, hipStream_t st) {
  const size_t nn = (size_t)n * n;
  size_t blocks = (nn * B + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (u_f64)
    hipLaunchKernelGGL(zero_if_zero_rhs_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (double*)u, nf2, nn, B);
  else
    hipLaunchKernelGGL(zero_if_zero_rhs_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (float*)u, nf2, nn, B);
}

// rt = r / D with D = diag A(a, b).
__global__ __launch_bounds__(256) void scale_by_diag_kernel(const float* __restrict__ a,
                                                            const float* __restrict__ bvec,
                                                            const float* __restrict__ r,
                                                            float* __restrict__ rt, int n,
                                                            int tiles_x, int tiles_per_prob,
                                                            int form) {
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int b = t / tiles_per_prob, tile = t % tiles_per_prob;
  const int j = (tile % tiles_x) * 64 + (threadIdx.x & 63);
  const int i = (tile / tiles_x) * 4 + (threadIdx.x >> 6);
  if (i >= n || j >= n) return;
  const float* A = a + (size_t)b * n * n;
  const size_t ij = (size_t)i * n + j;
  const double ac = A[ij];
  const double aE = (j + 1 < n) ? (form ? ac : harm<double>(ac, A[ij + 1])) : ac;
  const double aW = (j > 0) ? (form ? ac : harm<double>(ac, A[ij - 1])) : ac;
  const double aN = (i + 1 < n) ? (form ? ac : harm<double>(ac, A[ij + n])) : ac;
  const double aS = (i > 0) ? (form ? ac : harm<double>(ac, A[ij - n])) : ac;
  const double ih = (double)(n + 1);
  const double D = (aE + aW + aN + aS) * ih * ih + (fabs((double)bvec[2 * b]) + fabs((double)bvec[2 * b + 1])) * ih;
  rt[(size_t)b * n * n + ij] = (float)((double)r[(size_t)b * n * n + ij] / D);
}

void launch_scale_by_diag(const float* a, const float* b, const float* r, float* rt, int n, int B,
                          int form, hipStream_t st) {
  const int tx = (n + 63) / 64, ty = (n + 3) / 4;
  hipLaunchKernelGGL(scale_by_diag_kernel, dim3(tx * ty * B), dim3(256), 0, st, a, b, r, rt, n, tx,
                     tx * ty, form);
}

}  // namespace mg
