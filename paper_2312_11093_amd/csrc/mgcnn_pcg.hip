// Batched preconditioned conjugate gradients for symmetric problems (b = 0, divergence form):
// the short recurrence that a symmetric positive definite operator and preconditioner allow,
// with the V-cycle or the symmetric variant of the network (Sec. 3.3) as preconditioner of a
// Krylov method (Sec. 2.2).
//
// Each problem of the batch runs its own recurrence
//   z_k = M r_k,  beta = (r_k, z_k) / (r_{k-1}, z_{k-1}),  p_k = z_k + beta p_{k-1},
//   alpha = (r_k, z_k) / (p_k, A p_k),  u += alpha p_k,  r -= alpha A p_k
// with M = V-cycle(r / D) or D^-1/2 B(D^-1/2 r) for the network.  The vectors are float32,
// u float32 or float64, inner products f64.  The float32 recurrence residual drifts from the
// true one by float32 roundings of the updates (about 1e-7 of the largest residual of the
// cycle per step), so the recurrence runs in cycles, an iterative refinement: a cycle starts
// from the true residual f - A u (computed in f64) with beta = 0 and ends when its recurrence
// residual has dropped by PCG_CYCLE_DROP from that start, or meets the tolerance, or the step
// count reaches maxit; the next pass then recomputes f - A u for the same u, which decides the
// stopping rule.  Keeping the search direction across such a replacement (as in
// reliable-update schemes) fails here: once the recurrence sits below the true residual,
// beta = (r, z)_true / (r, z)_old is far too large.  One host synchronisation after (r, z) and
// one after (p, A p) per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_ctx.h"
#include "mgcnn_internal.h"
#include "mgcnn_krylov.h"
#include "mgcnn_pcg.h"

using namespace mg;
using namespace mg::api;

namespace mg {

namespace api {

// reduction of the recurrence residual within one cycle, well above the float32 drift
constexpr double PCG_CYCLE_DROP = 1e-5;

void free_pcg(mgcnn_ctx* c) {
  auto& P = c->pcg;
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(P.vec); fr(P.ones); fr(P.partial); fr(P.out); fr(P.coef); fr(P.unit); fr(P.lists);
  P = mgcnn_ctx::Pcg{};
}

static int ensure_pcg(mgcnn_ctx* c) {
  auto& P = c->pcg;
  if (P.vec && P.n == c->n && P.B == c->B) return MGCNN_OK;
  free_pcg(c);
  const size_t nn = (size_t)c->n * c->n * c->B;
  int r;
  if ((r = alloc(c, (void**)&P.vec, nn * 4 * 5))) return r;
  if ((r = alloc(c, (void**)&P.ones, krylov_vpad(c->n) * c->B * 4))) return r;
  if ((r = alloc(c, (void**)&P.partial, (size_t)c->B * pcg_blocks(c->n) * 2 * 8))) return r;
  if ((r = alloc(c, (void**)&P.out, (size_t)c->B * 2 * 8))) return r;
  if ((r = alloc(c, (void**)&P.coef, (size_t)c->B * 2 * 8))) return r;
  if ((r = alloc(c, (void**)&P.unit, (size_t)c->B * KRYLOV_LD * 8))) return r;
  if ((r = alloc(c, (void**)&P.lists, (size_t)c->B * 3 * 4))) return r;
  P.n = c->n; P.B = c->B;
  return MGCNN_OK;
}

int pcg_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
              double* relres_host, int* status_host) {
  const int B = c->B, n = c->n;
  hipStream_t s = c->stream;
  {
    std::vector<float> bh((size_t)2 * B);
    HIP_TRY(c, hipMemcpyAsync(bh.data(), c->d_b, bh.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    for (float v : bh)
      if (v != 0.f) return fail(c, MGCNN_E_ARG, "solve: conjugate gradients need b = 0 (a symmetric operator)");
  }
  int r = ensure_pcg(c);
  if (r) return r;
  auto& P = c->pcg;
  const bool u64 = c->u64();
  const bool net = c->opts.precond == MGCNN_PRECOND_NETWORK;
  const size_t nn = (size_t)n * n * B;
  const double nodes1 = (double)n * n, ub = u64 ? 8.0 : 4.0;
  float* R = P.vec;
  float* Pd = P.vec + nn;
  float* Q = P.vec + 2 * nn;
  float* Z = P.vec + 3 * nn;
  float* dsc = P.vec + 4 * nn;
  int* dU = P.lists;            // recurrence updates (also the direction phase's list)
  int* dT = P.lists + B;        // true residual of the current u
  int* dL = P.lists + 2 * B;    // every live problem
  // ||f||^2; a zero right-hand side gives u = 0
  launch_residual(c->d_a, c->d_b, f, nullptr, true, nullptr, c->d_partial, n, B, nullptr, c->form(), s);
  launch_sum_partials(c->d_partial, c->tiles, c->d_nf2, B, s);
  launch_zero_if_zero_rhs(u, u64, c->d_nf2, n, B, s);
  // the diagonal scaling of the preconditioner's input: 1/D for the V-cycle (it takes r / D),
  // D^-1/2 on both sides of the network
  std::vector<double> unit((size_t)B * KRYLOV_LD, 1.0);
  HIP_TRY(c, hipMemcpyAsync(P.unit, unit.data(), unit.size() * 8, hipMemcpyHostToDevice, s));
  launch_pcg_fill(P.ones, 1.f, krylov_vpad(n) * B, s);
  launch_normalize_diag(c->d_a, c->d_b, P.ones, dsc, P.unit, n, B, nullptr, c->form(), s);
  if (net) launch_pcg_sqrt(dsc, nn, s);
  LAUNCH_CHECK(c);
  std::vector<double> nf2(B);
  HIP_TRY(c, hipMemcpyAsync(nf2.data(), c->d_nf2, (size_t)B * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  // phase of a live problem in the next pass: 0 = true residual of the current u (a cycle
  // starts), 2 = recurrence update of u and r
  std::vector<int> status(B, MGCNN_NOT_CONVERGED), iters(B, 0), live(B, 0), phase(B, 0), started(B, 0);
  std::vector<double> relres(B, 0.0), rz_old(B, 0.0), start(B, 0.0), out((size_t)2 * B, 0.0),
      coef((size_t)2 * B, 0.0);
  std::vector<int> hU(B), hT(B), hL(B);
  for (int b = 0; b < B; ++b) {
    if (nf2[b] > 0.0) live[b] = 1;
    else status[b] = MGCNN_OK;
  }
  auto upload = [&](int* d, std::vector<int>& h, int cnt) {
    return cnt ? hipMemcpyAsync(d, h.data(), (size_t)cnt * 4, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  while (true) {
    int nU = 0, nT = 0, nL = 0;
    for (int b = 0; b < B; ++b) {
      if (!live[b]) continue;
      hL[nL++] = b;
      if (phase[b] == 2) hU[nU++] = b;
      else hT[nT++] = b;
    }
    if (nL == 0) break;
    HIP_TRY(c, upload(dU, hU, nU));
    HIP_TRY(c, upload(dT, hT, nT));
    HIP_TRY(c, upload(dL, hL, nL));
    HIP_TRY(c, hipMemcpyAsync(P.coef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice, s));
    if (nU) {
      Prof p(c, MGCNN_K_KRYLOV_COMBINE, 0, nodes1 * nU * (2.0 * ub + 24.0));
      launch_pcg_step(PCG_UPDATE, u, u64, Pd, R, Q, dsc, c->d_rt, P.coef, P.partial, n, nU, dU, s);
    }
    if (nT) {
      {
        Prof p(c, MGCNN_K_KRYLOV_RESIDUAL, 0, nodes1 * nT * (12.0 + ub));
        launch_krylov_residual(c->d_a, c->d_b, f, u, u64, R, (size_t)n * n, n, nT, dT, c->form(), s);
      }
      Prof p(c, MGCNN_K_KRYLOV_SCALE, 0, nodes1 * nT * 12.0);
      launch_pcg_step(PCG_PREP, u, u64, Pd, R, Q, dsc, c->d_rt, P.coef, P.partial, n, nT, dT, s);
    }
    // z = M r on every live problem, then (r, z) and |r|^2
    if ((r = vcycle(c, Z, false, dL, nL, false))) return r;
    {
      Prof p(c, MGCNN_K_KRYLOV_DOTS, 1, nodes1 * nL * (net ? 16.0 : 8.0));
      launch_pcg_rz(net, Z, R, dsc, P.partial, n, nL, dL, s);
      launch_pcg_reduce(P.partial, 2, P.out, n, nL, dL, s);
    }
    LAUNCH_CHECK(c);
    HIP_TRY(c, hipMemcpyAsync(out.data(), P.out, out.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->prof && (r = prof_drain(c))) return r;
    int nD = 0;
    for (int t = 0; t < nL; ++t) {
      const int b = hL[t];
      const double est = std::sqrt(std::max(out[2 * b], 0.0) / nf2[b]);
      const double rz = out[2 * b + 1];
      if (phase[b] != 2) {          // a true residual decides, and a new cycle starts
        relres[b] = est;
        if (est <= tol) { status[b] = MGCNN_OK; live[b] = 0; continue; }
        if (iters[b] >= maxit) { status[b] = MGCNN_NOT_CONVERGED; live[b] = 0; continue; }
        if (!(est <= 1e10)) { status[b] = MGCNN_E_DIVERGED; live[b] = 0; continue; }
        start[b] = est;
        started[b] = 0;
      } else if (est <= tol || est <= PCG_CYCLE_DROP * start[b] || iters[b] >= maxit || !(est <= 1e10)) {
        phase[b] = 0;               // end of the cycle: the true residual of this u next pass
        continue;
      }
      if (!(rz > 0.0) || !std::isfinite(rz)) {   // M or A not definite: breakdown
        if (phase[b] == 2) relres[b] = est;
        status[b] = MGCNN_E_DIVERGED;
        live[b] = 0;
        continue;
      }
      coef[2 * b + 1] = started[b] ? rz / rz_old[b] : 0.0;
      started[b] = 1;
      rz_old[b] = rz;
      hU[nD++] = b;
    }
    if (nD == 0) continue;
    // p = z + beta p, q = A p, (p, q)
    HIP_TRY(c, upload(dU, hU, nD));
    HIP_TRY(c, hipMemcpyAsync(P.coef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice, s));
    {
      Prof p(c, MGCNN_K_KRYLOV_SCALE, 1, nodes1 * nD * 12.0);
      launch_pcg_dir(Pd, Z, P.coef, n, nD, dU, s);
    }
    {
      Prof p(c, MGCNN_K_KRYLOV_APPLY_A, 0, nodes1 * nD * 12.0);
      launch_apply_A(c->d_a, c->d_b, Pd, Q, (size_t)n * n, n, nD, dU, c->form(), s);
    }
    {
      Prof p(c, MGCNN_K_KRYLOV_DOTS, 0, nodes1 * nD * 8.0);
      launch_pcg_dot(Pd, Q, P.partial, n, nD, dU, s);
      launch_pcg_reduce(P.partial, 1, P.out, n, nD, dU, s);
    }
    LAUNCH_CHECK(c);
    HIP_TRY(c, hipMemcpyAsync(out.data(), P.out, out.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->prof && (r = prof_drain(c))) return r;
    for (int t = 0; t < nD; ++t) {
      const int b = hU[t];
      const double pq = out[2 * b];
      if (!(pq > 0.0) || !std::isfinite(pq)) {
        status[b] = MGCNN_E_DIVERGED;
        live[b] = 0;
        continue;
      }
      coef[2 * b] = rz_old[b] / pq;
      iters[b] += 1;
      phase[b] = 2;
    }
  }
  bool diverged = false, notconv = false;
  for (int b = 0; b < B; ++b) {
    if (iters_host) iters_host[b] = iters[b];
    if (relres_host) relres_host[b] = relres[b];
    if (status_host) status_host[b] = status[b];
    diverged |= status[b] == MGCNN_E_DIVERGED;
    notconv |= status[b] == MGCNN_NOT_CONVERGED;
  }
  if (diverged) return fail(c, MGCNN_E_DIVERGED, "solve: a problem diverged or broke down");
  if (notconv) return MGCNN_NOT_CONVERGED;
  return MGCNN_OK;
}

}  // namespace api
}  // namespace mg
