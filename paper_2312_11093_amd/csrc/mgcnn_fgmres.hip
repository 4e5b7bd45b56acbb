// Batched restarted FGMRES with the MGCNN network as a fixed right preconditioner.
//
// The network is linear in its input (principle P2, Sec. 3.1), so it can serve as the
// preconditioner of a Krylov method (Sec. 2.2).  Each problem of the batch runs its own
// FGMRES(m): Arnoldi vectors and preconditioned vectors are float32 (classical Gram-Schmidt
// applied twice), the true residual f - A u is recomputed in f64 at every restart and u is
// accumulated in f64, so the outer loop is an iterative refinement and the tolerance is
// checked on the true relative residual.  Problems that meet the tolerance retire.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_ctx.h"
#include "mgcnn_internal.h"
#include "mgcnn_krylov.h"

using namespace mg;
using namespace mg::api;

namespace mg {
void launch_zero_if_zero_rhs(void* u, bool u_f64, const double* nf2, int n, int B, hipStream_t st);

namespace api {

void free_krylov(mgcnn_ctx* c) {
  auto& K = c->kr;
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(K.V); fr(K.Z); fr(K.partial); fr(K.h); fr(K.s); fr(K.act); fr(K.cyc);
  K = mgcnn_ctx::Krylov{};
}

static int ensure_krylov(mgcnn_ctx* c, int m) {
  auto& K = c->kr;
  if (K.n == c->n && K.B == c->B && K.m >= m) return MGCNN_OK;
  free_krylov(c);
  const size_t nn = (size_t)c->n * c->n * c->B;
  const size_t nv = krylov_vpad(c->n) * c->B;
  const size_t ld = (size_t)c->B * KRYLOV_LD * 8;
  int r;
  if ((r = alloc(c, (void**)&K.V, nv * 4 * (m + 1)))) return r;
  // the padding of every basis vector stays zero (set once here, outside any captured work)
  HIP_TRY(c, hipMemset(K.V, 0, nv * 4 * (m + 1)));
  if ((r = alloc(c, (void**)&K.Z, nn * 4 * m))) return r;
  if ((r = alloc(c, (void**)&K.partial, (size_t)krylov_blocks(c->n) * ld))) return r;
  if ((r = alloc(c, (void**)&K.h, ld))) return r;
  if ((r = alloc(c, (void**)&K.s, ld))) return r;
  if ((r = alloc(c, (void**)&K.act, (size_t)c->B * 4))) return r;
  if ((r = alloc(c, (void**)&K.cyc, (size_t)c->B * 4))) return r;
  K.n = c->n; K.B = c->B; K.m = m;
  return MGCNN_OK;
}

// Restarted FGMRES(m), right preconditioned by z = B(v / D), one Arnoldi process per problem.
// Orthogonalisation: classical Gram-Schmidt applied twice (three passes over the basis).  The
// small least-squares problems (Givens rotations) run on the host in f64.  Every launch covers
// a compact list of the problems still extending their basis.
int fgmres_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
                 double* relres_host, int* status_host) {
  const int m = std::max(1, std::min(c->opts.restart > 0 ? c->opts.restart : 30, KRYLOV_MAX_BASIS - 1));
  int r = ensure_krylov(c, m);
  if (r) return r;
  auto& K = c->kr;
  hipStream_t s = c->stream;
  const int B = c->B, n = c->n;
  const size_t nn = (size_t)n * n * B;
  const size_t vs = krylov_vpad(n) * B;      // stride between basis vectors (floats)
  const size_t zs = nn;                      // stride between preconditioned vectors
  const bool u64 = c->u64();
  const double nodes1 = (double)n * n;       // nodes of one problem
  const int LD = KRYLOV_LD;
  const bool two_pass = c->opts.gs_passes != 1;
  // ||f||^2
  launch_residual(c->d_a, c->d_b, f, nullptr, true, nullptr, c->d_partial, n, B, nullptr, c->form(), s);
  launch_sum_partials(c->d_partial, c->tiles, c->d_nf2, B, s);
  launch_zero_if_zero_rhs(u, u64, c->d_nf2, n, B, s);
  std::vector<double> nf2(B);
  HIP_TRY(c, hipMemcpyAsync(nf2.data(), c->d_nf2, (size_t)B * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  std::vector<int> status(B, MGCNN_NOT_CONVERGED), iters(B, 0), act(B, 0), cyc(B, 0);
  std::vector<double> relres(B, 0.0);
  for (int b = 0; b < B; ++b) {
    if (nf2[b] > 0.0) act[b] = 1;
    else { status[b] = MGCNN_OK; relres[b] = 0.0; }
  }
  const int HL = KRYLOV_MAX_BASIS;
  std::vector<double> H((size_t)B * (HL + 1) * HL), g((size_t)B * HL + B), cs((size_t)B * HL),
      sn((size_t)B * HL), hb((size_t)B * LD), hb2((size_t)B * LD), hb3((size_t)B * LD),
      sc((size_t)B * LD, 0.0),
      nw2(B, 0.0);
  std::vector<int> kb(B), list_live(B), list_cyc(B);
  auto Hij = [&](int b, int i, int j) -> double& { return H[((size_t)b * (HL + 1) + i) * HL + j]; };
  auto gi = [&](int b, int i) -> double& { return g[(size_t)b * (HL + 1) + i]; };
  // upload the compact list of the problems whose flag is set; returns its length.  The host
  // buffer stays untouched until the next upload, which follows a stream synchronisation.
  auto to_list = [&](int* d, std::vector<int>& buf, const std::vector<int>& flags, int& count) {
    count = 0;
    for (int b = 0; b < B; ++b)
      if (flags[b]) buf[count++] = b;
    if (count == 0) return hipSuccess;
    return hipMemcpyAsync(d, buf.data(), (size_t)count * 4, hipMemcpyHostToDevice, s);
  };
  auto from_dev = [&](std::vector<double>& h) {
    return hipMemcpyAsync(h.data(), K.h, (size_t)B * LD * 8, hipMemcpyDeviceToHost, s);
  };
  while (true) {
    // true residual of every live problem, its norm, and the stopping rule
    int nact = 0;
    HIP_TRY(c, to_list(K.act, list_live, act, nact));
    if (nact == 0) break;
    {
      Prof p(c, MGCNN_K_KRYLOV_RESIDUAL, 0, nodes1 * nact * (12.0 + (u64 ? 8 : 4)));
      launch_krylov_residual(c->d_a, c->d_b, f, u, u64, K.V, krylov_vpad(n), n, nact, K.act,
                             c->form(), s);
    }
    {
      Prof p(c, MGCNN_K_KRYLOV_DOTS, 0, nodes1 * nact * 4.0);
      launch_gs_pass(0, K.V, K.V, vs, 0, n, nact, nullptr, K.partial, K.h, K.act, s);
    }
    LAUNCH_CHECK(c);
    HIP_TRY(c, from_dev(hb));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->prof && (r = prof_drain(c))) return r;
    bool any = false;
    for (int b = 0; b < B; ++b) {
      cyc[b] = 0;
      if (!act[b]) continue;
      const double beta = std::sqrt(std::max(hb[(size_t)b * LD], 0.0));
      const double rho = beta / std::sqrt(nf2[b]);
      relres[b] = rho;
      if (rho <= tol) { status[b] = MGCNN_OK; act[b] = 0; }
      else if (iters[b] >= maxit) { status[b] = MGCNN_NOT_CONVERGED; act[b] = 0; }
      else if (!(rho <= 1e10)) { status[b] = MGCNN_E_DIVERGED; act[b] = 0; }
      else {
        cyc[b] = 1;
        any = true;
        sc[(size_t)b * LD] = 1.0 / beta;
        for (int i = 0; i <= HL; ++i) gi(b, i) = 0.0;
        gi(b, 0) = beta;
        std::fill(&Hij(b, 0, 0), &Hij(b, 0, 0) + (size_t)(HL + 1) * HL, 0.0);
        kb[b] = 0;
      }
    }
    if (!any) break;
    std::vector<int> live = cyc;                 // problems still extending their basis this cycle
    int ncyc = 0, nlive = 0;
    HIP_TRY(c, to_list(K.cyc, list_cyc, cyc, ncyc));
    HIP_TRY(c, to_list(K.act, list_live, live, nlive));
    for (int j = 0; j < m; ++j) {
      float* Vj = K.V + (size_t)j * vs;
      float* Vn = K.V + (size_t)(j + 1) * vs;
      float* Zj = K.Z + (size_t)j * zs;
      const double nodes = nodes1 * nlive;
      // v_j /= |v_j| (in place) and z_j = B(v_j / D)
      HIP_TRY(c, hipMemcpyAsync(K.s, sc.data(), (size_t)B * LD * 8, hipMemcpyHostToDevice, s));
      {
        Prof p(c, MGCNN_K_SCALE_BY_DIAG, 0, nodes * 16.0);
        launch_normalize_diag(c->d_a, c->d_b, Vj, c->d_rt, K.s, n, nlive, K.act, c->form(), s);
      }
      if ((r = vcycle(c, Zj, false, K.act, nlive, false))) return r;
      // optional further stationary steps on v_j: z_j += B((v_j - A z_j) / D)
      for (int k = 1; k < c->opts.inner_steps; ++k) {
        {
          Prof p(c, MGCNN_K_KRYLOV_APPLY_A, 1, nodes * 16.0);
          launch_inner_residual(c->d_a, c->d_b, Vj, Zj, c->d_rt, n, nlive, K.act, c->form(), s);
        }
        if ((r = vcycle(c, Zj, false, K.act, nlive, true))) return r;
      }
      // w = A z_j
      {
        Prof p(c, MGCNN_K_KRYLOV_APPLY_A, 0, nodes * 12.0);
        launch_apply_A(c->d_a, c->d_b, Zj, Vn, krylov_vpad(n), n, nlive, K.act, c->form(), s);
      }
      // classical Gram-Schmidt applied twice, in three passes:
      //   h1 = V^T w ; w -= V h1 and h2 = V^T w ; w -= V h2 and |w|^2
      // (once, in two passes, when opts.gs_passes = 1: h1 = V^T w ; w -= V h1 and |w|^2)
      const int cnt = j + 1;
      {
        Prof p(c, MGCNN_K_KRYLOV_DOTS, cnt, nodes * 4.0 * (cnt + 1));
        launch_gs_pass(0, Vn, K.V, vs, cnt, n, nlive, nullptr, K.partial, K.h, K.act, s);
      }
      HIP_TRY(c, from_dev(hb));
      if (two_pass) {
        Prof p(c, MGCNN_K_KRYLOV_ORTH, cnt, nodes * 4.0 * (cnt + 2));
        launch_gs_pass(1, Vn, K.V, vs, cnt, n, nlive, K.h, K.partial, K.h, K.act, s);
      }
      if (two_pass) HIP_TRY(c, from_dev(hb2));
      {
        Prof p(c, MGCNN_K_KRYLOV_ORTH, cnt, nodes * 4.0 * (cnt + 2));
        launch_gs_pass(2, Vn, K.V, vs, cnt, n, nlive, K.h, K.partial, K.h, K.act, s);
      }
      LAUNCH_CHECK(c);
      HIP_TRY(c, from_dev(hb3));
      HIP_TRY(c, hipStreamSynchronize(s));
      for (int b = 0; b < B; ++b) {
        if (!live[b]) continue;
        for (int i = 0; i < cnt; ++i)
          Hij(b, i, j) = hb[(size_t)b * LD + i] + (two_pass ? hb2[(size_t)b * LD + i] : 0.0);
        nw2[b] = hb3[(size_t)b * LD];
      }
      if (c->prof && (r = prof_drain(c))) return r;   // the stream is idle here
      bool more = false;
      for (int b = 0; b < B; ++b) {
        if (!live[b]) continue;
        const double hn = std::sqrt(std::max(nw2[b], 0.0));
        Hij(b, j + 1, j) = hn;
        sc[(size_t)b * LD] = hn > 0.0 ? 1.0 / hn : 0.0;
        // Givens rotations: previous ones on column j, then a new one for (j, j+1)
        for (int i = 0; i < j; ++i) {
          const double c0 = cs[(size_t)b * HL + i], s0 = sn[(size_t)b * HL + i];
          const double h0 = Hij(b, i, j), h1 = Hij(b, i + 1, j);
          Hij(b, i, j) = c0 * h0 + s0 * h1;
          Hij(b, i + 1, j) = -s0 * h0 + c0 * h1;
        }
        const double h0 = Hij(b, j, j), h1 = Hij(b, j + 1, j);
        const double rr = std::hypot(h0, h1);
        const double c0 = rr > 0.0 ? h0 / rr : 1.0, s0 = rr > 0.0 ? h1 / rr : 0.0;
        cs[(size_t)b * HL + j] = c0; sn[(size_t)b * HL + j] = s0;
        Hij(b, j, j) = rr; Hij(b, j + 1, j) = 0.0;
        const double gj = gi(b, j);
        gi(b, j) = c0 * gj;
        gi(b, j + 1) = -s0 * gj;
        iters[b] += 1;
        kb[b] = j + 1;
        const double est = std::fabs(gi(b, j + 1)) / std::sqrt(nf2[b]);
        if (est <= tol || iters[b] >= maxit || hn == 0.0 || !std::isfinite(est)) live[b] = 0;
        else more = true;
      }
      if (!more || j == m - 1) break;
      HIP_TRY(c, to_list(K.act, list_live, live, nlive));
    }
    // y = R^-1 g (upper triangular, k_b x k_b) and u += Z y
    std::fill(sc.begin(), sc.end(), 0.0);
    int kmax = 0;
    for (int b = 0; b < B; ++b) {
      if (!cyc[b]) continue;
      const int k = kb[b];
      kmax = std::max(kmax, k);
      for (int i = k - 1; i >= 0; --i) {
        double acc = gi(b, i);
        for (int l = i + 1; l < k; ++l) acc -= Hij(b, i, l) * sc[(size_t)b * LD + l];
        sc[(size_t)b * LD + i] = Hij(b, i, i) != 0.0 ? acc / Hij(b, i, i) : 0.0;
      }
    }
    HIP_TRY(c, hipMemcpyAsync(K.s, sc.data(), (size_t)B * LD * 8, hipMemcpyHostToDevice, s));
    {
      Prof p(c, MGCNN_K_KRYLOV_COMBINE, kmax, nodes1 * ncyc * (4.0 * kmax + 2.0 * (u64 ? 8 : 4)));
      launch_combine(u, u64, K.Z, zs, kmax, n, ncyc, K.s, K.cyc, s);
    }
    LAUNCH_CHECK(c);
    HIP_TRY(c, hipStreamSynchronize(s));      // sc and the list buffers are rewritten next cycle
  }
  bool diverged = false, notconv = false;
  for (int b = 0; b < B; ++b) {
    if (iters_host) iters_host[b] = iters[b];
    if (relres_host) relres_host[b] = relres[b];
    if (status_host) status_host[b] = status[b];
    diverged |= status[b] == MGCNN_E_DIVERGED;
    notconv |= status[b] == MGCNN_NOT_CONVERGED;
  }
  if (diverged) return fail(c, MGCNN_E_DIVERGED, "solve: a problem diverged");
  if (notconv) return MGCNN_NOT_CONVERGED;
  return MGCNN_OK;
}

}  // namespace api
}  // namespace mg
