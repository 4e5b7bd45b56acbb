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
void launch_scale_by_diag(const float* a, const float* b, const float* r, float* rt, int n, int B,
                          hipStream_t st);
void launch_zero_if_zero_rhs(void* u, bool u_f64, const double* nf2, int n, int B, hipStream_t st);
void launch_residual_plain(const float* a, const float* b, const float* f, const void* u, bool u_f64,
                           float* r, int n, int B, hipStream_t st);

namespace api {

void free_krylov(mgcnn_ctx* c) {
  auto& K = c->kr;
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(K.V); fr(K.Z); fr(K.partial); fr(K.h); fr(K.act); fr(K.cyc);
  K = mgcnn_ctx::Krylov{};
}

static int ensure_krylov(mgcnn_ctx* c, int m) {
  auto& K = c->kr;
  if (K.n == c->n && K.B == c->B && K.m >= m) return MGCNN_OK;
  free_krylov(c);
  const size_t nn = (size_t)c->n * c->n * c->B;
  int r;
  if ((r = alloc(c, (void**)&K.V, nn * 4 * (m + 1)))) return r;
  if ((r = alloc(c, (void**)&K.Z, nn * 4 * m))) return r;
  if ((r = alloc(c, (void**)&K.partial, (size_t)c->B * krylov_blocks(c->n) * KRYLOV_MAX_BASIS * 8))) return r;
  if ((r = alloc(c, (void**)&K.h, (size_t)c->B * KRYLOV_MAX_BASIS * 8))) return r;
  if ((r = alloc(c, (void**)&K.act, (size_t)c->B * 4))) return r;
  if ((r = alloc(c, (void**)&K.cyc, (size_t)c->B * 4))) return r;
  K.n = c->n; K.B = c->B; K.m = m;
  return MGCNN_OK;
}

int fgmres_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
                 double* relres_host, int* status_host) {
  const int m = std::max(1, std::min(c->opts.restart > 0 ? c->opts.restart : 30, KRYLOV_MAX_BASIS - 1));
  int r = ensure_krylov(c, m);
  if (r) return r;
  auto& K = c->kr;
  hipStream_t s = c->stream;
  const int B = c->B, n = c->n;
  const size_t nn = (size_t)n * n * B;
  const size_t vs = nn;                       // stride between basis vectors (floats)
  const bool u64 = c->u64();
  const double nodes = (double)nn;           // all problems; retired ones are skipped by the kernels
  // ||f||^2
  launch_residual(c->d_a, c->d_b, f, nullptr, true, nullptr, c->d_partial, n, B, nullptr, s);
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
  const int LD = KRYLOV_MAX_BASIS;
  std::vector<double> H((size_t)B * (LD + 1) * LD), g((size_t)B * LD), cs((size_t)B * LD),
      sn((size_t)B * LD), hbuf((size_t)B * LD), ybuf((size_t)B * LD), sc(B);
  std::vector<int> kb(B);
  auto Hij = [&](int b, int i, int j) -> double& { return H[((size_t)b * (LD + 1) + i) * LD + j]; };
  while (true) {
    // true residual of every live problem, its norm, and the stopping rule
    {
      Prof p(c, MGCNN_K_KRYLOV_RESIDUAL, 0, nodes * (12.0 + (u64 ? 8 : 4)));
      launch_residual_plain(c->d_a, c->d_b, f, u, u64, K.V, n, B, s);
    }
    HIP_TRY(c, hipMemcpyAsync(K.act, act.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
    {
      Prof p(c, MGCNN_K_KRYLOV_DOTS, 1, nodes * 4.0);
      launch_dots(K.V, K.V, vs, 1, n, B, K.partial, K.h, K.act, s);
    }
    LAUNCH_CHECK(c);
    HIP_TRY(c, hipMemcpyAsync(hbuf.data(), K.h, (size_t)B * LD * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    bool any = false;
    for (int b = 0; b < B; ++b) {
      cyc[b] = 0;
      if (!act[b]) continue;
      const double beta = std::sqrt(std::max(hbuf[(size_t)b * LD], 0.0));
      const double rho = beta / std::sqrt(nf2[b]);
      relres[b] = rho;
      if (rho <= tol) { status[b] = MGCNN_OK; act[b] = 0; }
      else if (iters[b] >= maxit) { status[b] = MGCNN_NOT_CONVERGED; act[b] = 0; }
      else if (!(rho <= 1e10)) { status[b] = MGCNN_E_DIVERGED; act[b] = 0; }
      else {
        cyc[b] = 1;
        any = true;
        sc[b] = 1.0 / beta;
        for (int i = 0; i < LD; ++i) { g[(size_t)b * LD + i] = 0.0; }
        g[(size_t)b * LD] = beta;
        std::fill(&Hij(b, 0, 0), &Hij(b, 0, 0) + (size_t)(LD + 1) * LD, 0.0);
        kb[b] = 0;
      }
    }
    if (!any) break;
    std::vector<int> live = cyc;                 // problems still extending their basis this cycle
    HIP_TRY(c, hipMemcpyAsync(K.cyc, cyc.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(K.act, live.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(K.h, sc.data(), (size_t)B * 8, hipMemcpyHostToDevice, s));
    {
      Prof p(c, MGCNN_K_KRYLOV_SCALE, 0, nodes * 8.0);
      launch_scale(K.V, n, B, K.h, K.act, s);
    }
    for (int j = 0; j < m; ++j) {
      float* Vj = K.V + (size_t)j * vs;
      float* Vn = K.V + (size_t)(j + 1) * vs;
      float* Zj = K.Z + (size_t)j * vs;
      // z_j = B(v_j / D)
      {
        Prof p(c, MGCNN_K_SCALE_BY_DIAG, 0, nodes * 12.0);
        launch_scale_by_diag(c->d_a, c->d_b, Vj, c->d_rt, n, B, s);
      }
      {
        Prof p(c, MGCNN_K_ZERO, 0, nodes * 4.0);
        launch_zero(Zj, nn * 4, s);
      }
      if ((r = vcycle(c, Zj, false, K.act))) return r;
      // w = A z_j, orthogonalised twice against v_0..v_j
      {
        Prof p(c, MGCNN_K_KRYLOV_APPLY_A, 0, nodes * 12.0);
        launch_apply_A(c->d_a, c->d_b, Zj, Vn, n, B, K.act, s);
      }
      for (int pass = 0; pass < 2; ++pass) {
        {
          Prof p(c, MGCNN_K_KRYLOV_DOTS, j + 1, nodes * 4.0 * (j + 2));
          launch_dots(Vn, K.V, vs, j + 1, n, B, K.partial, K.h, K.act, s);
        }
        HIP_TRY(c, hipMemcpyAsync(hbuf.data(), K.h, (size_t)B * LD * 8, hipMemcpyDeviceToHost, s));
        {
          Prof p(c, MGCNN_K_KRYLOV_ORTH, j + 1, nodes * 4.0 * (j + 3));
          launch_orth_update(Vn, K.V, vs, j + 1, n, B, K.h, K.act, s);
        }
        HIP_TRY(c, hipStreamSynchronize(s));
        for (int b = 0; b < B; ++b)
          if (live[b])
            for (int i = 0; i <= j; ++i) Hij(b, i, j) += hbuf[(size_t)b * LD + i];
      }
      {
        Prof p(c, MGCNN_K_KRYLOV_DOTS, 1, nodes * 4.0);
        launch_dots(Vn, Vn, vs, 1, n, B, K.partial, K.h, K.act, s);
      }
      LAUNCH_CHECK(c);
      HIP_TRY(c, hipMemcpyAsync(hbuf.data(), K.h, (size_t)B * LD * 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipStreamSynchronize(s));
      bool more = false;
      for (int b = 0; b < B; ++b) {
        if (!live[b]) continue;
        const double hn = std::sqrt(std::max(hbuf[(size_t)b * LD], 0.0));
        Hij(b, j + 1, j) = hn;
        sc[b] = hn > 0.0 ? 1.0 / hn : 0.0;
        // Givens rotations: previous ones on column j, then a new one for (j, j+1)
        for (int i = 0; i < j; ++i) {
          const double c0 = cs[(size_t)b * LD + i], s0 = sn[(size_t)b * LD + i];
          const double h0 = Hij(b, i, j), h1 = Hij(b, i + 1, j);
          Hij(b, i, j) = c0 * h0 + s0 * h1;
          Hij(b, i + 1, j) = -s0 * h0 + c0 * h1;
        }
        const double h0 = Hij(b, j, j), h1 = Hij(b, j + 1, j);
        const double rr = std::hypot(h0, h1);
        const double c0 = rr > 0.0 ? h0 / rr : 1.0, s0 = rr > 0.0 ? h1 / rr : 0.0;
        cs[(size_t)b * LD + j] = c0; sn[(size_t)b * LD + j] = s0;
        Hij(b, j, j) = rr; Hij(b, j + 1, j) = 0.0;
        const double gj = g[(size_t)b * LD + j];
        g[(size_t)b * LD + j] = c0 * gj;
        g[(size_t)b * LD + j + 1] = -s0 * gj;
        iters[b] += 1;
        kb[b] = j + 1;
        const double est = std::fabs(g[(size_t)b * LD + j + 1]) / std::sqrt(nf2[b]);
        if (est <= tol || iters[b] >= maxit || hn == 0.0 || !std::isfinite(est)) live[b] = 0;
        else more = true;
      }
      if (!more || j == m - 1) break;
      HIP_TRY(c, hipMemcpyAsync(K.h, sc.data(), (size_t)B * 8, hipMemcpyHostToDevice, s));
      {
        Prof p(c, MGCNN_K_KRYLOV_SCALE, 0, nodes * 8.0);
        launch_scale(Vn, n, B, K.h, K.act, s);
      }
      HIP_TRY(c, hipMemcpyAsync(K.act, live.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
    }
    // y = R^-1 g (upper triangular, k_b x k_b) and u += Z y
    std::fill(ybuf.begin(), ybuf.end(), 0.0);
    for (int b = 0; b < B; ++b) {
      if (!cyc[b]) continue;
      const int k = kb[b];
      for (int i = k - 1; i >= 0; --i) {
        double acc = g[(size_t)b * LD + i];
        for (int l = i + 1; l < k; ++l) acc -= Hij(b, i, l) * ybuf[(size_t)b * LD + l];
        ybuf[(size_t)b * LD + i] = Hij(b, i, i) != 0.0 ? acc / Hij(b, i, i) : 0.0;
      }
    }
    int kmax = 0;
    for (int b = 0; b < B; ++b) if (cyc[b]) kmax = std::max(kmax, kb[b]);
    HIP_TRY(c, hipMemcpyAsync(K.h, ybuf.data(), (size_t)B * LD * 8, hipMemcpyHostToDevice, s));
    {
      Prof p(c, MGCNN_K_KRYLOV_COMBINE, kmax, nodes * (4.0 * kmax + 2.0 * (u64 ? 8 : 4)));
      launch_combine(u, u64, K.Z, vs, kmax, n, B, K.h, K.cyc, s);
    }
    LAUNCH_CHECK(c);
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
