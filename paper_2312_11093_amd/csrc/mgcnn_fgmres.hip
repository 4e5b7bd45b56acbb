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
#include <thread>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_ctx.h"
#include "mgcnn_internal.h"
#include "mgcnn_krylov.h"

using namespace mg;
using namespace mg::api;

namespace mg {

namespace api {

void free_krylov(mgcnn_ctx* c) {
  auto& K = c->kr;
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(K.V); fr(K.Z); fr(K.partial); fr(K.h); fr(K.s); fr(K.act); fr(K.cyc); fr(K.grp); fr(K.coef);
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
  if ((r = alloc(c, (void**)&K.grp, (size_t)c->B * 4))) return r;
  // deflation coefficients: V and Z combinations, (KRYLOV_MAX_BASIS + 1) x KRYLOV_MAX_DEFLATE each
  if ((r = alloc(c, (void**)&K.coef, (size_t)c->B * 2 * (KRYLOV_MAX_BASIS + 1) * KRYLOV_MAX_DEFLATE * 8)))
    return r;
  K.n = c->n; K.B = c->B; K.m = m;
  return MGCNN_OK;
}

// Deflation at restart: the kd right singular vectors of the cycle's (k+1) x k Hessenberg matrix
// Hb with the smallest singular values -- eigenvectors of Hb^T Hb by cyclic Jacobi rotations in
// f64 -- as the columns of P (k x kd, row-major): Z P spans the directions in which the
// preconditioned operator of the cycle is smallest.  Returns false if the cycle is too short.
static bool smallest_singular_directions(const double* Hraw, int ldh, int k, int kd, double* P) {
  if (k < kd + 1) return false;
  std::vector<double> G((size_t)k * k, 0.0), E((size_t)k * k, 0.0);
  for (int a = 0; a < k; ++a)
    for (int b = 0; b <= a; ++b) {
      double acc = 0.0;
      for (int i = 0; i <= k; ++i) acc += Hraw[(size_t)i * ldh + a] * Hraw[(size_t)i * ldh + b];
      G[(size_t)a * k + b] = G[(size_t)b * k + a] = acc;
    }
  for (int a = 0; a < k; ++a) E[(size_t)a * k + a] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int a = 0; a < k; ++a) {
      diag += G[(size_t)a * k + a] * G[(size_t)a * k + a];
      for (int b = a + 1; b < k; ++b) off += G[(size_t)a * k + b] * G[(size_t)a * k + b];
    }
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = G[(size_t)p * k + q];
        if (std::fabs(apq) <= 1e-300) continue;
        const double theta = (G[(size_t)q * k + q] - G[(size_t)p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cth = 1.0 / std::sqrt(t * t + 1.0), sth = t * cth;
        for (int i = 0; i < k; ++i) {   // columns p, q
          const double gip = G[(size_t)i * k + p], giq = G[(size_t)i * k + q];
          G[(size_t)i * k + p] = cth * gip - sth * giq;
          G[(size_t)i * k + q] = sth * gip + cth * giq;
        }
        for (int i = 0; i < k; ++i) {   // rows p, q
          const double gpi = G[(size_t)p * k + i], gqi = G[(size_t)q * k + i];
          G[(size_t)p * k + i] = cth * gpi - sth * gqi;
          G[(size_t)q * k + i] = sth * gpi + cth * gqi;
        }
        for (int i = 0; i < k; ++i) {
          const double eip = E[(size_t)i * k + p], eiq = E[(size_t)i * k + q];
          E[(size_t)i * k + p] = cth * eip - sth * eiq;
          E[(size_t)i * k + q] = sth * eip + cth * eiq;
        }
      }
  }
  std::vector<int> order(k);
  for (int a = 0; a < k; ++a) order[a] = a;
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return G[(size_t)x * k + x] < G[(size_t)y * k + y]; });
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < kd; ++i) P[(size_t)j * kd + i] = E[(size_t)j * k + order[i]];
  return true;
}

// Restarted FGMRES(m), right preconditioned by z = B(v / D), one Arnoldi process per problem,
// optionally with deflated restarting (opts.deflate = kd: see smallest_singular_directions and
// the restart step at the end of a cycle).
// Orthogonalisation: classical Gram-Schmidt, once or twice.  The small least-squares problems
// (Givens rotations) run on the host in f64.  Every launch covers a compact list of the
// problems still extending their basis; a problem that restarts with deflation vectors joins
// the Arnoldi loop at step kd.
int fgmres_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
                 double* relres_host, int* status_host) {
  const int m = std::max(1, std::min(c->opts.restart > 0 ? c->opts.restart : 30, KRYLOV_MAX_BASIS - 1));
  const int kd = std::max(0, std::min(c->opts.deflate, m - 1));
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
  std::vector<double> H((size_t)B * (HL + 1) * HL), Hr((size_t)B * (HL + 1) * HL),
      g((size_t)B * HL + B), cs((size_t)B * HL), sn((size_t)B * HL), hb((size_t)B * LD),
      hb2((size_t)B * LD), hb3((size_t)B * LD), sc((size_t)B * LD, 0.0), nw2(B, 0.0);
  // deflation: per problem R (kd x kd, A Z_new = V_new R) and the combination coefficients of Z
  const size_t cstride = (size_t)(HL + 1) * KRYLOV_MAX_DEFLATE;
  std::vector<double> Rk((size_t)B * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE),
      coefZ((size_t)B * cstride, 0.0);
  std::vector<int> kb(B), start(B, 0), dgrp(B, 0), list_live(B), list_cyc(B), list_grp(B);
  auto Hij = [&](int b, int i, int j) -> double& { return H[((size_t)b * (HL + 1) + i) * HL + j]; };
  auto Hrij = [&](int b, int i, int j) -> double& { return Hr[((size_t)b * (HL + 1) + i) * HL + j]; };
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
  auto Vw = [&](int j) { return K.V + (size_t)j * vs; };
  while (true) {
    // true residual of every live problem, its norm, and the stopping rule.  Problems that
    // restart plainly put it in slot 0; problems that carry kd deflation vectors (slots
    // 0..kd-1) put it in slot kd and orthogonalise it against them.
    std::vector<int> plain(B, 0), defl(B, 0);
    for (int b = 0; b < B; ++b) {
      plain[b] = act[b] && !dgrp[b];
      defl[b] = act[b] && dgrp[b];
    }
    int nplain = 0, ndefl = 0;
    HIP_TRY(c, to_list(K.act, list_live, plain, nplain));
    HIP_TRY(c, to_list(K.grp, list_grp, defl, ndefl));
    if (nplain + ndefl == 0) break;
    if (nplain) {
      Prof p(c, MGCNN_K_KRYLOV_RESIDUAL, 0, nodes1 * nplain * (12.0 + (u64 ? 8 : 4)));
      launch_krylov_residual(c->d_a, c->d_b, f, u, u64, Vw(0), krylov_vpad(n), n, nplain, K.act,
                             c->form(), s);
    }
    if (ndefl) {
      Prof p(c, MGCNN_K_KRYLOV_RESIDUAL, 0, nodes1 * ndefl * (12.0 + (u64 ? 8 : 4)));
      launch_krylov_residual(c->d_a, c->d_b, f, u, u64, Vw(kd), krylov_vpad(n), n, ndefl, K.grp,
                             c->form(), s);
    }
    if (nplain) {
      Prof p(c, MGCNN_K_KRYLOV_DOTS, 0, nodes1 * nplain * 4.0);
      launch_gs_pass(0, Vw(0), K.V, vs, 0, n, nplain, nullptr, K.partial, K.h, K.act, s);
    }
    if (ndefl) {
      Prof p(c, MGCNN_K_KRYLOV_DOTS, kd, nodes1 * ndefl * 4.0 * (kd + 1));
      launch_gs_pass(0, Vw(kd), K.V, vs, kd, n, ndefl, nullptr, K.partial, K.h, K.grp, s);
    }
    LAUNCH_CHECK(c);
    HIP_TRY(c, from_dev(hb));
    if (ndefl) {
      Prof p(c, MGCNN_K_KRYLOV_ORTH, kd, nodes1 * ndefl * 4.0 * (kd + 2));
      launch_gs_pass(2, Vw(kd), K.V, vs, kd, n, ndefl, K.h, K.partial, K.h, K.grp, s);
      LAUNCH_CHECK(c);
      HIP_TRY(c, from_dev(hb3));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->prof && (r = prof_drain(c))) return r;
    bool any = false;
    std::vector<int> live(B, 0);
    for (int b = 0; b < B; ++b) {
      cyc[b] = 0;
      if (!act[b]) continue;
      const double* hrow = &hb[(size_t)b * LD];
      const double beta = std::sqrt(std::max(hrow[dgrp[b] ? kd : 0], 0.0));
      const double rho = beta / std::sqrt(nf2[b]);
      relres[b] = rho;
      if (rho <= tol) { status[b] = MGCNN_OK; act[b] = 0; }
      else if (iters[b] >= maxit) { status[b] = MGCNN_NOT_CONVERGED; act[b] = 0; }
      else if (!(rho <= 1e10)) { status[b] = MGCNN_E_DIVERGED; act[b] = 0; }
      else {
        cyc[b] = 1;
        any = true;
        for (int i = 0; i <= HL; ++i) gi(b, i) = 0.0;
        std::fill(&Hij(b, 0, 0), &Hij(b, 0, 0) + (size_t)(HL + 1) * HL, 0.0);
        std::fill(&Hrij(b, 0, 0), &Hrij(b, 0, 0) + (size_t)(HL + 1) * HL, 0.0);
        if (!dgrp[b]) {
          sc[(size_t)b * LD] = 1.0 / beta;
          gi(b, 0) = beta;
          start[b] = 0;
          kb[b] = 0;
          live[b] = 1;
        } else {
          // columns 0..kd-1: A Z_i = V R e_i, already upper triangular (no rotation); the
          // residual is V_0..V_{kd-1} c + |r_perp| v_kd
          const double rp = std::sqrt(std::max(hb3[(size_t)b * LD], 0.0));
          const double* R = &Rk[(size_t)b * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE];
          for (int j = 0; j < kd; ++j) {
            for (int i = 0; i <= j; ++i) Hij(b, i, j) = Hrij(b, i, j) = R[(size_t)i * kd + j];
            cs[(size_t)b * HL + j] = 1.0;
            sn[(size_t)b * HL + j] = 0.0;
            gi(b, j) = hrow[j];
          }
          gi(b, kd) = rp;
          start[b] = kd;
          kb[b] = kd;
          if (rp > 0.0) {
            sc[(size_t)b * LD] = 1.0 / rp;
            live[b] = 1;
          }
        }
      }
    }
    if (!any) break;
    int ncyc = 0, nlive = 0;
    HIP_TRY(c, to_list(K.cyc, list_cyc, cyc, ncyc));
    int jfirst = m;
    for (int b = 0; b < B; ++b)
      if (live[b]) jfirst = std::min(jfirst, start[b]);
    for (int j = jfirst; j < m; ++j) {
      // problems in the Arnoldi loop at step j
      std::vector<int> step(B, 0);
      bool more = false;
      for (int b = 0; b < B; ++b) {
        step[b] = live[b] && start[b] <= j;
        more |= live[b] != 0;
      }
      if (!more) break;
      HIP_TRY(c, to_list(K.act, list_live, step, nlive));
      if (nlive == 0) continue;
      float* Vj = Vw(j);
      float* Vn = Vw(j + 1);
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
        if (!step[b]) continue;
        for (int i = 0; i < cnt; ++i)
          Hij(b, i, j) = Hrij(b, i, j) =
              hb[(size_t)b * LD + i] + (two_pass ? hb2[(size_t)b * LD + i] : 0.0);
        nw2[b] = hb3[(size_t)b * LD];
      }
      if (c->prof && (r = prof_drain(c))) return r;   // the stream is idle here
      for (int b = 0; b < B; ++b) {
        if (!step[b]) continue;
        const double hn = std::sqrt(std::max(nw2[b], 0.0));
        Hij(b, j + 1, j) = Hrij(b, j + 1, j) = hn;
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
      }
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
    // deflated restart: the next cycle's first kd preconditioned vectors Z P, their images
    // A Z P recomputed and orthonormalised (Gram-Schmidt twice) into V_0..V_{kd-1} with R, so
    // that A Z_new = V_new R holds to one rounding (a relation carried over from cycle to cycle
    // would accumulate the float32 roundings, amplified by the small singular values kept)
    std::fill(dgrp.begin(), dgrp.end(), 0);
    if (kd > 0) {
      std::vector<int> todo;
      for (int b = 0; b < B; ++b)
        if (cyc[b] && kb[b] >= kd + 1) todo.push_back(b);
      std::vector<int> ok(B, 0);
      auto work = [&](size_t first, size_t step) {
        for (size_t t = first; t < todo.size(); t += step) {
          const int b = todo[t];
          double* cZ = &coefZ[(size_t)b * cstride];
          std::fill(cZ, cZ + cstride, 0.0);
          ok[b] = smallest_singular_directions(&Hrij(b, 0, 0), HL, kb[b], kd, cZ);
          cZ[cstride - 1] = kb[b];      // the combination reads Z_0..Z_{kb-1}
        }
      };
      const size_t nth = std::min<size_t>(
          todo.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
      std::vector<std::thread> pool;
      for (size_t t = 1; t < nth; ++t) pool.emplace_back(work, t, nth);
      if (nth > 0) work(0, nth);
      for (auto& th : pool) th.join();
      int cmax = 0;
      for (int b : todo)
        if (ok[b]) { dgrp[b] = 1; cmax = std::max(cmax, kb[b]); }
      int nd = 0;
      HIP_TRY(c, to_list(K.grp, list_grp, dgrp, nd));
      if (nd > 0) {
        HIP_TRY(c, hipMemcpyAsync(K.coef, coefZ.data(), coefZ.size() * 8, hipMemcpyHostToDevice, s));
        {
          Prof p(c, MGCNN_K_KRYLOV_COMBINE, kd, nodes1 * nd * 4.0 * (cmax + kd));
          launch_basis_combine(K.Z, zs, (size_t)n * n, cmax, kd, K.coef, cstride, nd, K.grp, s);
        }
        std::vector<double> Rd((size_t)B * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE, 0.0);
        for (int i = 0; i < kd; ++i) {
          float* Vi = Vw(i);
          {
            Prof p(c, MGCNN_K_KRYLOV_APPLY_A, 0, nodes1 * nd * 12.0);
            launch_apply_A(c->d_a, c->d_b, K.Z + (size_t)i * zs, Vi, krylov_vpad(n), n, nd, K.grp,
                           c->form(), s);
          }
          launch_gs_pass(0, Vi, K.V, vs, i, n, nd, nullptr, K.partial, K.h, K.grp, s);
          HIP_TRY(c, from_dev(hb));
          if (i > 0) {
            launch_gs_pass(1, Vi, K.V, vs, i, n, nd, K.h, K.partial, K.h, K.grp, s);
            HIP_TRY(c, from_dev(hb2));
            launch_gs_pass(2, Vi, K.V, vs, i, n, nd, K.h, K.partial, K.h, K.grp, s);
            HIP_TRY(c, from_dev(hb3));
          }
          LAUNCH_CHECK(c);
          HIP_TRY(c, hipStreamSynchronize(s));
          for (int b = 0; b < B; ++b) {
            if (!dgrp[b]) continue;
            double* R = &Rd[(size_t)b * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE];
            const double raw2 = hb[(size_t)b * LD + i];               // |A z_i|^2 (slot cnt = i)
            const double nrm2 = i > 0 ? hb3[(size_t)b * LD] : raw2;
            for (int l = 0; l < i; ++l)
              R[(size_t)l * kd + i] = hb[(size_t)b * LD + l] + hb2[(size_t)b * LD + l];
            const double nrm = std::sqrt(std::max(nrm2, 0.0));
            // a direction (numerically) inside the span of the previous ones: no deflation
            if (!(nrm > 1e-7 * std::sqrt(std::max(raw2, 0.0)))) { dgrp[b] = 0; continue; }
            R[(size_t)i * kd + i] = nrm;
            sc[(size_t)b * LD] = 1.0 / nrm;
          }
          HIP_TRY(c, hipMemcpyAsync(K.s, sc.data(), (size_t)B * LD * 8, hipMemcpyHostToDevice, s));
          launch_normalize_diag(c->d_a, c->d_b, Vi, c->d_rt, K.s, n, nd, K.grp, c->form(), s);
          LAUNCH_CHECK(c);
        }
        for (int b = 0; b < B; ++b)
          if (dgrp[b])
            std::copy(&Rd[(size_t)b * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE],
                      &Rd[(size_t)(b + 1) * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE],
                      &Rk[(size_t)b * KRYLOV_MAX_DEFLATE * KRYLOV_MAX_DEFLATE]);
      }
    }
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
