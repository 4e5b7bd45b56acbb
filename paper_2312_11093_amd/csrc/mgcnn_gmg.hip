// Host side of the geometric multigrid preconditioner (Sec. 2.3, Alg. 1 as a V-cycle; the
// GMG settings of Sec. 4.1): hierarchy set-up and one cycle per call, in the same calling
// convention as the network's V-cycle so that the stationary and FGMRES drivers use either.
#include <algorithm>

#include "mgcnn_ctx.h"
#include "mgcnn_gmg.h"

namespace mg {
namespace api {

int gmg_levels_for(const mgcnn_ctx* c, int n) {
  int k = 0;
  while ((1 << k) - 1 < n) ++k;                  // log2(n + 1)
  const int lo = std::max(1, k - 3);             // coarsest side (n+1)/2^(L-1) - 1 <= 15
  const int L = c->opts.gmg_levels == 0 ? lo : c->opts.gmg_levels;
  return (L >= lo && L <= k) ? L : 0;
}

void gmg_free(mgcnn_ctx* c) {
  auto& G = c->gmg;
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  for (auto* v : {&G.a, &G.rhs, &G.pre, &G.cor})
    for (float* p : *v) fr(p);
  G.a.clear(); G.rhs.clear(); G.pre.clear(); G.cor.clear();
  fr(G.inv);
  G.inv = nullptr;
  G.levels = 0;
  G.nl.clear();
}

int gmg_alloc(mgcnn_ctx* c, int n, int B) {
  auto& G = c->gmg;
  const int L = gmg_levels_for(c, n);
  if (L == 0) return fail(c, MGCNN_E_ARG, "setup: gmg_levels out of range for this n");
  G.levels = L;
  G.nl.assign(L, 0);
  for (int l = 0, m = n; l < L; ++l, m = (m - 1) / 2) G.nl[l] = m;
  G.a.assign(L, nullptr); G.rhs.assign(L, nullptr); G.pre.assign(L, nullptr); G.cor.assign(L, nullptr);
  int r;
  for (int l = 0; l < L; ++l) {
    const size_t bytes = (size_t)G.nl[l] * G.nl[l] * B * 4;
    if (l >= 1) {
      if ((r = alloc(c, (void**)&G.a[l], bytes))) return r;
      if ((r = alloc(c, (void**)&G.rhs[l], bytes))) return r;
      if ((r = alloc(c, (void**)&G.cor[l], bytes))) return r;
    }
    if (l + 1 < L && (r = alloc(c, (void**)&G.pre[l], bytes))) return r;
  }
  const size_t N = (size_t)G.nl[L - 1] * G.nl[L - 1];
  return alloc(c, (void**)&G.inv, N * N * B * 8);
}

int gmg_setup(mgcnn_ctx* c) {
  auto& G = c->gmg;
  const int L = G.levels, B = c->B;
  hipStream_t s = c->stream;
  for (int l = 1; l < L; ++l)
    launch_gmg_inject(l == 1 ? c->d_a : G.a[l - 1], G.a[l], G.nl[l - 1], B, s);
  launch_gmg_coarse_inverse(L == 1 ? c->d_a : G.a[L - 1], c->d_b, G.inv, G.nl[L - 1], B, c->form(),
                            s);
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

// One V-cycle on the problems of `list` (count of them): the right-hand side is c->d_rt = r / D
// on the finest level; the correction is stored into (or added to) u.
int gmg_cycle(mgcnn_ctx* c, void* u, bool u_f64, const int* list, int count, bool accumulate,
              const int* flags) {
  auto& G = c->gmg;
  const int L = G.levels, B = count, nu = c->opts.gmg_sweeps;
  const float omega = c->opts.gmg_omega;
  hipStream_t s = c->stream;
  const int mode = u_f64 ? (accumulate ? GMG_OUT_F64_ADD : GMG_OUT_F64)
                         : (accumulate ? GMG_OUT_F32_ADD : GMG_OUT_F32);
  const double ub = (u_f64 ? 8.0 : 4.0) * (accumulate ? 2.0 : 1.0);   // bytes of u per node
  auto A = [&](int l) -> const float* { return l == 0 ? c->d_a : G.a[l]; };
  auto R = [&](int l) -> const float* { return l == 0 ? c->d_rt : G.rhs[l]; };
  auto nodes = [&](int l) { return (double)G.nl[l] * G.nl[l] * B; };
  // algorithmic flops per node: 12 per sweep (five products, five sums, the weighting), 12 for
  // the residual, 17/4 per fine node for the full weighting, 4 per fine node for the bilinear
  // interpolation
  const int mcL = G.nl[L - 1];
  const double Nc = (double)mcL * mcL;
  auto coarse = [&](const float* rhs, bool scaled, void* out, int md, const int* fl, double outb) {
    Prof p(c, MGCNN_K_GMG_COARSE, L - 1, B * (Nc * Nc * 8.0 + Nc * (4.0 + outb)), B * Nc * Nc * 2.0);
    launch_gmg_coarse_solve(G.inv, A(L - 1), c->d_b, rhs, scaled, out, md, fl, mcL, B, list,
                            c->form(), s);
  };
  if (L == 1) {
    coarse(c->d_rt, true, u, mode, flags, ub);
    LAUNCH_CHECK(c);
    return MGCNN_OK;
  }
  for (int l = 0; l + 1 < L; ++l) {
    Prof p(c, MGCNN_K_GMG_DOWN, l, nodes(l) * 12.0 + nodes(l + 1) * 4.0,
           nodes(l) * (12.0 * nu + 12.0 + 17.0 / 4.0));
    launch_gmg_down(nu, A(l), c->d_b, R(l), l == 0, omega, G.pre[l], G.rhs[l + 1], G.nl[l], B,
                    list, c->form(), s);
  }
  coarse(G.rhs[L - 1], false, G.cor[L - 1], GMG_OUT_F32, nullptr, 4.0);
  for (int l = L - 2; l >= 0; --l) {
    const bool fin = l == 0;
    Prof p(c, MGCNN_K_GMG_UP, l, nodes(l) * (12.0 + (fin ? ub : 4.0)) + nodes(l + 1) * 4.0,
           nodes(l) * (12.0 * nu + 4.0));
    launch_gmg_up(nu, A(l), c->d_b, R(l), fin, omega, G.pre[l], G.cor[l + 1],
                  fin ? u : (void*)G.cor[l], fin ? mode : GMG_OUT_F32, fin ? flags : nullptr,
                  G.nl[l], B, list, c->form(), s);
  }
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

}  // namespace api
}  // namespace mg
