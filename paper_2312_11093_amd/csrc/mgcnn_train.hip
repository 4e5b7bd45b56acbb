// Training entry points: recorded forward, residual loss and the hand-written reverse pass
// through K unrolled iterations and the setup network (loss of Sec. 3.4, Eq. (19), taken
// after K iterations and normalised per problem; setup and solve networks trained jointly).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_adjoint.h"
#include "mgcnn_ctx.h"
#include "mgcnn_internal.h"

using namespace mg;
using namespace mg::api;

namespace mg {
namespace api {

void free_train(mgcnn_ctx* c) {
  auto& T = c->tr;
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(T.uk);
  for (auto* v : {&T.xin, &T.xdn, &T.v, &T.xup, &T.g1, &T.g2, &T.gs, &T.c, &T.gc, &T.z, &T.t})
    for (float* p : *v) fr(p);
  for (auto* v : {&T.xin, &T.xdn, &T.v, &T.xup, &T.g1, &T.g2, &T.gs, &T.c, &T.gc, &T.z, &T.t}) v->clear();
  fr(T.F); fr(T.gz0); fr(T.gz1); fr(T.grt); fr(T.lam0); fr(T.lam1); fr(T.r); fr(T.grad);
  fr(T.partial); fr(T.d_loss); fr(T.d_rr);
  T = mgcnn_ctx::Train{};
}

static int ensure_train(mgcnn_ctx* c, int K) {
  auto& T = c->tr;
  if (T.alloc_n == c->n && T.alloc_B == c->B && T.alloc_K >= K) return MGCNN_OK;
  free_train(c);
  const int n = c->n, B = c->B, L = c->L;
  const size_t nn = (size_t)n * n * B;
  int r;
  auto A = [&](float** p, size_t floats) { return alloc(c, (void**)p, floats * 4); };
  if ((r = A(&T.uk, nn * std::max(K, 1)))) return r;
  for (auto* v : {&T.xin, &T.xdn, &T.v, &T.xup, &T.g1, &T.g2, &T.gs, &T.c, &T.gc}) v->assign(L, nullptr);
  T.z.assign(L * NUM_SETUP_LAYERS, nullptr);
  T.t.assign(L * NUM_SETUP_LAYERS, nullptr);
  for (int l = 0; l < L; ++l) {
    const size_t cnt = (size_t)c->nl[l] * c->nl[l] * B * C;
    for (auto* v : {&T.xin, &T.xdn, &T.v, &T.xup, &T.g1, &T.g2, &T.gs, &T.c, &T.gc})
      if ((r = A(&(*v)[l], cnt))) return r;
    for (int k = 0; k < NUM_SETUP_LAYERS; ++k) {
      if ((r = A(&T.z[l * NUM_SETUP_LAYERS + k], cnt))) return r;
      if ((r = A(&T.t[l * NUM_SETUP_LAYERS + k], cnt))) return r;
    }
  }
  if ((r = A(&T.F, nn * 4))) return r;
  if ((r = A(&T.gz0, nn * C))) return r;
  if ((r = A(&T.gz1, nn * C))) return r;
  if ((r = A(&T.grt, nn))) return r;
  if ((r = A(&T.lam0, nn))) return r;
  if ((r = A(&T.lam1, nn))) return r;
  if ((r = A(&T.r, nn))) return r;
  if ((r = A(&T.grad, c->off.total))) return r;
  // largest partial table: same-size 16x16 weight gradient at the finest level
  const size_t blocks = (size_t)((n + 63) / 64) * ((n + 3) / 4) * B;
  const size_t blocks_s2 = (size_t)((n + 31) / 32) * ((n + 3) / 4) * B;
  T.partial_floats = std::max(blocks, blocks_s2) * C * C * 9;
  if ((r = A(&T.partial, T.partial_floats))) return r;
  if ((r = alloc(c, (void**)&T.d_loss, 8))) return r;
  if ((r = alloc(c, (void**)&T.d_rr, (size_t)B * 8))) return r;
  T.alloc_n = n; T.alloc_B = B; T.alloc_K = K;
  return MGCNN_OK;
}

int forward_record(mgcnn_ctx* c, const float* f, float* u, int K) {
  if (c->st() == ST_BF16 || c->s16() || c->u64())
    return fail(c, MGCNN_E_ARG, "forward(record): needs f32 state and f32 u");
  if (c->opts.up_post) return fail(c, MGCNN_E_ARG, "forward(record): no reverse pass for up_post");
  int r = ensure_train(c, K);
  if (r) return r;
  auto& T = c->tr;
  const size_t nn = (size_t)c->n * c->n * c->B;
  for (int k = 0; k < K; ++k) {
    HIP_TRY(c, hipMemcpyAsync(T.uk + (size_t)k * nn, u, nn * 4, hipMemcpyDeviceToDevice, c->stream));
    launch_residual(c->d_a, c->d_b, f, u, false, c->d_rt, c->d_partial, c->n, c->B, nullptr,
                    c->form(), c->stream);
    if ((r = vcycle(c, u, false, nullptr, c->B))) return r;
  }
  T.K = K;
  T.f = f;
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

// weight gradient of one conv into grad[off : off + ne], accumulated
static void wgrad_acc(mgcnn_ctx* c, WgradArgs G, size_t off, int ne) {
  G.partial = c->tr.partial;
  const int nb = launch_wgrad(G, c->B, c->stream);
  launch_reduce_partials(c->tr.partial, nb, ne, c->tr.grad + off, true, c->stream);
}

static ConvArgs conv_args(const float* x, const float* W, float* y, int mi, int mo, int ci, int co,
                          int gm, int ep, int trans, int flip) {
  ConvArgs A;
  A.x = x; A.W = W; A.y = y; A.mi = mi; A.mo = mo; A.ci = ci; A.co = co; A.gm = gm; A.ep = ep;
  A.trans = trans; A.flip = flip;
  return A;
}

// Recompute the activations of one V-cycle (Alg. 3) from c->d_rt into separate buffers.
static void recompute_vcycle(mgcnn_ctx* c) {
  auto& T = c->tr;
  const int L = c->L, B = c->B;
  hipStream_t s = c->stream;
  launch_conv_in(1, c->d_rt, c->W(c->off.solve_in), T.xin[0], ST_F32, c->n, B, nullptr, s);
  for (int l = 0; l < L; ++l) {
    launch_conv16(CM_SMOOTH, ST_F32, T.xin[l], c->s[l], c->W(c->off.smooth_down), nullptr, T.xdn[l],
                  c->nl[l], B, nullptr, s);
    if (l < L - 1)
      launch_conv16(CM_RESTRICT, ST_F32, T.xdn[l], nullptr, c->W(c->off.restrict_), nullptr,
                    T.xin[l + 1], c->nl[l], B, nullptr, s);
  }
  const size_t cL = (size_t)c->nl[L - 1] * c->nl[L - 1] * B * C * 4;
  (void)hipMemcpyAsync(T.v[L - 1], T.xdn[L - 1], cL, hipMemcpyDeviceToDevice, s);
  for (int l = L - 1; l >= 0; --l) {
    launch_conv16(CM_SMOOTH, ST_F32, T.v[l], c->s[l], c->W(c->off.smooth_up), nullptr, T.xup[l],
                  c->nl[l], B, nullptr, s);
    if (l > 0) {
      const size_t cnt = (size_t)c->nl[l - 1] * c->nl[l - 1] * B * C * 4;
      (void)hipMemcpyAsync(T.v[l - 1], T.xdn[l - 1], cnt, hipMemcpyDeviceToDevice, s);
      launch_prolong_add(ST_F32, T.xup[l], c->W(c->off.prolong), T.v[l - 1], c->nl[l], B, nullptr, s);
    }
  }
}

// Reverse of one V-cycle: lam (dL/d output, [B][n][n]) -> grt (dL/d rt); accumulates weight
// gradients and dL/ds_l (into T.gs).
static void vcycle_reverse(mgcnn_ctx* c, const float* lam) {
  auto& T = c->tr;
  const int L = c->L, B = c->B, n = c->n;
  hipStream_t s = c->stream;
  const auto& o = c->off;
  // reChannel-out: out = W_out * xup0 (16 -> 1)
  {
    WgradArgs G; G.A = lam; G.Bx = T.xup[0]; G.ma = n; G.mb = n; G.ca = 1; G.cb = C; G.gm = GM_SAME;
    wgrad_acc(c, G, o.solve_out, C * 9);
    launch_dconv(conv_args(lam, c->W(o.solve_out), T.g1[0], n, n, 1, C, GM_SAME, EP_STORE, 1, 1), B, s);
  }
  // up cycle, reversed: l = 0 .. L-1;  g1[l] = dL/dxup[l]
  for (int l = 0; l < L; ++l) {
    const int m = c->nl[l];
    {
      WgradArgs G; G.A = T.g1[l]; G.Bx = T.v[l]; G.Bm = (const float*)c->s[l]; G.ma = m; G.mb = m;
      G.ca = C; G.cb = C; G.gm = GM_SAME; G.pmb = PM_MUL;
      wgrad_acc(c, G, o.smooth_up, C * C * 9);
    }
    {
      ConvArgs A = conv_args(T.g1[l], c->W(o.smooth_up), T.g2[l], m, m, C, C, GM_SAME, EP_SMOOTH_BWD, 1, 1);
      A.skip = T.g1[l]; A.m2 = (const float*)c->s[l]; A.m3 = T.v[l]; A.gs = T.gs[l];
      launch_dconv(A, B, s);      // g2[l] = dL/dv[l] (= dL/dxdn[l] from the up side)
    }
    if (l < L - 1) {
      const int mc = c->nl[l + 1];
      WgradArgs G; G.A = T.xup[l + 1]; G.Bx = T.g2[l]; G.ma = mc; G.mb = m; G.ca = C; G.cb = C; G.gm = GM_S2;
      wgrad_acc(c, G, o.prolong, C * C * 9);
      launch_dconv(conv_args(T.g2[l], c->W(o.prolong), T.g1[l + 1], m, mc, C, C, GM_S2, EP_STORE, 0, 0), B, s);
    }
  }
  // down cycle, reversed: l = L-1 .. 0;  g2[l] = dL/dxdn[l] (complete when reached)
  for (int l = L - 1; l >= 0; --l) {
    const int m = c->nl[l];
    {
      WgradArgs G; G.A = T.g2[l]; G.Bx = T.xin[l]; G.Bm = (const float*)c->s[l]; G.ma = m; G.mb = m;
      G.ca = C; G.cb = C; G.gm = GM_SAME; G.pmb = PM_MUL;
      wgrad_acc(c, G, o.smooth_down, C * C * 9);
    }
    {
      ConvArgs A = conv_args(T.g2[l], c->W(o.smooth_down), T.g1[l], m, m, C, C, GM_SAME, EP_SMOOTH_BWD, 1, 1);
      A.skip = T.g2[l]; A.m2 = (const float*)c->s[l]; A.m3 = T.xin[l]; A.gs = T.gs[l];
      launch_dconv(A, B, s);      // g1[l] = dL/dxin[l]
    }
    if (l > 0) {
      const int mf = c->nl[l - 1];
      WgradArgs G; G.A = T.g1[l]; G.Bx = T.xdn[l - 1]; G.ma = m; G.mb = mf; G.ca = C; G.cb = C; G.gm = GM_S2;
      wgrad_acc(c, G, o.restrict_, C * C * 9);
      launch_dconv(conv_args(T.g1[l], c->W(o.restrict_), T.g2[l - 1], m, mf, C, C, GM_T2, EP_ADD, 1, 0), B, s);
    }
  }
  // reChannel-in: x1 = W_in * rt (1 -> 16)
  {
    WgradArgs G; G.A = T.g1[0]; G.Bx = c->d_rt; G.ma = n; G.mb = n; G.ca = C; G.cb = 1; G.gm = GM_SAME;
    wgrad_acc(c, G, o.solve_in, C * 9);
    launch_dconv(conv_args(T.g1[0], c->W(o.solve_in), T.grt, n, n, C, 1, GM_SAME, EP_STORE, 1, 1), B, s);
  }
}

// Recompute the setup tape with the reverse-pass kernels: F, c_l, z_{l,k}, t_{l,k}.
static void recompute_setup(mgcnn_ctx* c) {
  auto& T = c->tr;
  const int L = c->L, B = c->B, n = c->n;
  hipStream_t s = c->stream;
  const auto& o = c->off;
  launch_features(c->d_a, c->d_b, T.F, n, B, c->form(), s);
  launch_dconv(conv_args(T.F, c->W(o.setup_in), T.c[0], n, n, 4, C, GM_SAME, EP_STORE, 0, 0), B, s);
  for (int l = 0; l < L; ++l) {
    const int m = c->nl[l];
    const size_t cnt = (size_t)m * m * B * C;
    const float* zin = T.c[l];
    for (int k = 0; k < NUM_SETUP_LAYERS; ++k) {
      float* zk = T.z[l * NUM_SETUP_LAYERS + k];
      float* tk = T.t[l * NUM_SETUP_LAYERS + k];
      if (zin != zk) (void)hipMemcpyAsync(zk, zin, cnt * 4, hipMemcpyDeviceToDevice, s);
      ConvArgs A = conv_args(zk, c->W(o.res_w[k]), tk, m, m, C, C, GM_SAME, EP_TANH_BIAS, 0, 0);
      A.bias = c->W(o.res_b[k]);
      launch_dconv(A, B, s);
      if (k < NUM_SETUP_LAYERS - 1) {
        float* znext = T.z[l * NUM_SETUP_LAYERS + k + 1];
        launch_add(zk, tk, znext, cnt, s);   // z_{k+1} = z_k + tanh(W_k z_k + beta_k)
        zin = znext;
      }
    }
    if (l < L - 1)
      launch_dconv(conv_args(T.c[l], c->W(o.setup_restrict), T.c[l + 1], m, c->nl[l + 1], C, C, GM_S2,
                             EP_STORE, 0, 0), B, s);
  }
}

static void setup_reverse(mgcnn_ctx* c) {
  auto& T = c->tr;
  const int L = c->L, B = c->B, n = c->n;
  hipStream_t s = c->stream;
  const auto& o = c->off;
  for (int l = 0; l < L; ++l)
    launch_zero(T.gc[l], (size_t)c->nl[l] * c->nl[l] * B * C * 4, s);
  for (int l = L - 1; l >= 0; --l) {
    const int m = c->nl[l];
    const size_t cnt = (size_t)m * m * B * C;
    (void)hipMemcpyAsync(T.gz0, T.gs[l], cnt * 4, hipMemcpyDeviceToDevice, s);
    float* gz = T.gz0;
    float* gn = T.gz1;
    for (int k = NUM_SETUP_LAYERS - 1; k >= 0; --k) {
      const float* zk = T.z[l * NUM_SETUP_LAYERS + k];
      const float* tk = T.t[l * NUM_SETUP_LAYERS + k];
      WgradArgs G; G.A = gz; G.Am = tk; G.Bx = zk; G.ma = m; G.mb = m; G.ca = C; G.cb = C;
      G.gm = GM_SAME; G.pma = PM_TANHD;
      wgrad_acc(c, G, o.res_w[k], C * C * 9);
      const int nb = launch_bias_grad(gz, tk, T.partial, cnt / C, s);
      launch_reduce_partials(T.partial, nb, C, T.grad + o.res_b[k], true, s);
      ConvArgs A = conv_args(gz, c->W(o.res_w[k]), gn, m, m, C, C, GM_SAME, EP_SKIP, 1, 1);
      A.pm = PM_TANHD; A.m = tk; A.skip = gz;
      launch_dconv(A, B, s);
      std::swap(gz, gn);
    }
    launch_add(T.gc[l], gz, T.gc[l], cnt, s);
    if (l > 0) {
      const int mf = c->nl[l - 1];
      WgradArgs G; G.A = T.gc[l]; G.Bx = T.c[l - 1]; G.ma = m; G.mb = mf; G.ca = C; G.cb = C; G.gm = GM_S2;
      wgrad_acc(c, G, o.setup_restrict, C * C * 9);
      launch_dconv(conv_args(T.gc[l], c->W(o.setup_restrict), T.gc[l - 1], m, mf, C, C, GM_T2, EP_ADD, 1, 0), B, s);
    }
  }
  WgradArgs G; G.A = T.gc[0]; G.Bx = T.F; G.ma = n; G.mb = n; G.ca = C; G.cb = 4; G.gm = GM_SAME;
  wgrad_acc(c, G, o.setup_in, C * 4 * 9);
}

}  // namespace api
}  // namespace mg

extern "C" {

int mgcnn_set_weights_device(mgcnn_ctx* c, const float* w_dev) {
  if (!c || !w_dev) return MGCNN_E_ARG;
  if (c->pairs()) return fail(c, MGCNN_E_STATE, "set_weights_device: not with pack_pairs (host weights only)");
  c->tr.K = 0;             // a recorded forward was taken with the previous weights
  c->tr.f = nullptr;
  HIP_TRY(c, hipMemcpyAsync(c->d_w, w_dev, c->off.total * 4, hipMemcpyDeviceToDevice, c->stream));
  return MGCNN_OK;
}

int mgcnn_residual(mgcnn_ctx* c, const float* f, const void* u, float* r) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "residual: call mgcnn_setup first");
  if (!f || !u || !r) return fail(c, MGCNN_E_ARG, "residual: null pointer");
  launch_residual_plain(c->d_a, c->d_b, f, u, c->u64(), r, c->n, c->B, c->form(), c->stream);
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

int mgcnn_loss(mgcnn_ctx* c, const float* f, const float* u, double* loss_host, float* dloss_du,
               float* dloss_df) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "loss: call mgcnn_setup first");
  if (!f || !u) return fail(c, MGCNN_E_ARG, "loss: null f or u");
  if (c->pairs()) return fail(c, MGCNN_E_STATE, "loss: no training with pack_pairs");
  if (c->u64()) return fail(c, MGCNN_E_ARG, "loss: needs f32 u");
  int r = ensure_train(c, std::max(c->tr.alloc_K, 1));
  if (r) return r;
  auto& T = c->tr;
  hipStream_t s = c->stream;
  const int B = c->B, n = c->n;
  launch_residual(c->d_a, c->d_b, f, nullptr, true, nullptr, c->d_partial, n, B, nullptr, c->form(), s);
  launch_sum_partials(c->d_partial, c->tiles, c->d_nf2, B, s);
  launch_residual_plain(c->d_a, c->d_b, f, u, false, T.r, n, B, c->form(), s);
  // ||r||^2 per problem in f64 from the float32 residual
  launch_residual(c->d_a, c->d_b, T.r, nullptr, true, nullptr, c->d_partial, n, B, nullptr, c->form(), s);
  launch_sum_partials(c->d_partial, c->tiles, T.d_rr, B, s);
  launch_loss_finalize(T.d_rr, c->d_nf2, B, T.d_loss, s);
  if (dloss_du)
    launch_apply_AT(c->d_a, c->d_b, T.r, nullptr, c->d_nf2, -2.0, false, dloss_du, nullptr, n, B, c->form(), s);
  if (dloss_df) launch_loss_df(T.r, f, T.d_rr, c->d_nf2, dloss_df, n, B, s);
  LAUNCH_CHECK(c);
  if (loss_host) {
    HIP_TRY(c, hipMemcpyAsync(loss_host, T.d_loss, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return MGCNN_OK;
}

int mgcnn_backward(mgcnn_ctx* c, const float* dL_du, float* dL_dweights, float* dL_df) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "backward: call mgcnn_setup first");
  if (c->gmg_on()) return fail(c, MGCNN_E_STATE, "backward: no weights with the GMG preconditioner");
  if (c->pairs()) return fail(c, MGCNN_E_STATE, "backward: no training with pack_pairs");
  if (c->opts.up_post) return fail(c, MGCNN_E_ARG, "backward: no reverse pass for up_post");
  auto& T = c->tr;
  if (T.K <= 0 || T.f == nullptr || T.alloc_n != c->n || T.alloc_B != c->B)
    return fail(c, MGCNN_E_NORECORD, "backward: no recorded forward for this problem set");
  if (!dL_du || !dL_dweights) return fail(c, MGCNN_E_ARG, "backward: null pointer");
  hipStream_t s = c->stream;
  const int B = c->B, n = c->n, L = c->L;
  const size_t nn = (size_t)n * n * B;
  launch_zero(T.grad, c->off.total * 4, s);
  for (int l = 0; l < L; ++l) launch_zero(T.gs[l], (size_t)c->nl[l] * c->nl[l] * B * C * 4, s);
  HIP_TRY(c, hipMemcpyAsync(T.lam0, dL_du, nn * 4, hipMemcpyDeviceToDevice, s));
  float* lam = T.lam0;
  float* lam_next = T.lam1;
  for (int k = T.K - 1; k >= 0; --k) {
    const float* uk = T.uk + (size_t)k * nn;
    launch_residual(c->d_a, c->d_b, T.f, uk, false, c->d_rt, c->d_partial, n, B, nullptr, c->form(), s);
    recompute_vcycle(c);
    vcycle_reverse(c, lam);
    // lam_k = lam_{k+1} - A^T (grt / D); dL/df += grt / D
    launch_apply_AT(c->d_a, c->d_b, T.grt, lam, nullptr, -1.0, true, lam_next, dL_df, n, B, c->form(), s);
    std::swap(lam, lam_next);
  }
  recompute_setup(c);
  setup_reverse(c);
  HIP_TRY(c, hipMemcpyAsync(dL_dweights, T.grad, c->off.total * 4, hipMemcpyDeviceToDevice, s));
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

}  // extern "C"
