// C-ABI of the MGCNN solver library: context, workspace, setup phase, solve loop.
// The kernels live in kernels_*.hip; this file only validates arguments, owns device
// memory and sequences launches on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_internal.h"
#include "mgcnn_ctx.h"
#include "mgcnn_gmg.h"

using namespace mg;

namespace mg {

WeightOffsets weight_offsets() {
  WeightOffsets w{};
  size_t o = 0;
  w.setup_in = o; o += C * 4 * 9;
  for (int k = 0; k < NUM_SETUP_LAYERS; ++k) {
    w.res_w[k] = o; o += C * C * 9;
    w.res_b[k] = o; o += C;
  }
  w.setup_restrict = o; o += C * C * 9;
  w.solve_in = o; o += C * 9;
  w.smooth_down = o; o += C * C * 9;
  w.smooth_up = o; o += C * C * 9;
  w.restrict_ = o; o += C * C * 9;
  w.prolong = o; o += C * C * 9;
  w.solve_out = o; o += C * 9;
  w.total = o;
  return w;
}

void launch_bf16_to_f32(const bf16_t* in, float* out, size_t count, hipStream_t st);
void launch_scale_by_diag(const float* a, const float* b, const float* r, float* rt, int n, int B,
                          int form, hipStream_t st);

}  // namespace mg

namespace mg {
namespace api {

int fail(mgcnn_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(mgcnn_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, MGCNN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

hipEvent_t pool_event(mgcnn_ctx* c) {
  if (c->pool_used == c->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->pool.push_back(e);
  }
  return c->pool[c->pool_used++];
}

int prof_drain(mgcnn_ctx* c) {
  for (const auto& r : c->recs) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, r.e0, r.e1));
    mgcnn_kernel_stat* hit = nullptr;
    for (auto& a : c->agg)
      if (a.kind == r.kind && a.level == r.level) { hit = &a; break; }
    if (!hit) {
      mgcnn_kernel_stat z{};
      z.kind = r.kind; z.level = r.level;
      c->agg.push_back(z);
      hit = &c->agg.back();
    }
    hit->launches += 1;
    hit->ms_total += ms;
    hit->bytes_per_launch += r.bytes;
    hit->flops_per_launch += r.flops;
  }
  c->recs.clear();
  c->pool_used = 0;
  return MGCNN_OK;
}

bool valid_n(int n) {
  if (n < 3 || n > 4095) return false;
  return ((n + 1) & n) == 0;
}

int level_count(int n) {
  int L = 0;
  while ((1 << L) - 1 < n) ++L;
  return L;
}

// Levels of the networks for grid side n under opts.levels; 0 if out of range.
int net_levels(const mgcnn_ctx* c, int n) {
  const int full = level_count(n), o = c->opts.levels;
  const int L = o == 0 ? full : (o < 0 ? full + o : o);
  return (L >= 1 && L <= full) ? L : 0;
}

void drop_graph(mgcnn_ctx* c);

void free_problem(mgcnn_ctx* c) {
  drop_graph(c);
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  fr(c->d_a); fr(c->d_b); fr(c->d_rt); fr(c->d_partial); fr(c->d_nf2);
  fr(c->d_active); fr(c->d_plist); fr(c->d_slist); fr(c->d_status); fr(c->d_iters); fr(c->d_relres);
  for (auto p : c->s) fr(p);
  for (auto p : c->xin) fr(p);
  for (auto p : c->xdn) fr(p);
  fr(c->setup_tmp);
  c->setup_tmp = nullptr;
  c->s.clear(); c->xin.clear(); c->xdn.clear();
  gmg_free(c);
  c->d_a = c->d_b = c->d_rt = nullptr;
  c->d_partial = c->d_nf2 = c->d_relres = nullptr;
  c->d_active = c->d_plist = c->d_slist = c->d_status = c->d_iters = nullptr;
  c->alloc_n = c->alloc_B = 0;
  c->ready = false;
}

int alloc(mgcnn_ctx* c, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, MGCNN_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return MGCNN_OK;
}

int ensure_problem(mgcnn_ctx* c, int n, int B) {
  if (c->alloc_n == n && c->alloc_B == B) return MGCNN_OK;
  free_problem(c);
  const int L = c->gmg_on() ? level_count(n) : net_levels(c, n);
  c->nl.assign(L, 0);
  int m = n;
  for (int l = 0; l < L; ++l) { c->nl[l] = m; m = (m - 1) / 2; }
  const size_t nn = (size_t)n * n * B;
  // packed pairs: (B + 1) / 2 state slots; rt holds two planes per slot, the unused second half
  // of an odd batch's last slot stays zero
  const int slots = c->pairs() ? (B + 1) / 2 : B;
  int r;
  if ((r = alloc(c, (void**)&c->d_a, nn * 4))) return r;
  if ((r = alloc(c, (void**)&c->d_b, (size_t)B * 2 * 4))) return r;
  if ((r = alloc(c, (void**)&c->d_rt, (size_t)n * n * (c->pairs() ? 2 * slots : B) * 4))) return r;
  if (c->pairs()) HIP_TRY(c, hipMemset(c->d_rt, 0, (size_t)n * n * 2 * slots * 4));
  if ((r = alloc(c, (void**)&c->d_slist, (size_t)slots * 4))) return r;
  c->tiles = residual_tiles(n);
  if ((r = alloc(c, (void**)&c->d_partial, (size_t)c->tiles * B * 8))) return r;
  if ((r = alloc(c, (void**)&c->d_nf2, (size_t)B * 8))) return r;
  if ((r = alloc(c, (void**)&c->d_active, (size_t)B * 4))) return r;
  if ((r = alloc(c, (void**)&c->d_plist, (size_t)B * 4))) return r;
  if ((r = alloc(c, (void**)&c->d_status, (size_t)B * 4))) return r;
  if ((r = alloc(c, (void**)&c->d_iters, (size_t)B * 4))) return r;
  if ((r = alloc(c, (void**)&c->d_relres, (size_t)B * 8))) return r;
  c->s.assign(L, nullptr); c->xin.assign(L, nullptr); c->xdn.assign(L, nullptr);
  if (c->gmg_on()) {
    if ((r = gmg_alloc(c, n, B))) return r;
  } else {
  for (int l = 0; l < L; ++l) {
    const size_t bytes = (size_t)c->nl[l] * c->nl[l] * slots * C * c->state_bytes();
    if ((r = alloc(c, &c->s[l], (size_t)c->nl[l] * c->nl[l] * slots * C * c->s_bytes()))) return r;
    if ((r = alloc(c, &c->xin[l], bytes))) return r;
    if ((r = alloc(c, &c->xdn[l], bytes))) return r;
  }
  }
  c->alloc_n = n;
  c->alloc_B = B;
  c->slots = slots;
  c->L = L;
  c->gen += 1;
  return MGCNN_OK;
}

int solve_step(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit);

void drop_graph(mgcnn_ctx* c) {
  if (c->gcache.exec) (void)hipGraphExecDestroy(c->gcache.exec);
  if (c->gcache.graph) (void)hipGraphDestroy(c->gcache.graph);
  c->gcache = mgcnn_ctx::GraphCache{};
}

// Run `chunk` solver iterations, from a cached hipGraph when enabled.
int run_chunk(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int chunk, bool graph) {
  if (!graph) {
    for (int k = 0; k < chunk; ++k) {
      int r = solve_step(c, f, u, tol, maxit);
      if (r) return r;
    }
    return MGCNN_OK;
  }
  auto& G = c->gcache;
  const bool hit = G.exec && G.f == f && G.u == u && G.tol == tol && G.maxit == maxit &&
                   G.chunk == chunk && G.gen == c->gen && G.count == c->plist_count &&
                   G.scount == c->slist_count;
  if (!hit) {
    drop_graph(c);
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    int r = MGCNN_OK;
    for (int k = 0; k < chunk && r == MGCNN_OK; ++k) r = solve_step(c, f, u, tol, maxit);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (r) { if (g) (void)hipGraphDestroy(g); return r; }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); G.exec = nullptr; return hip_fail(c, e, "hipGraphInstantiate"); }
    G.graph = g; G.f = f; G.u = u; G.tol = tol; G.maxit = maxit; G.chunk = chunk; G.gen = c->gen;
    G.count = c->plist_count;
    G.scount = c->slist_count;
  }
  HIP_TRY(c, hipGraphLaunch(G.exec, c->stream));
  return MGCNN_OK;
}

// One application of the solve network (Alg. 3) to c->d_rt, added into u (u += B(rt)), or
// stored into u (u = B(rt)) when !accumulate.
int vcycle(mgcnn_ctx* c, void* u, bool u_f64, const int* active, int count, bool accumulate,
           const int* flags) {
  if (c->gmg_on()) return gmg_cycle(c, u, u_f64, active, count, accumulate, flags);
  const StateType st = c->st();
  const int L = c->L, B = count;
  hipStream_t s = c->stream;
  const double S = (double)c->state_bytes() * C;        // bytes of one 16-channel pixel
  const double SS = (double)c->s_bytes() * C;            // bytes of one pixel of s
  const bool sb = c->s16() && st != ST_BF16;             // f32 state reading bf16 s
  // algorithmic flops per node: 16 -> 16 3x3 conv (multiply-add = 2), smoother adds s . x and
  // the skip, 1 <-> 16 3x3 conv
  const double FL_CONV = 2.0 * 9 * C * C, FL_SMOOTH = FL_CONV + 2.0 * C, FL_IN = 2.0 * 9 * C;
  auto nodes = [&](int l) { return (double)c->nl[l] * c->nl[l] * B; };
  const ConvMode up_mode = c->opts.up_post ? CM_SMOOTH_POST : CM_SMOOTH;   // up smoother form
  for (int l = 0; l < L; ++l) {
    if (l == 0) {
      // finest level: reChannel-in folded into the down smoother
      Prof p(c, MGCNN_K_SMOOTH_IN, 0, nodes(0) * (4.0 + S + SS), nodes(0) * (FL_SMOOTH + FL_IN));
      launch_smooth_in(st == ST_F32X && c->opts.f32_split == 2 ? ST_F32X2 : st, c->d_rt, c->s[0],
                       c->W(c->off.solve_in), c->W(c->off.smooth_down), c->xdn[0], c->nl[0], B, active, s, sb,
                       c->pairs());
    } else {
      Prof p(c, MGCNN_K_SMOOTH_DOWN, l, nodes(l) * (2.0 * S + SS), nodes(l) * FL_SMOOTH);
      launch_conv16(CM_SMOOTH, st, c->xin[l], c->s[l], c->W(c->off.smooth_down), nullptr, c->xdn[l],
                    c->nl[l], B, active, s, sb);
    }
    if (l < L - 1) {
      Prof p(c, MGCNN_K_RESTRICT, l, (nodes(l) + nodes(l + 1)) * S, nodes(l + 1) * FL_CONV);
      launch_conv16(CM_RESTRICT, st, c->xdn[l], nullptr, c->W(c->off.restrict_), nullptr,
                    c->xin[l + 1], c->nl[l], B, active, s);
    }
  }
  {
    Prof p(c, MGCNN_K_SMOOTH_UP, L - 1, nodes(L - 1) * (2.0 * S + SS), nodes(L - 1) * FL_SMOOTH);
    launch_conv16(up_mode, st, c->xdn[L - 1], c->s[L - 1], c->W(c->off.smooth_up), nullptr,
                  c->xin[L - 1], c->nl[L - 1], B, active, s, sb);
  }
  for (int l = L - 2; l >= 0; --l) {
    {
      Prof p(c, MGCNN_K_PROLONG, l, (nodes(l + 1) + 2.0 * nodes(l)) * S,
             nodes(l + 1) * FL_CONV + nodes(l) * C);
      launch_prolong_add(st, c->xin[l + 1], c->W(c->off.prolong), c->xdn[l], c->nl[l + 1], B,
                         active, s);
    }
    {
      Prof p(c, MGCNN_K_SMOOTH_UP, l, nodes(l) * (2.0 * S + SS), nodes(l) * FL_SMOOTH);
      launch_conv16(up_mode, st, c->xdn[l], c->s[l], c->W(c->off.smooth_up), nullptr, c->xin[l],
                    c->nl[l], B, active, s, sb);
    }
  }
  {
    Prof p(c, MGCNN_K_OUT_UPDATE, 0, nodes(0) * (S + (accumulate ? 2.0 : 1.0) * (u_f64 ? 8 : 4)),
           nodes(0) * (FL_IN + 1.0));
    if (c->pairs())
      launch_out_update_pairs(st, c->xin[0], c->W(c->off.solve_out), u, u_f64, c->n, B, c->B, active, s,
                              accumulate, flags);
    else
      launch_out_update(st, c->xin[0], c->W(c->off.solve_out), u, u_f64, c->n, B, active, s,
                        accumulate, flags);
  }
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

// residual of the current iterate, stopping test, then one V-cycle for live problems
int solve_step(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit) {
  {
    const double nodes = (double)c->n * c->n * c->plist_count;
    Prof p(c, MGCNN_K_RESIDUAL, 0, nodes * (12.0 + (c->u64() ? 8 : 4)));
    launch_residual(c->d_a, c->d_b, f, u, c->u64(), c->d_rt, c->d_partial, c->n, c->plist_count,
                    c->d_plist, c->form(), c->stream);
  }
  {
    Prof p(c, MGCNN_K_FINALIZE, 0, (double)c->tiles * c->B * 8.0);
    launch_finalize(c->d_partial, c->tiles, c->d_nf2, tol, maxit, c->d_active, c->d_status,
                    c->d_iters, c->d_relres, c->B, c->stream);
  }
  if (c->pairs()) return vcycle(c, u, c->u64(), c->d_slist, c->slist_count, true, c->d_active);
  return vcycle(c, u, c->u64(), c->d_plist, c->plist_count, true, c->d_active);
}

// Packed pairs: the weights of a network with at most 8 hidden channels, given in the 16-channel
// layout (every entry that reads or writes a channel >= 8 zero), turned into the weights that
// run two problems side by side: every 16 -> 16 conv becomes diag(W8, W8) and each tanh layer's
// bias repeats its first eight entries; the 4 -> 16, 1 -> 16 and 16 -> 1 convs stay as given
// (their kernels use the first eight output rows / input columns for each half).  Returns false
// if the weights use channels 8..15.
bool pack_pair_weights(const WeightOffsets& off, const float* w, std::vector<float>& out) {
  out.assign(w, w + off.total);
  auto zero = [](float v) { return v == 0.f; };
  // 16 -> 16 convs W[o][c][9]
  const size_t sq[] = {off.res_w[0], off.res_w[1], off.res_w[2], off.res_w[3], off.setup_restrict,
                       off.smooth_down, off.smooth_up, off.restrict_, off.prolong};
  for (size_t base : sq) {
    for (int o = 0; o < C; ++o)
      for (int ci = 0; ci < C; ++ci)
        for (int k = 0; k < 9; ++k) {
          const float v = w[base + ((size_t)o * C + ci) * 9 + k];
          if ((o >= 8 || ci >= 8) && !zero(v)) return false;
          const bool diag = (o < 8) == (ci < 8);
          out[base + ((size_t)o * C + ci) * 9 + k] = diag ? w[base + ((size_t)(o % 8) * C + ci % 8) * 9 + k] : 0.f;
        }
  }
  for (int k = 0; k < NUM_SETUP_LAYERS; ++k)
    for (int o = 0; o < C; ++o) {
      if (o >= 8 && !zero(w[off.res_b[k] + o])) return false;
      out[off.res_b[k] + o] = w[off.res_b[k] + o % 8];
    }
  for (int o = 8; o < C; ++o) {
    for (int k = 0; k < 4 * 9; ++k)
      if (!zero(w[off.setup_in + (size_t)o * 4 * 9 + k])) return false;
    for (int k = 0; k < 9; ++k)
      if (!zero(w[off.solve_in + (size_t)o * 9 + k]) || !zero(w[off.solve_out + (size_t)o * 9 + k])) return false;
  }
  return true;
}

}  // namespace api
}  // namespace mg

using namespace mg::api;

extern "C" {

void mgcnn_default_opts(mgcnn_opts* o) {
  if (!o) return;
  o->channels = 16;
  o->state_dtype = MGCNN_F32;
  o->u_dtype = MGCNN_U_F64;
  o->use_graph = 0;
  o->check_every = 4;
  o->method = MGCNN_METHOD_STATIONARY;
  o->restart = 30;
  o->f32_split = 1;
  o->s_bf16 = 0;
  o->inner_steps = 1;
  o->gs_passes = 2;
  o->precond = MGCNN_PRECOND_NETWORK;
  o->gmg_levels = 0;
  o->gmg_sweeps = 3;
  o->gmg_omega = 0.67f;
  o->op_form = MGCNN_OP_DIV;
  o->deflate = 0;
  o->levels = 0;
  o->up_post = 0;
  o->pack_pairs = 0;
}

size_t mgcnn_num_weights(int channels) {
  if (channels <= 0) return 0;
  return (size_t)81 * channels * channels + (size_t)58 * channels;
}

int mgcnn_create(mgcnn_ctx** out, const mgcnn_opts* opts, const float* weights_host,
                 void* hip_stream) {
  if (!out) return MGCNN_E_ARG;
  *out = nullptr;
  mgcnn_opts o;
  if (opts) o = *opts; else mgcnn_default_opts(&o);
  if (o.channels != C) return MGCNN_E_ARG;
  if (o.state_dtype != MGCNN_F32 && o.state_dtype != MGCNN_BF16) return MGCNN_E_ARG;
  if (o.u_dtype != MGCNN_U_F32 && o.u_dtype != MGCNN_U_F64) return MGCNN_E_ARG;
  if (o.check_every < 1) return MGCNN_E_ARG;
  if (o.method != MGCNN_METHOD_STATIONARY && o.method != MGCNN_METHOD_FGMRES && o.method != MGCNN_METHOD_PCG)
    return MGCNN_E_ARG;
  // conjugate gradients need a symmetric preconditioner: the network only in its symmetric form
  if (o.method == MGCNN_METHOD_PCG && o.precond == MGCNN_PRECOND_NETWORK && !o.up_post) return MGCNN_E_ARG;
  if (o.method == MGCNN_METHOD_PCG && (o.op_form != MGCNN_OP_DIV || o.inner_steps != 1))
    return MGCNN_E_ARG;
  if (o.f32_split < 0 || o.f32_split > 2) return MGCNN_E_ARG;
  if (o.s_bf16 != 0 && o.s_bf16 != 1) return MGCNN_E_ARG;
  if (o.inner_steps < 1 || o.inner_steps > 16) return MGCNN_E_ARG;
  if (o.gs_passes != 1 && o.gs_passes != 2) return MGCNN_E_ARG;
  if (o.method == MGCNN_METHOD_FGMRES && (o.restart < 1 || o.restart > 63)) return MGCNN_E_ARG;
  if (o.precond != MGCNN_PRECOND_NETWORK && o.precond != MGCNN_PRECOND_GMG) return MGCNN_E_ARG;
  if (o.gmg_levels < 0 || o.gmg_sweeps < 1 || o.gmg_sweeps > GMG_MAX_SWEEPS) return MGCNN_E_ARG;
  if (!(o.gmg_omega > 0.f && o.gmg_omega < 2.f)) return MGCNN_E_ARG;
  if (o.op_form != MGCNN_OP_DIV && o.op_form != MGCNN_OP_NONDIV) return MGCNN_E_ARG;
  if (o.deflate < 0 || o.deflate > 32) return MGCNN_E_ARG;
  // at least half of every deflated cycle must be new Krylov vectors: with fewer, a cycle adds
  // too little to its kept directions and the restarted iteration can stagnate
  if (o.method == MGCNN_METHOD_FGMRES && o.deflate > 0 && 2 * o.deflate > o.restart) return MGCNN_E_ARG;
  if (o.levels < -11 || o.levels > 12) return MGCNN_E_ARG;
  if (o.up_post != 0 && o.up_post != 1) return MGCNN_E_ARG;
  if (o.pack_pairs != 0 && o.pack_pairs != 1) return MGCNN_E_ARG;
  if (o.pack_pairs && (o.method != MGCNN_METHOD_STATIONARY || o.precond != MGCNN_PRECOND_NETWORK || o.s_bf16))
    return MGCNN_E_ARG;
  mgcnn_ctx* c = new (std::nothrow) mgcnn_ctx();
  if (!c) return MGCNN_E_NOMEM;
  c->opts = o;
  c->stream = (hipStream_t)hip_stream;
  c->off = weight_offsets();
  if (alloc(c, (void**)&c->d_w, c->off.total * 4)) { delete c; return MGCNN_E_NOMEM; }
  int r = mgcnn_set_weights(c, weights_host);
  if (r) { (void)hipFree(c->d_w); delete c; return r; }
  *out = c;
  return MGCNN_OK;
}

int mgcnn_set_weights(mgcnn_ctx* c, const float* w) {
  if (!c) return MGCNN_E_ARG;
  c->tr.K = 0;             // a recorded forward was taken with the previous weights
  c->tr.f = nullptr;
  if (w == nullptr) {
    launch_zero(c->d_w, c->off.total * 4, c->stream);
    LAUNCH_CHECK(c);
    return MGCNN_OK;
  }
  std::vector<float> packed;
  if (c->pairs()) {
    if (!pack_pair_weights(c->off, w, packed))
      return fail(c, MGCNN_E_ARG, "set_weights: pack_pairs needs a network of at most 8 hidden channels "
                                  "(channels 8..15 zero)");
    w = packed.data();
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_w, w, c->off.total * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MGCNN_OK;
}

int mgcnn_set_stream(mgcnn_ctx* c, void* s) {
  if (!c) return MGCNN_E_ARG;
  c->stream = (hipStream_t)s;
  return MGCNN_OK;
}

// Copy the host velocities [B][2] to c->d_b through the context's pinned staging buffer: the
// host copy into it is synchronous, so b_host may be released when the call returns, and the
// previous setup's copy out of it is waited for before it is overwritten.
static int stage_velocities(mgcnn_ctx* c, const float* b_host, int B) {
  if (c->bstage_pending) {
    HIP_TRY(c, hipEventSynchronize(c->bstage_ev));
    c->bstage_pending = false;
  }
  if (!c->bstage_ev) HIP_TRY(c, hipEventCreateWithFlags(&c->bstage_ev, hipEventDisableTiming));
  if (c->bstage_cap < 2 * B) {
    if (c->h_bstage) HIP_TRY(c, hipHostFree(c->h_bstage));
    c->h_bstage = nullptr;
    c->bstage_cap = 0;
    HIP_TRY(c, hipHostMalloc((void**)&c->h_bstage, (size_t)B * 2 * 4, hipHostMallocDefault));
    c->bstage_cap = 2 * B;
  }
  std::memcpy(c->h_bstage, b_host, (size_t)B * 2 * 4);
  HIP_TRY(c, hipMemcpyAsync(c->d_b, c->h_bstage, (size_t)B * 2 * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipEventRecord(c->bstage_ev, c->stream));
  c->bstage_pending = true;
  return MGCNN_OK;
}

int mgcnn_setup(mgcnn_ctx* c, const float* a, const float* b_host, int n, int B) {
  if (!c) return MGCNN_E_ARG;
  if (!a || !b_host) return fail(c, MGCNN_E_ARG, "setup: null a or b");
  if (!valid_n(n)) return fail(c, MGCNN_E_SIZE, "setup: n must be 2^L - 1 in [3, 4095]");
  if (B < 1) return fail(c, MGCNN_E_SIZE, "setup: batch must be >= 1");
  for (int i = 0; i < 2 * B; ++i)
    if (!std::isfinite(b_host[i])) return fail(c, MGCNN_E_ARG, "setup: non-finite velocity");
  if (c->gmg_on() && gmg_levels_for(c, n) == 0)
    return fail(c, MGCNN_E_ARG, "setup: gmg_levels out of range for this n");
  if (!c->gmg_on() && net_levels(c, n) == 0)
    return fail(c, MGCNN_E_ARG, "setup: levels out of range for this n");
  c->ready = false;
  c->tr.K = 0;             // a recorded forward belongs to the previous problem set
  c->tr.f = nullptr;
  int r = ensure_problem(c, n, B);
  if (r) return r;
  c->n = n;
  c->B = B;
  hipStream_t s = c->stream;
  const size_t nn = (size_t)n * n * B;
  HIP_TRY(c, hipMemcpyAsync(c->d_a, a, nn * 4, hipMemcpyDeviceToDevice, s));
  if ((r = stage_velocities(c, b_host, B))) return r;
  if (c->gmg_on()) {
    if ((r = gmg_setup(c))) return r;
    c->ready = true;
    return MGCNN_OK;
  }
  // Alg. 2 with the levels' tanh layers fused (Setup2 does not couple the levels once the
  // restricted coefficient tensors exist): features and reChannel on the finest level, the
  // restriction chain c_1 -> c_2 -> ... -> c_L, then each of the four tanh layers as one launch
  // over all levels.  With f32 storage the level tensors hold the intermediates (c_l in xin_l,
  // the layers ping-pong between xdn_l and s_l and end in s_l); bf16 storage uses two f32 level
  // pyramids kept in the context for the next setup of this size: the first holds c_l, then the
  // outputs of the second and fourth layers, the second the outputs of the first and third.
  const int L = c->L, SL = c->slots;                   // SL: state slots (packed pairs: (B + 1) / 2)
  const bool f32_store = c->state_bytes() == 4 && !c->s16();
  size_t pyr = 0;                                      // floats of one f32 level pyramid
  for (int l = 0; l < L; ++l) pyr += (size_t)c->nl[l] * c->nl[l] * SL * C;
  if (!c->setup_tmp && (r = alloc(c, &c->setup_tmp, nn * 16 + (f32_store ? 0 : 2 * pyr * 4)))) return r;
  float* F = (float*)c->setup_tmp;
  float *cl[MAX_LEVELS], *za[MAX_LEVELS], *zb[MAX_LEVELS];
  {
    float* p = F + nn * 4;
    for (int l = 0; l < L; ++l) {
      const size_t cnt = (size_t)c->nl[l] * c->nl[l] * SL * C;
      if (f32_store) {
        cl[l] = (float*)c->xin[l];
        za[l] = (float*)c->xdn[l];
        zb[l] = (float*)c->s[l];
      } else {
        cl[l] = p;
        za[l] = p + pyr;
        zb[l] = p;
        p += cnt;
      }
    }
  }
  launch_features(c->d_a, c->d_b, F, n, B, c->form(), s);
  if (c->pairs()) launch_conv_in_pairs(F, c->W(c->off.setup_in), cl[0], n, B, s);
  else launch_conv_in(4, F, c->W(c->off.setup_in), cl[0], ST_F32, n, B, nullptr, s);
  for (int l = 0; l + 1 < L; ++l)
    launch_conv16(CM_RESTRICT, ST_F32, cl[l], nullptr, c->W(c->off.setup_restrict), nullptr, cl[l + 1],
                  c->nl[l], SL, nullptr, s);
  int bl[MAX_LEVELS];
  for (int l = 0; l < L; ++l) bl[l] = SL;
  // the tanh layers compute in f32 intermediates: float32-level products (three-way split), or,
  // with bf16 state (the setup tensors then rounded to 2^-8), the two-way split (about 2^-16);
  // s_bf16 with f32 state keeps the f32 tensors rounded once
  const StateType tanh_t = !c->opts.f32_split ? ST_F32 : (c->st() == ST_BF16 ? ST_F32X2 : ST_F32X);
  float** src[NUM_SETUP_LAYERS] = {cl, za, zb, za};
  float** dst[NUM_SETUP_LAYERS] = {za, zb, za, zb};
  for (int k = 0; k < NUM_SETUP_LAYERS; ++k)
    launch_tanh_levels(tanh_t, src[k], dst[k], c->nl.data(), bl, L, c->W(c->off.res_w[k]),
                       c->W(c->off.res_b[k]), s);
  if (!f32_store)
    for (int l = 0; l < L; ++l)
      launch_f32_to_bf16(zb[l], (bf16_t*)c->s[l], (size_t)c->nl[l] * c->nl[l] * SL * C, s);
  LAUNCH_CHECK(c);
  c->ready = true;
  return MGCNN_OK;
}

int mgcnn_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
                double* relres_host, int* status_host) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "solve: call mgcnn_setup first");
  if (!f || !u) return fail(c, MGCNN_E_ARG, "solve: null f or u");
  if (!(tol > 0.0) || maxit < 0) return fail(c, MGCNN_E_ARG, "solve: need tol > 0 and maxit >= 0");
  if (c->opts.method == MGCNN_METHOD_FGMRES)
    return fgmres_solve(c, f, u, tol, maxit, iters_host, relres_host, status_host);
  if (c->opts.method == MGCNN_METHOD_PCG)
    return pcg_solve(c, f, u, tol, maxit, iters_host, relres_host, status_host);
  const bool graph = c->opts.use_graph != 0 && !c->prof;
  hipStream_t user = c->stream;
  if (graph && user == nullptr) {
    // stream capture needs a non-null stream: work on a private one ordered after the user's
    if (!c->cap_stream) {
      HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    }
    HIP_TRY(c, hipEventRecord(c->join_ev, user));
    HIP_TRY(c, hipStreamWaitEvent(c->cap_stream, c->join_ev, 0));
    c->stream = c->cap_stream;
  }
  struct Restore { mgcnn_ctx* c; hipStream_t s; ~Restore() { c->stream = s; } } restore{c, user};
  hipStream_t s = c->stream;
  const int B = c->B;
  // ||f||^2 per problem
  launch_residual(c->d_a, c->d_b, f, nullptr, true, nullptr, c->d_partial, c->n, B, nullptr,
                  c->form(), s);
  launch_sum_partials(c->d_partial, c->tiles, c->d_nf2, B, s);
  launch_solve_init(c->d_nf2, c->d_active, c->d_status, c->d_iters, c->d_relres, B, s);
  launch_zero_if_zero_rhs(u, c->u64(), c->d_nf2, c->n, B, s);
  LAUNCH_CHECK(c);
  // the launches cover a compact list of the problems still iterating, rebuilt at every host
  // check; problems that finish between checks are held by their flag (u is left unchanged)
  // (packed pairs: the state launches cover the slots with a live problem, `slist`)
  std::vector<int> act(B), plist(B), slist(c->slots);
  for (int b = 0; b < B; ++b) plist[b] = b;
  for (int v = 0; v < c->slots; ++v) slist[v] = v;
  c->plist_count = B;
  c->slist_count = c->slots;
  HIP_TRY(c, hipMemcpyAsync(c->d_plist, plist.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_slist, slist.data(), (size_t)c->slots * 4, hipMemcpyHostToDevice, s));
  int steps = 0;
  const int max_steps = maxit + 1;
  while (steps < max_steps) {
    const int chunk = std::min(c->opts.check_every, max_steps - steps);
    int r = run_chunk(c, f, u, tol, maxit, chunk, graph && chunk == c->opts.check_every);
    if (r) return r;
    steps += chunk;
    HIP_TRY(c, hipMemcpyAsync(act.data(), c->d_active, (size_t)B * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->prof && (r = prof_drain(c))) return r;
    int cnt = 0;
    for (int b = 0; b < B; ++b)
      if (act[b] != 0) plist[cnt++] = b;
    if (cnt == 0) break;
    if (cnt != c->plist_count) {
      c->plist_count = cnt;
      HIP_TRY(c, hipMemcpyAsync(c->d_plist, plist.data(), (size_t)cnt * 4, hipMemcpyHostToDevice, s));
      if (c->pairs()) {
        int sc = 0;
        for (int v = 0; v < c->slots; ++v)
          if (act[2 * v] != 0 || (2 * v + 1 < B && act[2 * v + 1] != 0)) slist[sc++] = v;
        c->slist_count = sc;
        HIP_TRY(c, hipMemcpyAsync(c->d_slist, slist.data(), (size_t)sc * 4, hipMemcpyHostToDevice, s));
      }
      HIP_TRY(c, hipStreamSynchronize(s));   // plist and slist are rewritten at the next check
    }
  }
  std::vector<int> st(B), it(B);
  std::vector<double> rr(B);
  HIP_TRY(c, hipMemcpyAsync(st.data(), c->d_status, (size_t)B * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(it.data(), c->d_iters, (size_t)B * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(rr.data(), c->d_relres, (size_t)B * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  bool diverged = false, notconv = false;
  for (int b = 0; b < B; ++b) {
    if (iters_host) iters_host[b] = it[b];
    if (relres_host) relres_host[b] = rr[b];
    if (status_host) status_host[b] = st[b];
    diverged |= st[b] == MGCNN_E_DIVERGED;
    notconv |= st[b] == MGCNN_NOT_CONVERGED;
  }
  if (diverged) return fail(c, MGCNN_E_DIVERGED, "solve: a problem diverged");
  if (notconv) return MGCNN_NOT_CONVERGED;
  return MGCNN_OK;
}

int mgcnn_forward(mgcnn_ctx* c, const float* f, void* u, int K, int record) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "forward: call mgcnn_setup first");
  if (!f || !u || K < 0) return fail(c, MGCNN_E_ARG, "forward: bad argument");
  if (record && c->gmg_on())
    return fail(c, MGCNN_E_STATE, "forward: recording needs the network preconditioner");
  if (record && c->pairs()) return fail(c, MGCNN_E_STATE, "forward: no recording with pack_pairs");
  if (record) return forward_record(c, f, (float*)u, K);
  for (int k = 0; k < K; ++k) {
    {
      const double nodes = (double)c->n * c->n * c->B;
      Prof p(c, MGCNN_K_RESIDUAL, 0, nodes * (12.0 + (c->u64() ? 8 : 4)));
      launch_residual(c->d_a, c->d_b, f, u, c->u64(), c->d_rt, c->d_partial, c->n, c->B, nullptr,
                      c->form(), c->stream);
    }
    int r = vcycle(c, u, c->u64(), nullptr, c->slots);
    if (r) return r;
  }
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

int mgcnn_apply(mgcnn_ctx* c, const float* r, float* z) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "apply: call mgcnn_setup first");
  if (!r || !z) return fail(c, MGCNN_E_ARG, "apply: null pointer");
  launch_scale_by_diag(c->d_a, c->d_b, r, c->d_rt, c->n, c->B, c->form(), c->stream);
  return vcycle(c, z, false, nullptr, c->slots, false);
}

int mgcnn_residual_norms(mgcnn_ctx* c, const float* f, const void* u, double* relres_host) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "residual: call mgcnn_setup first");
  if (!f || !u || !relres_host) return fail(c, MGCNN_E_ARG, "residual: null pointer");
  hipStream_t s = c->stream;
  const int B = c->B;
  launch_residual(c->d_a, c->d_b, f, nullptr, true, nullptr, c->d_partial, c->n, B, nullptr,
                  c->form(), s);
  launch_sum_partials(c->d_partial, c->tiles, c->d_nf2, B, s);
  launch_residual(c->d_a, c->d_b, f, u, c->u64(), nullptr, c->d_partial, c->n, B, nullptr,
                  c->form(), s);
  launch_relres(c->d_partial, c->tiles, c->d_nf2, c->d_relres, B, s);
  LAUNCH_CHECK(c);
  HIP_TRY(c, hipMemcpyAsync(relres_host, c->d_relres, (size_t)B * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return MGCNN_OK;
}

int mgcnn_get_setup_tensor(mgcnn_ctx* c, int level, float* out) {
  if (!c) return MGCNN_E_ARG;
  if (!c->ready) return fail(c, MGCNN_E_STATE, "get_setup_tensor: no setup");
  if (c->gmg_on()) return fail(c, MGCNN_E_STATE, "get_setup_tensor: no setup tensors with GMG");
  if (c->pairs()) return fail(c, MGCNN_E_STATE, "get_setup_tensor: setup tensors are packed in pairs");
  if (level < 1 || level > c->L || !out) return fail(c, MGCNN_E_ARG, "get_setup_tensor: bad level");
  const int m = c->nl[level - 1];
  const size_t cnt = (size_t)m * m * c->B * C;
  if (!c->s16())
    HIP_TRY(c, hipMemcpyAsync(out, c->s[level - 1], cnt * 4, hipMemcpyDeviceToDevice, c->stream));
  else
    launch_bf16_to_f32((const bf16_t*)c->s[level - 1], out, cnt, c->stream);
  LAUNCH_CHECK(c);
  return MGCNN_OK;
}

int mgcnn_profile_begin(mgcnn_ctx* c) {
  if (!c) return MGCNN_E_ARG;
  c->recs.clear();
  c->agg.clear();
  c->pool_used = 0;
  c->prof = true;
  return MGCNN_OK;
}

int mgcnn_profile_end(mgcnn_ctx* c, mgcnn_kernel_stat* stats, int max_stats, int* n_stats) {
  if (!c) return MGCNN_E_ARG;
  c->prof = false;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int r = prof_drain(c);
  if (r) return r;
  std::vector<mgcnn_kernel_stat> out = c->agg;
  for (auto& a : out) {
    a.bytes_per_launch = a.launches ? a.bytes_per_launch / a.launches : 0.0;
    a.flops_per_launch = a.launches ? a.flops_per_launch / a.launches : 0.0;
  }
  c->agg.clear();
  if (n_stats) *n_stats = (int)out.size();
  if (stats)
    for (int i = 0; i < (int)out.size() && i < max_stats; ++i) stats[i] = out[i];
  return MGCNN_OK;
}

int mgcnn_levels(const mgcnn_ctx* c) { return (c && c->ready) ? c->L : 0; }

int mgcnn_gmg_levels(const mgcnn_ctx* c) {
  return (c && c->ready && c->gmg_on()) ? c->gmg.levels : 0;
}

const char* mgcnn_status_string(int s) {
  switch (s) {
    case MGCNN_OK: return "ok";
    case MGCNN_NOT_CONVERGED: return "not converged (maxit reached)";
    case MGCNN_E_ARG: return "invalid argument";
    case MGCNN_E_SIZE: return "invalid size";
    case MGCNN_E_STATE: return "invalid call order";
    case MGCNN_E_NOMEM: return "out of device memory";
    case MGCNN_E_HIP: return "HIP runtime error";
    case MGCNN_E_DIVERGED: return "diverged";
    case MGCNN_E_NORECORD: return "no recorded forward";
    case MGCNN_E_SCRATCH:
      return "input exceeds the fixed scratch buffer of mgcnn_residual_norms_noalloc "
             "(MGCNN_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

const char* mgcnn_last_error(const mgcnn_ctx* c) { return c ? c->err.c_str() : "null context"; }

static bool tile_args_ok(int op, int state_dtype) {
  return op >= 0 && op < TILE_OPS && (state_dtype == MGCNN_F32 || state_dtype == MGCNN_BF16);
}

int mgcnn_set_tile_variant(int op, int state_dtype, int m, int variant) {
  if (!tile_args_ok(op, state_dtype) || variant < 0 || variant >= TILE_VARIANTS || m < 1 || m > 4095 ||
      tile_variant_rows(op, state_dtype == MGCNN_BF16, variant) <= 0)
    return MGCNN_E_ARG;
  if (op == TILE_SETUP && state_dtype == MGCNN_BF16) return MGCNN_E_ARG;   // the setup runs in f32
  set_tile_variant(op, state_dtype == MGCNN_BF16, m, variant);
  return MGCNN_OK;
}

int mgcnn_tile_variant(int op, int state_dtype, int m) {
  if (!tile_args_ok(op, state_dtype) || m < 1 || m > 4095) return MGCNN_E_ARG;
  return get_tile_variant(op, state_dtype == MGCNN_BF16, m);
}

int mgcnn_tile_rows(int op, int state_dtype, int variant) {
  if (!tile_args_ok(op, state_dtype)) return MGCNN_E_ARG;
  const int r = tile_variant_rows(op, state_dtype == MGCNN_BF16, variant);
  return r > 0 ? r : MGCNN_E_ARG;
}

void mgcnn_destroy(mgcnn_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
  free_train(c);
  free_krylov(c);
  free_pcg(c);
  drop_graph(c);
  free_problem(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->join_ev) (void)hipEventDestroy(c->join_ev);
  if (c->bstage_ev) (void)hipEventDestroy(c->bstage_ev);
  if (c->h_bstage) (void)hipHostFree(c->h_bstage);
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->d_w) (void)hipFree(c->d_w);
  delete c;
}

}  // extern "C"
