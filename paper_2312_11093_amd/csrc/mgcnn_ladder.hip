// Uneven-size batches with the levels of all problems aligned by grid size (see mgcnn_ladder.h):
// setup network (Alg. 2) and stationary iteration (Eq. (1), Alg. 3) over the whole mixed batch
// on one stream, one launch per operation and level size.
#include "mgcnn_ladder.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace mg {

size_t Ladder::sbytes() const {
  return (opts.state_dtype == MGCNN_BF16 || opts.s_bf16) ? 2 : 4;
}
size_t Ladder::xbytes() const { return opts.state_dtype == MGCNN_BF16 ? 2 : 4; }

namespace {

int lfail(Ladder* L, int status, const std::string& msg) {
  L->err = msg;
  return status;
}

#define LTRY(call)                                                        \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      return lfail(L, MGCNN_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int lalloc(Ladder* L, void** p, size_t bytes) {
  if (hipMalloc(p, bytes < 256 ? 256 : bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return lfail(L, MGCNN_E_NOMEM, "group: hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return MGCNN_OK;
}

bool valid_side(int n) { return n >= 3 && n <= 4095 && ((n + 1) & n) == 0; }

int log2p1(int n) {   // log2(n + 1) for n = 2^p - 1
  int p = 0;
  while ((1 << p) < n + 1) ++p;
  return p;
}

void drop_graph(Ladder* L) {
  if (L->gexec) (void)hipGraphExecDestroy(L->gexec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->gexec = nullptr;
  L->graph = nullptr;
  L->g_chunk = 0;
}

void free_arrays(Ladder* L) {
  drop_graph(L);
  auto fr = [](void* p) { if (p) (void)hipFree(p); };
  for (auto* v : {&L->s, &L->xin, &L->xdn, &L->u})
    for (void* p : *v) fr(p);
  for (auto* v : {&L->a, &L->f, &L->rt})
    for (float* p : *v) fr(p);
  for (double* p : L->partial) fr(p);
  L->s.clear(); L->xin.clear(); L->xdn.clear(); L->u.clear();
  L->a.clear(); L->f.clear(); L->rt.clear(); L->partial.clear();
  fr(L->d_b); fr(L->nf2); fr(L->relres); fr(L->active); fr(L->status); fr(L->iters); fr(L->clock);
  L->d_b = nullptr; L->nf2 = nullptr; L->relres = nullptr;
  L->active = L->status = L->iters = nullptr;
  L->clock = nullptr;
  L->ready = false;
  L->count = 0;
  L->real = 0;
}

StateType state_of(const mgcnn_opts& o) {
  if (o.state_dtype == MGCNN_BF16) return ST_BF16;
  return o.f32_split ? ST_F32X : ST_F32;
}

// residual and stopping test of every problem at its finest grid, then one V-cycle over the
// aligned levels; u += B(r / D) for the problems still iterating
void step(Ladder* L, double tol, int maxit) {
  const mgcnn_opts& o = L->opts;
  hipStream_t st = L->stream;
  const bool u64 = o.u_dtype == MGCNN_U_F64;
  const StateType t = state_of(o);
  const StateType t_in = (t == ST_F32X && o.f32_split == 2) ? ST_F32X2 : t;
  const bool sb = o.s_bf16 && t != ST_BF16;
  const ConvMode up_mode = o.up_post ? CM_SMOOTH_POST : CM_SMOOTH;
  const size_t xb = L->xbytes(), sbb = L->sbytes();
  auto at = [&](const std::vector<void*>& v, size_t bytes, int j, int q) {
    return (void*)((char*)v[j] + (size_t)q * L->m[j] * L->m[j] * C * bytes);
  };
  auto W = [&](size_t off) { return (const float*)(L->d_w + off); };
  for (int j = 0; j < L->J; ++j) {
    const int cj = L->c(j), lo = L->lo[j];
    if (cj == 0) continue;
    launch_residual(L->a[j], L->d_b + 2 * lo, L->f[j], L->u[j], u64, L->rt[j], L->partial[j], L->m[j],
                    cj, nullptr, o.op_form, st);
    launch_finalize(L->partial[j], residual_tiles(L->m[j]), L->nf2 + lo, tol, maxit, L->active + lo,
                    L->status + lo, L->iters + lo, L->relres + lo, cj, st, L->clock + lo);
  }
  // state tensors are indexed by slot (sorted position, or position / 2 with packed pairs)
  for (int j = 0; j < L->J; ++j) {
    const int cj = L->c(j), lo = L->lo[j], mj = L->m[j];
    if (cj > 0)   // finest grid of the problems [lo, k_j): reChannel-in folded into the smoother
      launch_smooth_in(t_in, L->rt[j], at(L->s, sbb, j, L->sl(lo)), W(L->off.solve_in), W(L->off.smooth_down),
                       at(L->xdn, xb, j, L->sl(lo)), mj, L->sl(cj), nullptr, st, sb, L->pairs);
    if (lo > 0)   // coarser level of the larger problems [0, lo)
      launch_conv16(CM_SMOOTH, t, L->xin[j], L->s[j], W(L->off.smooth_down), nullptr, L->xdn[j], mj, L->sl(lo),
                    nullptr, st, sb);
    if (j < L->J - 1)
      launch_conv16(CM_RESTRICT, t, L->xdn[j], nullptr, W(L->off.restrict_), nullptr, L->xin[j + 1], mj,
                    L->sl(L->k[j]), nullptr, st);
  }
  const int jc = L->J - 1;
  launch_conv16(up_mode, t, L->xdn[jc], L->s[jc], W(L->off.smooth_up), nullptr, L->xin[jc], L->m[jc],
                L->sl(L->k[jc]), nullptr, st, sb);
  for (int j = L->J - 2; j >= 0; --j) {
    launch_prolong_add(t, L->xin[j + 1], W(L->off.prolong), L->xdn[j], L->m[j + 1], L->sl(L->k[j]), nullptr,
                       st);
    launch_conv16(up_mode, t, L->xdn[j], L->s[j], W(L->off.smooth_up), nullptr, L->xin[j], L->m[j],
                  L->sl(L->k[j]), nullptr, st, sb);
  }
  for (int j = 0; j < L->J; ++j) {
    const int cj = L->c(j), lo = L->lo[j];
    if (cj == 0) continue;
    if (L->pairs)
      launch_out_update_pairs(t, at(L->xin, xb, j, lo / 2), W(L->off.solve_out), L->u[j], u64, L->m[j], cj / 2,
                              cj, nullptr, st, true, L->active + lo);
    else
      launch_out_update(t, at(L->xin, xb, j, lo), W(L->off.solve_out), L->u[j], u64, L->m[j], cj, nullptr,
                        st, true, L->active + lo);
  }
}

}  // namespace

bool ladder_supported(const mgcnn_opts& o) {
  return o.method == MGCNN_METHOD_STATIONARY && o.precond == MGCNN_PRECOND_NETWORK && o.levels <= 0;
}

int ladder_create(Ladder* L, const mgcnn_opts& o, const float* weights_host) {
  L->opts = o;
  L->off = weight_offsets();
  L->pairs = o.pack_pairs != 0;
  std::vector<float> packed;
  if (L->pairs && weights_host) {
    if (!api::pack_pair_weights(L->off, weights_host, packed))
      return lfail(L, MGCNN_E_ARG, "group: pack_pairs needs a network of at most 8 hidden channels");
    weights_host = packed.data();
  }
  if (int r = lalloc(L, (void**)&L->d_w, L->off.total * 4)) return r;
  if (weights_host)
    LTRY(hipMemcpy(L->d_w, weights_host, L->off.total * 4, hipMemcpyHostToDevice));
  else
    LTRY(hipMemset(L->d_w, 0, L->off.total * 4));
  LTRY(hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking));
  int dev = 0;
  LTRY(hipGetDevice(&dev));
  LTRY(hipDeviceGetAttribute(&L->clock_khz, hipDeviceAttributeWallClockRate, dev));
  return MGCNN_OK;
}

void ladder_free(Ladder* L) {
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  free_arrays(L);
  if (L->tmp) (void)hipFree(L->tmp);
  L->tmp = nullptr;
  L->tmp_bytes = 0;
  if (L->d_w) (void)hipFree(L->d_w);
  L->d_w = nullptr;
  if (L->stream) (void)hipStreamDestroy(L->stream);
  L->stream = nullptr;
}

static int wait_on(Ladder* L, hipStream_t user) {
  hipEvent_t ev;
  LTRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  hipError_t e = hipEventRecord(ev, user);
  if (e == hipSuccess) e = hipStreamWaitEvent(L->stream, ev, 0);
  (void)hipEventDestroy(ev);
  if (e != hipSuccess) return lfail(L, MGCNN_E_HIP, hipGetErrorString(e));
  return MGCNN_OK;
}

int ladder_setup(Ladder* L, const float* const* a, const float* b_host, const int* n_host,
                 int count, hipStream_t user) {
  const mgcnn_opts& o = L->opts;
  for (int i = 0; i < count; ++i) {
    if (!valid_side(n_host[i])) return lfail(L, MGCNN_E_SIZE, "group_setup: n must be 2^L - 1 in [3, 4095]");
    if (!a[i]) return lfail(L, MGCNN_E_ARG, "group_setup: null coefficient pointer");
  }
  for (int i = 0; i < 2 * count; ++i)
    if (!std::isfinite(b_host[i])) return lfail(L, MGCNN_E_ARG, "group_setup: non-finite velocity");
  // coarsest side shared by every problem: 1 (opts.levels = 0) or 2^(d+1) - 1 (levels = -d)
  const int d = -o.levels;
  const int coarsest = (1 << (d + 1)) - 1;
  for (int i = 0; i < count; ++i)
    if (n_host[i] < coarsest)
      return lfail(L, MGCNN_E_ARG, "group_setup: levels out of range for a problem size");
  if (int r = wait_on(L, user)) return r;
  std::vector<int> sorted(count);
  std::iota(sorted.begin(), sorted.end(), 0);
  std::stable_sort(sorted.begin(), sorted.end(), [&](int x, int y) { return n_host[x] > n_host[y]; });
  // sorted positions; with packed pairs a phantom (-1) closes every size group of odd count
  std::vector<int> order, nq;
  for (int i = 0; i < count; ++i) {
    const int n = n_host[sorted[i]];
    order.push_back(sorted[i]);
    nq.push_back(n);
    const bool group_end = i + 1 == count || n_host[sorted[i + 1]] != n;
    if (L->pairs && group_end && order.size() % 2 == 1) {
      order.push_back(-1);
      nq.push_back(n);
    }
  }
  // the device arrays depend only on the sorted sizes: a setup with the same sizes keeps them
  // (freeing and reallocating tens of GB at every setup costs more than the setup itself)
  const bool same_layout = L->ready && !L->s.empty() && nq == L->nq;   // the last setup completed
  if (!same_layout) free_arrays(L);
  drop_graph(L);
  L->ready = false;
  const int real = count;
  L->order = order;
  L->nq = nq;
  L->real = real;
  count = (int)L->order.size();
  L->count = count;
  L->pos.assign(L->real, 0);
  for (int q = 0; q < count; ++q)
    if (L->order[q] >= 0) L->pos[L->order[q]] = q;
  L->J = log2p1(L->nq[0]) - log2p1(coarsest) + 1;
  L->m.assign(L->J, 0); L->k.assign(L->J, 0); L->lo.assign(L->J, 0);
  for (int j = 0, mj = L->nq[0]; j < L->J; ++j, mj = (mj - 1) / 2) {
    L->m[j] = mj;
    int kj = 0, lj = 0;
    for (int q = 0; q < count; ++q) {
      kj += L->nq[q] >= mj;
      lj += L->nq[q] > mj;
    }
    L->k[j] = kj;
    L->lo[j] = lj;
  }
  const size_t xb = L->xbytes(), sbb = L->sbytes(), ub = o.u_dtype == MGCNN_U_F64 ? 8 : 4;
  int r;
  size_t max_fine = 0;
  for (int j = 0; j < L->J; ++j)
    if (L->c(j) > 0) max_fine = std::max(max_fine, (size_t)L->m[j] * L->m[j] * L->c(j));
  if (!same_layout) {
    L->s.assign(L->J, nullptr); L->xin.assign(L->J, nullptr); L->xdn.assign(L->J, nullptr);
    L->u.assign(L->J, nullptr); L->a.assign(L->J, nullptr); L->f.assign(L->J, nullptr);
    L->rt.assign(L->J, nullptr); L->partial.assign(L->J, nullptr);
    for (int j = 0; j < L->J; ++j) {
      const size_t mm = (size_t)L->m[j] * L->m[j];
      const size_t cnt = mm * L->sl(L->k[j]) * C;
      if ((r = lalloc(L, &L->s[j], cnt * sbb)) || (r = lalloc(L, &L->xin[j], cnt * xb)) ||
          (r = lalloc(L, &L->xdn[j], cnt * xb)))
        return r;
      const int cj = L->c(j);
      if (cj == 0) continue;
      if ((r = lalloc(L, (void**)&L->a[j], mm * cj * 4)) || (r = lalloc(L, (void**)&L->f[j], mm * cj * 4)) ||
          (r = lalloc(L, (void**)&L->rt[j], mm * cj * 4)) || (r = lalloc(L, &L->u[j], mm * cj * ub)) ||
          (r = lalloc(L, (void**)&L->partial[j], (size_t)residual_tiles(L->m[j]) * cj * 8)))
        return r;
    }
    if ((r = lalloc(L, (void**)&L->d_b, (size_t)count * 8)) || (r = lalloc(L, (void**)&L->nf2, (size_t)count * 8)) ||
        (r = lalloc(L, (void**)&L->relres, (size_t)count * 8)) ||
        (r = lalloc(L, (void**)&L->active, (size_t)count * 4)) ||
        (r = lalloc(L, (void**)&L->status, (size_t)count * 4)) ||
        (r = lalloc(L, (void**)&L->iters, (size_t)count * 4)) ||
        (r = lalloc(L, (void**)&L->clock, (size_t)(count + 1) * 8)))
      return r;
  }
  hipStream_t st = L->stream;
  // coefficients and velocities in sorted order
  std::vector<float> bs((size_t)2 * count, 0.f);     // phantoms: b = 0
  for (int q = 0; q < count; ++q) {
    const int i = L->order[q];
    if (i < 0) continue;
    bs[2 * q] = b_host[2 * i];
    bs[2 * q + 1] = b_host[2 * i + 1];
  }
  LTRY(hipMemcpy(L->d_b, bs.data(), bs.size() * 4, hipMemcpyHostToDevice));
  for (int q = 0; q < count; ++q) {
    const int n = L->nq[q];
    int j = 0;
    while (L->m[j] != n) ++j;
    float* dst = L->a[j] + (size_t)(q - L->lo[j]) * n * n;
    if (L->order[q] >= 0)
      LTRY(hipMemcpyAsync(dst, a[L->order[q]], (size_t)n * n * 4, hipMemcpyDeviceToDevice, st));
    else   // phantom: a = 1 everywhere (bit pattern of 1.0f)
      LTRY(hipMemsetD32Async((hipDeviceptr_t)dst, (int)0x3f800000, (size_t)n * n, st));
  }
  // setup network (Alg. 2) over the aligned levels: reChannel of the features at each problem's
  // finest size, the restriction chain of the coefficient tensors down the sizes, then each tanh
  // layer as one launch over every level size (Setup2 does not couple the levels).  With f32
  // storage the level tensors hold the intermediates (c_j in xin_j, the layers ping-pong between
  // xdn_j and s_j and end in s_j); bf16 storage uses f32 level pyramids.
  const bool f32_store = L->xbytes() == 4 && sbb == 4;
  size_t pyr = 0;
  for (int j = 0; j < L->J; ++j) pyr += (size_t)L->m[j] * L->m[j] * L->sl(L->k[j]) * C;
  // temporaries (features of the largest finest group; with bf16 storage two f32 level pyramids)
  // are kept for the next setup and grown when a setup needs more
  const size_t need = max_fine * 4 * 4 + (f32_store ? 0 : 2 * pyr * 4);
  if (L->tmp_bytes < need) {
    if (L->tmp) (void)hipFree(L->tmp);
    L->tmp = nullptr;
    L->tmp_bytes = 0;
    if ((r = lalloc(L, (void**)&L->tmp, need))) return r;
    L->tmp_bytes = need;
  }
  float* F = L->tmp;
  float* tmp = L->tmp + max_fine * 4;
  auto W = [&](size_t off) { return (const float*)(L->d_w + off); };
  float *cl[MAX_LEVELS], *za[MAX_LEVELS], *zb[MAX_LEVELS];
  {
    float* p = tmp;
    for (int j = 0; j < L->J; ++j) {
      if (f32_store) {
        cl[j] = (float*)L->xin[j];
        za[j] = (float*)L->xdn[j];
        zb[j] = (float*)L->s[j];
      } else {
        cl[j] = p;            // c_j, then the second and fourth layers' output
        za[j] = p + pyr;
        zb[j] = p;
        p += (size_t)L->m[j] * L->m[j] * L->sl(L->k[j]) * C;
      }
    }
  }
  for (int j = 0; j < L->J; ++j) {
    const int mj = L->m[j], cj = L->c(j), lo = L->lo[j], kj = L->k[j];
    const size_t mm = (size_t)mj * mj;
    if (cj > 0) {
      launch_features(L->a[j], L->d_b + 2 * lo, F, mj, cj, o.op_form, st);
      if (L->pairs) launch_conv_in_pairs(F, W(L->off.setup_in), cl[j] + mm * (lo / 2) * C, mj, cj, st);
      else launch_conv_in(4, F, W(L->off.setup_in), cl[j] + mm * lo * C, ST_F32, mj, cj, nullptr, st);
    }
    if (j + 1 < L->J)
      launch_conv16(CM_RESTRICT, ST_F32, cl[j], nullptr, W(L->off.setup_restrict), nullptr, cl[j + 1], mj,
                    L->sl(kj), nullptr, st);
  }
  std::vector<int> slots_per_level(L->J);
  for (int j = 0; j < L->J; ++j) slots_per_level[j] = L->sl(L->k[j]);
  // float32-level products, or the two-way split with bf16 state (as mgcnn_setup)
  const StateType tanh_t = !o.f32_split ? ST_F32 : (L->xbytes() == 2 ? ST_F32X2 : ST_F32X);
  float** src[NUM_SETUP_LAYERS] = {cl, za, zb, za};
  float** dst[NUM_SETUP_LAYERS] = {za, zb, za, zb};
  for (int kk = 0; kk < NUM_SETUP_LAYERS; ++kk)
    launch_tanh_levels(tanh_t, src[kk], dst[kk], L->m.data(), slots_per_level.data(), L->J, W(L->off.res_w[kk]),
                       W(L->off.res_b[kk]), st);
  if (!f32_store)
    for (int j = 0; j < L->J; ++j)
      launch_f32_to_bf16(zb[j], (bf16_t*)L->s[j], (size_t)L->m[j] * L->m[j] * L->sl(L->k[j]) * C, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return lfail(L, MGCNN_E_HIP, std::string("group_setup: ") + hipGetErrorString(e));
  L->ready = true;
  return MGCNN_OK;
}

static int run_block(Ladder* L, double tol, int maxit, int chunk, bool graph) {
  if (!graph) {
    for (int it = 0; it < chunk; ++it) step(L, tol, maxit);
    LTRY(hipGetLastError());
    return MGCNN_OK;
  }
  if (!(L->gexec && L->g_tol == tol && L->g_maxit == maxit && L->g_chunk == chunk)) {
    drop_graph(L);
    LTRY(hipStreamBeginCapture(L->stream, hipStreamCaptureModeRelaxed));
    for (int it = 0; it < chunk; ++it) step(L, tol, maxit);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(L->stream, &g);
    if (e != hipSuccess) return lfail(L, MGCNN_E_HIP, std::string("group capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&L->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      L->gexec = nullptr;
      return lfail(L, MGCNN_E_HIP, std::string("group graph: ") + hipGetErrorString(e));
    }
    L->graph = g;
    L->g_tol = tol;
    L->g_maxit = maxit;
    L->g_chunk = chunk;
  }
  LTRY(hipGraphLaunch(L->gexec, L->stream));
  return MGCNN_OK;
}

int ladder_solve(Ladder* L, const float* const* f, void* const* u, double tol, int maxit,
                 int* iters_host, double* relres_host, int* status_host, hipStream_t user) {
  const mgcnn_opts& o = L->opts;
  const int count = L->count;
  const bool u64 = o.u_dtype == MGCNN_U_F64;
  const size_t ub = u64 ? 8 : 4;
  hipStream_t st = L->stream;
  if (int r = wait_on(L, user)) return r;
  auto slot = [&](int q, int* jq) {
    int j = 0;
    while (L->m[j] != L->nq[q]) ++j;
    *jq = j;
    return (size_t)(q - L->lo[j]) * L->m[j] * L->m[j];
  };
  for (int q = 0; q < count; ++q) {
    int j;
    const size_t off = slot(q, &j);
    const size_t nn = (size_t)L->m[j] * L->m[j];
    const int i = L->order[q];
    if (i < 0) {   // phantom: f = 0 (so u = 0 and the problem is done before the first step)
      LTRY(hipMemsetAsync(L->f[j] + off, 0, nn * 4, st));
      continue;
    }
    LTRY(hipMemcpyAsync(L->f[j] + off, f[i], nn * 4, hipMemcpyDeviceToDevice, st));
    LTRY(hipMemcpyAsync((char*)L->u[j] + off * ub, u[i], nn * ub, hipMemcpyDeviceToDevice, st));
  }
  // ||f||^2 per problem, solver state, u = 0 for a zero right-hand side, start clock
  for (int j = 0; j < L->J; ++j) {
    const int cj = L->c(j);
    if (cj == 0) continue;
    launch_residual(L->a[j], L->d_b + 2 * L->lo[j], L->f[j], nullptr, true, nullptr, L->partial[j], L->m[j],
                    cj, nullptr, o.op_form, st);
    launch_sum_partials(L->partial[j], residual_tiles(L->m[j]), L->nf2 + L->lo[j], cj, st);
  }
  launch_solve_init(L->nf2, L->active, L->status, L->iters, L->relres, count, st);
  for (int j = 0; j < L->J; ++j)
    if (L->c(j) > 0) launch_zero_if_zero_rhs(L->u[j], u64, L->nf2 + L->lo[j], L->m[j], L->c(j), st);
  launch_zero(L->clock, (size_t)count * 8, st);
  launch_clock_stamp(L->clock + count, st);
  LTRY(hipGetLastError());
  const bool graph = o.use_graph != 0;
  std::vector<int> act(count);
  int steps = 0;
  const int max_steps = maxit + 1;
  while (steps < max_steps) {
    const int chunk = std::min(std::max(o.check_every, 1), max_steps - steps);
    if (int r = run_block(L, tol, maxit, chunk, graph && chunk == o.check_every)) return r;
    steps += chunk;
    LTRY(hipMemcpyAsync(act.data(), L->active, (size_t)count * 4, hipMemcpyDeviceToHost, st));
    LTRY(hipStreamSynchronize(st));
    if (std::none_of(act.begin(), act.end(), [](int x) { return x != 0; })) break;
  }
  std::vector<int> sv(count), iv(count);
  std::vector<double> rv(count);
  std::vector<long long> ck(count + 1);
  LTRY(hipMemcpyAsync(sv.data(), L->status, (size_t)count * 4, hipMemcpyDeviceToHost, st));
  LTRY(hipMemcpyAsync(iv.data(), L->iters, (size_t)count * 4, hipMemcpyDeviceToHost, st));
  LTRY(hipMemcpyAsync(rv.data(), L->relres, (size_t)count * 8, hipMemcpyDeviceToHost, st));
  LTRY(hipMemcpyAsync(ck.data(), L->clock, (size_t)(count + 1) * 8, hipMemcpyDeviceToHost, st));
  for (int q = 0; q < count; ++q) {
    int j;
    const size_t off = slot(q, &j);
    const size_t nn = (size_t)L->m[j] * L->m[j];
    if (L->order[q] < 0) continue;
    LTRY(hipMemcpyAsync(u[L->order[q]], (const char*)L->u[j] + off * ub, nn * ub, hipMemcpyDeviceToDevice, st));
  }
  LTRY(hipStreamSynchronize(st));
  L->completion_s.assign(L->real, 0.0);
  bool diverged = false, notconv = false;
  for (int q = 0; q < count; ++q) {
    const int i = L->order[q];
    if (i < 0) continue;
    if (iters_host) iters_host[i] = iv[q];
    if (relres_host) relres_host[i] = rv[q];
    if (status_host) status_host[i] = sv[q];
    diverged |= sv[q] == MGCNN_E_DIVERGED;
    notconv |= sv[q] == MGCNN_NOT_CONVERGED;
    if (ck[q] > 0 && L->clock_khz > 0) L->completion_s[i] = (double)(ck[q] - ck[count]) / (1e3 * L->clock_khz);
  }
  if (diverged) return lfail(L, MGCNN_E_DIVERGED, "group_solve: a problem diverged");
  if (notconv) return MGCNN_NOT_CONVERGED;
  return MGCNN_OK;
}

}  // namespace mg
