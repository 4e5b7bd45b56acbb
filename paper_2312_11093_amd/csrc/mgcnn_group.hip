// Uneven-size batches: problems of different sizes in one call.
//
// The stationary iteration with the network preconditioner and a level count relative to the
// grid (opts.levels <= 0) runs on the aligned levels of mgcnn_ladder.h: one stream, one launch
// per operation and level size over the whole mixed batch.
//
// Every other configuration (FGMRES, PCG, the GMG preconditioner, a fixed level count) buckets
// the problems by size; each bucket is an ordinary batched problem set (its own context,
// workspace and HIP stream at the default priority).  Setup gathers the coefficients of a bucket
// into one contiguous batch; solve gathers f and u, runs the buckets' solves concurrently (one
// host thread per bucket, since a solve blocks its thread at every host check) and scatters u
// back.  Per problem the arithmetic is that of a batch of one on either path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_ladder.h"

namespace {

struct Bucket {
  int n = 0;
  std::vector<int> index;            // positions of the bucket's problems in the caller's arrays
  mgcnn_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  float* a = nullptr;                // [B][n][n]
  float* f = nullptr;                // [B][n][n]
  void* u = nullptr;                 // [B][n][n], f32 or f64
};

}  // namespace

struct mgcnn_group {
  mgcnn_opts opts{};
  std::vector<float> weights;
  hipStream_t user = nullptr;
  hipEvent_t ready = nullptr;
  std::vector<Bucket> buckets;
  int count = 0;
  mg::Ladder* lad = nullptr;         // aligned levels (stationary network iteration)
  std::string err;
};

namespace {

int gfail(mgcnn_group* g, int status, const std::string& msg) {
  g->err = msg;
  return status;
}

void free_buckets(mgcnn_group* g) {
  for (auto& k : g->buckets) {
    if (k.stream) (void)hipStreamSynchronize(k.stream);
    if (k.ctx) mgcnn_destroy(k.ctx);
    if (k.a) (void)hipFree(k.a);
    if (k.f) (void)hipFree(k.f);
    if (k.u) (void)hipFree(k.u);
    if (k.stream) (void)hipStreamDestroy(k.stream);
  }
  g->buckets.clear();
  g->count = 0;
}

size_t u_bytes(const mgcnn_group* g) { return g->opts.u_dtype == MGCNN_U_F64 ? 8 : 4; }

// Make every bucket stream wait for the work queued so far on the caller's stream.
int wait_user(mgcnn_group* g) {
  hipError_t e = hipEventRecord(g->ready, g->user);
  if (e != hipSuccess) return gfail(g, MGCNN_E_HIP, hipGetErrorString(e));
  for (auto& k : g->buckets) {
    e = hipStreamWaitEvent(k.stream, g->ready, 0);
    if (e != hipSuccess) return gfail(g, MGCNN_E_HIP, hipGetErrorString(e));
  }
  return MGCNN_OK;
}

}  // namespace

extern "C" {

int mgcnn_group_create(mgcnn_group** group, const mgcnn_opts* opts, const float* weights_host,
                       void* hip_stream) {
  if (!group) return MGCNN_E_ARG;
  *group = nullptr;
  mgcnn_opts o;
  if (opts) o = *opts; else mgcnn_default_opts(&o);
  // validate the options once with a throw-away context
  mgcnn_ctx* probe = nullptr;
  int r = mgcnn_create(&probe, &o, weights_host, hip_stream);
  if (r != MGCNN_OK) return r;
  mgcnn_destroy(probe);
  mgcnn_group* g = new (std::nothrow) mgcnn_group();
  if (!g) return MGCNN_E_NOMEM;
  g->opts = o;
  g->weights.assign(mgcnn_num_weights(o.channels), 0.f);
  if (weights_host) std::copy(weights_host, weights_host + g->weights.size(), g->weights.begin());
  g->user = (hipStream_t)hip_stream;
  if (hipEventCreateWithFlags(&g->ready, hipEventDisableTiming) != hipSuccess) {
    delete g;
    return MGCNN_E_HIP;
  }
  if (mg::ladder_supported(o)) {
    g->lad = new (std::nothrow) mg::Ladder();
    if (!g->lad) { (void)hipEventDestroy(g->ready); delete g; return MGCNN_E_NOMEM; }
    r = mg::ladder_create(g->lad, o, g->weights.data());
    if (r != MGCNN_OK) {
      mg::ladder_free(g->lad);
      delete g->lad;
      (void)hipEventDestroy(g->ready);
      delete g;
      return r;
    }
  }
  *group = g;
  return MGCNN_OK;
}

int mgcnn_group_setup(mgcnn_group* g, const float* const* a, const float* b_host, const int* n_host,
                      int count) {
  if (!g) return MGCNN_E_ARG;
  if (!a || !b_host || !n_host || count < 1) return gfail(g, MGCNN_E_ARG, "group_setup: bad argument");
  for (int i = 0; i < count; ++i)
    if (!a[i]) return gfail(g, MGCNN_E_ARG, "group_setup: null coefficient pointer");
  free_buckets(g);
  if (g->lad) {
    g->count = 0;
    int r = mg::ladder_setup(g->lad, a, b_host, n_host, count, g->user);
    if (r != MGCNN_OK) return gfail(g, r, g->lad->err);
    g->count = count;
    return MGCNN_OK;
  }
  std::map<int, std::vector<int>> by_n;
  for (int i = 0; i < count; ++i) by_n[n_host[i]].push_back(i);
  for (auto& kv : by_n) {
    Bucket k;
    k.n = kv.first;
    k.index = kv.second;
    g->buckets.push_back(k);
  }
  g->count = count;
  for (auto& k : g->buckets) {
    if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess)
      return gfail(g, MGCNN_E_HIP, "group_setup: stream creation failed");
    int r = mgcnn_create(&k.ctx, &g->opts, g->weights.data(), k.stream);
    if (r != MGCNN_OK) return gfail(g, r, "group_setup: context creation failed");
  }
  int r = wait_user(g);
  if (r) return r;
  for (auto& k : g->buckets) {
    const int B = (int)k.index.size();
    const size_t nn = (size_t)k.n * k.n;
    if (k.n < 3 || k.n > 4095 || ((k.n + 1) & k.n) != 0)
      return gfail(g, MGCNN_E_SIZE, "group_setup: n must be 2^L - 1 in [3, 4095]");
    if (hipMalloc((void**)&k.a, nn * B * 4) != hipSuccess || hipMalloc((void**)&k.f, nn * B * 4) != hipSuccess ||
        hipMalloc(&k.u, nn * B * u_bytes(g)) != hipSuccess)
      return gfail(g, MGCNN_E_NOMEM, "group_setup: out of device memory");
    std::vector<float> bb((size_t)2 * B);
    for (int q = 0; q < B; ++q) {
      const int i = k.index[q];
      bb[2 * q] = b_host[2 * i];
      bb[2 * q + 1] = b_host[2 * i + 1];
      if (hipMemcpyAsync(k.a + nn * q, a[i], nn * 4, hipMemcpyDeviceToDevice, k.stream) != hipSuccess)
        return gfail(g, MGCNN_E_HIP, "group_setup: copy failed");
    }
    // mgcnn_setup copies the velocities into its pinned staging buffer before it returns
    r = mgcnn_setup(k.ctx, k.a, bb.data(), k.n, B);
    if (r != MGCNN_OK) return gfail(g, r, std::string("group_setup: ") + mgcnn_last_error(k.ctx));
  }
  for (auto& k : g->buckets)
    if (hipStreamSynchronize(k.stream) != hipSuccess) return gfail(g, MGCNN_E_HIP, "group_setup: sync failed");
  return MGCNN_OK;
}

int mgcnn_group_solve(mgcnn_group* g, const float* const* f, void* const* u, double tol, int maxit,
                      int* iters_host, double* relres_host, int* status_host) {
  if (!g) return MGCNN_E_ARG;
  if (g->lad ? !g->lad->ready : g->buckets.empty())
    return gfail(g, MGCNN_E_STATE, "group_solve: call mgcnn_group_setup first");
  if (!f || !u) return gfail(g, MGCNN_E_ARG, "group_solve: null pointer");
  for (int i = 0; i < g->count; ++i)
    if (!f[i] || !u[i]) return gfail(g, MGCNN_E_ARG, "group_solve: null problem pointer");
  if (!(tol > 0.0) || maxit < 0) return gfail(g, MGCNN_E_ARG, "group_solve: need tol > 0 and maxit >= 0");
  if (g->lad) {
    if (!g->lad->ready) return gfail(g, MGCNN_E_STATE, "group_solve: call mgcnn_group_setup first");
    int r = mg::ladder_solve(g->lad, f, u, tol, maxit, iters_host, relres_host, status_host, g->user);
    if (r != MGCNN_OK && r != MGCNN_NOT_CONVERGED) return gfail(g, r, g->lad->err);
    return r;
  }
  int r = wait_user(g);
  if (r) return r;
  const size_t ub = u_bytes(g);
  for (auto& k : g->buckets) {
    const size_t nn = (size_t)k.n * k.n;
    for (int q = 0; q < (int)k.index.size(); ++q) {
      const int i = k.index[q];
      if (hipMemcpyAsync(k.f + nn * q, f[i], nn * 4, hipMemcpyDeviceToDevice, k.stream) != hipSuccess ||
          hipMemcpyAsync((char*)k.u + nn * ub * q, u[i], nn * ub, hipMemcpyDeviceToDevice, k.stream) != hipSuccess)
        return gfail(g, MGCNN_E_HIP, "group_solve: copy failed");
    }
  }
  const int nb = (int)g->buckets.size();
  std::vector<int> rc(nb, MGCNN_OK);
  std::vector<std::vector<int>> it(nb), st(nb);
  std::vector<std::vector<double>> rr(nb);
  auto run = [&](int w) {
    Bucket& k = g->buckets[w];
    const int B = (int)k.index.size();
    it[w].assign(B, 0); st[w].assign(B, 0); rr[w].assign(B, 0.0);
    rc[w] = mgcnn_solve(k.ctx, k.f, k.u, tol, maxit, it[w].data(), rr[w].data(), st[w].data());
  };
  {
    std::vector<std::thread> th;
    for (int w = 1; w < nb; ++w) th.emplace_back(run, w);
    run(0);
    for (auto& t : th) t.join();
  }
  bool diverged = false, notconv = false;
  int hard = MGCNN_OK;
  std::string msg;
  for (int w = 0; w < nb; ++w) {
    Bucket& k = g->buckets[w];
    if (rc[w] < 0 && rc[w] != MGCNN_E_DIVERGED && hard == MGCNN_OK) {
      hard = rc[w];
      msg = mgcnn_last_error(k.ctx);
    }
    const size_t nn = (size_t)k.n * k.n;
    for (int q = 0; q < (int)k.index.size(); ++q) {
      const int i = k.index[q];
      if (iters_host) iters_host[i] = it[w][q];
      if (relres_host) relres_host[i] = rr[w][q];
      if (status_host) status_host[i] = st[w][q];
      diverged |= st[w][q] == MGCNN_E_DIVERGED;
      notconv |= st[w][q] == MGCNN_NOT_CONVERGED;
      if (hipMemcpyAsync(u[i], (const char*)k.u + nn * ub * q, nn * ub, hipMemcpyDeviceToDevice, k.stream) !=
          hipSuccess)
        return gfail(g, MGCNN_E_HIP, "group_solve: copy failed");
    }
  }
  for (auto& k : g->buckets)
    if (hipStreamSynchronize(k.stream) != hipSuccess) return gfail(g, MGCNN_E_HIP, "group_solve: sync failed");
  if (hard != MGCNN_OK) return gfail(g, hard, "group_solve: " + msg);
  if (diverged) return gfail(g, MGCNN_E_DIVERGED, "group_solve: a problem diverged");
  if (notconv) return MGCNN_NOT_CONVERGED;
  return MGCNN_OK;
}

int mgcnn_group_buckets(const mgcnn_group* g) {
  if (!g) return 0;
  if (g->lad) {
    int sizes = 0;
    for (int j = 0; j < g->lad->J; ++j) sizes += g->lad->c(j) > 0;
    return g->lad->ready ? sizes : 0;
  }
  return (int)g->buckets.size();
}

int mgcnn_group_completion_times(const mgcnn_group* g, double* seconds_host) {
  if (!g || !seconds_host) return MGCNN_E_ARG;
  if (!g->lad || (int)g->lad->completion_s.size() != g->count || g->count == 0) return MGCNN_E_STATE;
  std::copy(g->lad->completion_s.begin(), g->lad->completion_s.end(), seconds_host);
  return MGCNN_OK;
}

int mgcnn_group_aligned(const mgcnn_group* g) { return g && g->lad ? 1 : 0; }

const char* mgcnn_group_last_error(const mgcnn_group* g) { return g ? g->err.c_str() : "null group"; }

void mgcnn_group_destroy(mgcnn_group* g) {
  if (!g) return;
  free_buckets(g);
  if (g->lad) {
    mg::ladder_free(g->lad);
    delete g->lad;
  }
  if (g->ready) (void)hipEventDestroy(g->ready);
  delete g;
}

}  // extern "C"
