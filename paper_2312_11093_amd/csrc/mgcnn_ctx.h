// Internal definition of the library context shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_internal.h"

struct mgcnn_ctx {
  mgcnn_opts opts{};
  hipStream_t stream = nullptr;
  mg::WeightOffsets off{};
  float* d_w = nullptr;
  std::string err;

  // problem set
  int n = 0, B = 0, L = 0;
  int alloc_n = 0, alloc_B = 0;
  std::vector<int> nl;
  float* d_a = nullptr;
  float* d_b = nullptr;
  std::vector<void*> s, xin, xdn;
  float* d_rt = nullptr;
  double* d_partial = nullptr;
  int tiles = 0;
  double* d_nf2 = nullptr;
  int* d_active = nullptr;          // per-problem flags of the stationary solve
  int* d_plist = nullptr;           // compact list of the problems still iterating
  int plist_count = 0;              // its length (the grid size of the solver launches)
  // packed pairs (opts.pack_pairs): slot b of every state tensor holds problems 2b and 2b + 1
  int slots = 0;                    // state-tensor slots: B, or (B + 1) / 2 with packed pairs
  int* d_slist = nullptr;           // packed pairs: compact list of the slots with a live problem
  int slist_count = 0;
  int* d_status = nullptr;
  int* d_iters = nullptr;
  double* d_relres = nullptr;
  bool ready = false;
  // setup: the host velocities go through a pinned staging buffer (the caller's array need not
  // outlive the call; the event guards the buffer against reuse before its copy has run), and
  // the setup network's temporaries are kept for the next setup of the same size
  float* h_bstage = nullptr;
  int bstage_cap = 0;
  hipEvent_t bstage_ev = nullptr;
  bool bstage_pending = false;
  void* setup_tmp = nullptr;

  // per-launch profiling (HIP events around every kernel launch of the solve loop)
  struct ProfRec { int kind, level; double bytes, flops; hipEvent_t e0, e1; };
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<mgcnn_kernel_stat> agg;   // records already folded in (bytes_per_launch holds the sum)
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;

  // hipGraph of one block of `check_every` solver iterations (replayed while problems are live)
  struct GraphCache {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* f = nullptr;
    void* u = nullptr;
    double tol = 0.0;
    int maxit = -1, chunk = 0, gen = -1, count = -1, scount = -1;
  } gcache;
  int gen = 0;                      // bumped whenever problem buffers are reallocated
  hipStream_t cap_stream = nullptr; // capture stream used when the context stream is the null stream
  hipEvent_t join_ev = nullptr;

  // Krylov (FGMRES) workspace
  struct Krylov {
    int n = 0, B = 0, m = 0;
    float* V = nullptr;       // (m+1) Arnoldi vectors [B][n][n]
    float* Z = nullptr;       // m preconditioned vectors
    double* partial = nullptr;
    double* h = nullptr;      // per-problem inner products returned to the host
    double* s = nullptr;      // per-problem scale factors / combination coefficients
    int* act = nullptr;       // problems extending their basis
    int* cyc = nullptr;       // problems live in the current restart cycle
    int* grp = nullptr;       // problems restarting with deflation vectors
    double* coef = nullptr;   // deflation: basis combination coefficients (V, then Z)
  } kr;

  // preconditioned conjugate gradients: r, p, q, z and the diagonal scaling, [B][n][n] each
  struct Pcg {
    int n = 0, B = 0;
    float* vec = nullptr;     // 5 vectors of B * n * n floats: r, p, q, z, dsc
    float* ones = nullptr;    // B * krylov_vpad(n) ones (input of the diagonal pass)
    double* partial = nullptr;
    double* out = nullptr;    // 2 per problem: |r|^2 or (p, A p), then (r, z)
    double* coef = nullptr;   // 2 per problem: alpha, beta
    double* unit = nullptr;   // B * KRYLOV_LD ones (the diagonal pass's scale factors)
    int* lists = nullptr;     // three compact problem lists of B entries each
  } pcg;

  // geometric multigrid preconditioner (opts.precond == MGCNN_PRECOND_GMG), per level l
  struct Gmg {
    int levels = 0;
    std::vector<int> nl;                       // side of level l
    std::vector<float*> a;                     // injected coefficient (l >= 1; level 0 is d_a)
    std::vector<float*> rhs;                   // restricted residual (l >= 1; level 0 is d_rt)
    std::vector<float*> pre;                   // correction after the pre-sweeps (l < levels-1)
    std::vector<float*> cor;                   // final correction (l >= 1)
    double* inv = nullptr;                     // [B][N][N] inverse of the coarsest operator^T
  } gmg;

  // training: recorded forward (checkpoints of u_0..u_{K-1}) and reverse-pass workspace
  struct Train {
    int alloc_n = 0, alloc_B = 0, alloc_K = 0;
    int K = 0;                       // iterations recorded by the last forward(record)
    const float* f = nullptr;        // right-hand side of the recorded forward (caller-owned)
    float* uk = nullptr;             // [K][B][n][n] checkpoints
    std::vector<float*> xin, xdn, v, xup, g1, g2, gs;   // per level, [B][m][m][16]
    std::vector<float*> c, gc;       // setup: coefficient tensors and their gradients per level
    std::vector<float*> z, t;        // setup: layer inputs / tanh outputs, [level * 4 + k]
    float *F = nullptr, *gz0 = nullptr, *gz1 = nullptr;
    float *grt = nullptr, *lam0 = nullptr, *lam1 = nullptr, *r = nullptr;
    float* grad = nullptr;           // [num_weights]
    float* partial = nullptr;        // weight-gradient partial sums
    size_t partial_floats = 0;
    double* d_loss = nullptr;
    double* d_rr = nullptr;
  } tr;

  size_t state_bytes() const { return opts.state_dtype == MGCNN_BF16 ? 2 : 4; }
  // setup tensors s_l in bf16 (bf16 state, or f32 state with opts.s_bf16)
  bool s16() const { return opts.state_dtype == MGCNN_BF16 || opts.s_bf16 != 0; }
  size_t s_bytes() const { return s16() ? 2 : 4; }
  mg::StateType st() const {
    if (opts.state_dtype == MGCNN_BF16) return mg::ST_BF16;
    return opts.f32_split ? mg::ST_F32X : mg::ST_F32;
  }
  bool u64() const { return opts.u_dtype == MGCNN_U_F64; }
  bool pairs() const { return opts.pack_pairs != 0; }
  bool gmg_on() const { return opts.precond == MGCNN_PRECOND_GMG; }
  int form() const { return opts.op_form; }
  const float* W(size_t o) const { return d_w + o; }
};


namespace mg {
namespace api {

int fail(mgcnn_ctx* ctx, int code, const std::string& msg);
int hip_fail(mgcnn_ctx* ctx, hipError_t e, const char* what);
int alloc(mgcnn_ctx* c, void** p, size_t bytes);
hipEvent_t pool_event(mgcnn_ctx* c);
// Fold completed profiling records into c->agg and recycle their events (stream synchronised).
int prof_drain(mgcnn_ctx* c);
// list/count: the problems the launches cover (list null: all c->B); flags (optional): problems
// whose flag is 0 keep u unchanged.
int vcycle(mgcnn_ctx* c, void* u, bool u_f64, const int* list, int count, bool accumulate = true,
           const int* flags = nullptr);
int forward_record(mgcnn_ctx* c, const float* f, float* u, int K);
void free_train(mgcnn_ctx* c);
void free_krylov(mgcnn_ctx* c);
void free_pcg(mgcnn_ctx* c);
int pcg_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
              double* relres_host, int* status_host);
int fgmres_solve(mgcnn_ctx* c, const float* f, void* u, double tol, int maxit, int* iters_host,
                 double* relres_host, int* status_host);

#define HIP_TRY(ctx, call)                                            \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) return mg::api::hip_fail((ctx), e_, #call); \
  } while (0)

#define LAUNCH_CHECK(ctx)                                                      \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess) return mg::api::hip_fail((ctx), e_, "kernel launch"); \
  } while (0)

// Record events around one launch when profiling is on.
struct Prof {
  mgcnn_ctx* c;
  mgcnn_ctx::ProfRec r{};
  bool on;
  Prof(mgcnn_ctx* c_, int kind, int level, double bytes, double flops = 0.0) : c(c_), on(c_->prof) {
    if (!on) return;
    r.kind = kind; r.level = level;
    r.bytes = bytes;
    r.flops = flops;
    r.e0 = pool_event(c); r.e1 = pool_event(c);
    if (!r.e0 || !r.e1) { on = false; return; }
    (void)hipEventRecord(r.e0, c->stream);
  }
  ~Prof() {
    if (!on) return;
    (void)hipEventRecord(r.e1, c->stream);
    c->recs.push_back(r);
  }
};

}  // namespace api
}  // namespace mg
