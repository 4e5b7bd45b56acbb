/*
 * mgcnn.h -- C interface of the MI355X (gfx950) MGCNN solver library (libmgcnn.so).
 *
 * MGCNN (Xie, Lv, Zhang, "MGCNN: a learnable multigrid solver for sparse linear systems
 * from PDEs on structured grids") solves A(a,b) u = f, the zero-Dirichlet discretisation of
 *     -div(a grad u) + b . grad u = f   on the unit square, n x n interior nodes,
 * with the stationary iteration u_{k+1} = u_k + B(f - A u_k) (Sec. 2.2, Eq. (1)), where B is
 * a learned, linear multilevel convolutional network (the "decoder" of Sec. 2.1).  B is
 * built once per problem from a (setup phase, Sec. 3.2, Alg. 2) and applied every iteration
 * (solve phase, Sec. 3.3, Alg. 3).  Training minimises the residual loss (Sec. 3.4, Eq. (19)).
 *
 * Conventions shared by every entry point
 *   - Grid: n = 2^L - 1 (3 <= n <= 4095), h = 1/(n+1), L = log2(n+1) levels, level l has
 *     2^(L-l+1) - 1 points per side, the coarsest is 1 x 1.
 *   - Fields are row-major [batch][n][n] (index i*n + j, j along +x, i along +y), contiguous,
 *     16-byte aligned, in DEVICE memory owned by the caller.  `b` (the constant velocity of
 *     each problem, [batch][2] = (bx, by)) is in HOST memory.
 *   - Operator: 5-point diffusion plus first-order upwind convection (Sec. 2.5, Eqs. (8)-(12)),
 *     physical scaling 1/h^2 and 1/h; by default the divergence form with harmonic-mean face
 *     coefficients (a boundary face uses the interior node's a), or the non-divergence form of
 *     Eq. (7) (opts.op_form).  D = diag(A).  The network acts on the row-scaled residual
 *     (f - A u) / D.
 *   - Weights: one flat float32 host vector of mgcnn_num_weights(16) = 21664 entries in the
 *     order: setup reChannel [16][4][3][3]; 4 x (setup ResNet conv [16][16][3][3], bias [16]);
 *     setup restriction [16][16][3][3]; solve reChannel-in [16][1][3][3]; down smoother, up
 *     smoother, restriction [16][16][3][3]; prolongation (transposed conv, [C_in][C_out][3][3]);
 *     reChannel-out [1][16][3][3].  Convolutions are cross-correlations with zero padding 1
 *     (same size) or no padding (stride 2, n -> (n-1)/2 and back to 2m+1).
 *   - Streams: every call enqueues on the context's HIP stream and returns without a host
 *     synchronisation unless stated.  A context is not thread-safe; contexts are independent.
 *   - Errors: every call returns a status (never aborts).  Argument errors are detected before
 *     any launch.  mgcnn_last_error() gives a message for the last failure of a context.
 */
#ifndef MGCNN_H
#define MGCNN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgcnn_ctx mgcnn_ctx;

/* Status codes. */
enum {
  MGCNN_OK = 0,
  MGCNN_NOT_CONVERGED = 1,   /* maxit reached (solve) */
  MGCNN_E_ARG = -1,          /* invalid argument (null pointer, tol <= 0, maxit < 0, ...) */
  MGCNN_E_SIZE = -2,         /* n not of the form 2^L - 1, or outside [3, 4095], batch < 1 */
  MGCNN_E_STATE = -3,        /* call order violated (e.g. solve before setup) */
  MGCNN_E_NOMEM = -4,        /* device allocation failed */
  MGCNN_E_HIP = -5,          /* a HIP runtime call failed; see mgcnn_last_error */
  MGCNN_E_DIVERGED = -6,     /* relative residual non-finite or > 1e10 (solve) */
  MGCNN_E_NORECORD = -7,     /* backward without a recorded forward */
  MGCNN_E_SCRATCH = -8       /* mgcnn_residual_norms_noalloc: the input needs more scratch memory
                                than MGCNN_NOALLOC_SCRATCH_BYTES */
};

/* Precision of the network state, setup tensors and conv weights. */
enum { MGCNN_F32 = 0, MGCNN_BF16 = 1 };
/* Precision of u, of the residual arithmetic and of the stopping test. */
enum { MGCNN_U_F32 = 0, MGCNN_U_F64 = 1 };
/* Preconditioner B of the iteration (both outer methods). */
enum {
  MGCNN_PRECOND_NETWORK = 0,    /* the MGCNN solve network (Alg. 3) on the setup tensors (Alg. 2) */
  MGCNN_PRECOND_GMG = 1         /* the geometric multigrid baseline of Sec. 2.3 / Sec. 4.1: a V-cycle
                                   with the PDE rediscretised on every coarse grid (coefficient
                                   injected: a_c[I][J] = a[2I+1][2J+1], h doubled), bilinear
                                   prolongation, full-weighting restriction (P^T / 4), gmg_sweeps
                                   weighted-Jacobi sweeps (weight gmg_omega) before and after the
                                   coarse correction, exact solve on the coarsest grid.  B(r/D) is
                                   the cycle applied to r.  No weights, no setup network; training
                                   entry points return MGCNN_E_STATE. */
};
/* Form of the operator A(a, b) (both: 5-point diffusion + first-order upwind convection, zero
 * Dirichlet values, physical scaling 1/h^2 and 1/h). */
enum {
  MGCNN_OP_DIV = 0,     /* -div(a grad u) + b . grad u (Eq. (12)): the face coefficient between two
                           nodes is the harmonic mean of their a (a boundary face: the node's a) */
  MGCNN_OP_NONDIV = 1   /* -a (u_xx + u_yy) + b . grad u (Eq. (7), the form the paper computes
                           with): every face of row (i, j) takes a[i][j] */
};
/* Outer method of mgcnn_solve. */
enum {
  MGCNN_METHOD_STATIONARY = 0,  /* u += B((f - A u)/D), Sec. 2.2 Eq. (1) */
  MGCNN_METHOD_FGMRES = 1,      /* restarted flexible GMRES, B((.)/D) as right preconditioner (Sec. 2.2) */
  MGCNN_METHOD_PCG = 2          /* preconditioned conjugate gradients, the short recurrence that a
                                   symmetric operator and preconditioner allow (Sec. 2.2; the
                                   symmetric variant, Sec. 3.3).  Needs b = 0 and the divergence
                                   form (A symmetric positive definite; mgcnn_solve returns
                                   MGCNN_E_ARG for a problem with b != 0) and inner_steps = 1; the
                                   preconditioner is the GMG V-cycle, or the network with up_post = 1
                                   applied as D^-1/2 B(D^-1/2 r) (symmetric positive semi-definite
                                   when W_up, W_T and W_out are the adjoints of W_dn, W_R and W_in:
                                   every level is G^T (I + R^T M_coarse R) G with G the down
                                   smoother); mgcnn_create rejects the network without up_post.
                                   The f32 recurrence runs in cycles (an iterative refinement):
                                   each starts from the f64 true residual f - A u and ends when its
                                   recurrence residual has dropped by 1e-5, meets the tolerance or
                                   the step count reaches maxit; the true residual of u then decides
                                   the stopping rule.  iters counts the steps (u updates).
                                   (r, z) <= 0 or (p, A p) <= 0 (a preconditioner or weights that
                                   are not definite) ends the problem with MGCNN_E_DIVERGED */
};

typedef struct {
  int channels;     /* hidden channels; must be 16 */
  int state_dtype;  /* MGCNN_F32 or MGCNN_BF16 (bf16 storage, MFMA with f32 accumulation) */
  int u_dtype;      /* MGCNN_U_F32: u float32, residual in f32 arithmetic;
                       MGCNN_U_F64: u float64, residual in f64 arithmetic */
  int use_graph;    /* 1: capture each block of check_every iterations in a hipGraph */
  int check_every;  /* iterations between host convergence checks in mgcnn_solve (>= 1) */
  int method;       /* MGCNN_METHOD_STATIONARY or MGCNN_METHOD_FGMRES */
  int restart;      /* FGMRES restart length m, 1..63 (Krylov vectors are float32; the true
                       residual is recomputed in f64 at every restart); not used by PCG */
  int f32_split;    /* MGCNN_F32 state only: 1 = 16->16 convs on bf16 matrix cores with both
                       operands split into three bf16 parts (float32-level products, several
                       times the f32 matrix rate); 2 = as 1, but the finest down smoother (with
                       the reChannel-in conv folded in) splits into two bf16 parts: products to
                       about 2^-16 relative, half its f32 matrix time (a preconditioner setting:
                       the solve network is then not float32-exact); 0 = float32 matrix
                       instructions */
  int s_bf16;       /* MGCNN_F32 state only: 1 = keep the setup tensors s_l in bf16 (rounded once
                       after the setup network; the network stays a fixed linear operator, so a
                       solve still reaches its tolerance), halving their HBM traffic; 0 = f32 */
  int inner_steps;  /* FGMRES only: the preconditioner is this many steps (1..16) of the stationary
                       iteration of Eq. (1) on v from zero, z = B(v/D) then z += B((v - A z)/D) */
  int gs_passes;    /* FGMRES only: classical Gram-Schmidt applied 2 (default) or 1 times per
                       Arnoldi step */
  int precond;      /* MGCNN_PRECOND_NETWORK (default) or MGCNN_PRECOND_GMG */
  int gmg_levels;   /* GMG only: levels of the cycle; 0 (default) = log2(n+1) - 3, at least 1
                       (coarsest grid 15 x 15, as in Sec. 4.1); otherwise a value in
                       [max(1, log2(n+1) - 3), log2(n+1)] (the coarsest grid, solved exactly, has
                       at most 15 x 15 nodes), checked by mgcnn_setup (MGCNN_E_ARG) */
  int gmg_sweeps;   /* GMG only: sweeps before and after the coarse correction, 1..4 (default 3) */
  float gmg_omega;  /* GMG only: weighted-Jacobi weight, in (0, 2) (default 0.67) */
  int op_form;      /* MGCNN_OP_DIV (default) or MGCNN_OP_NONDIV: the operator of every call */
  int deflate;      /* FGMRES only: 0 = plain restarts; k in 1..32 with 2k <= restart = deflated
                       restarts: each restart keeps the k directions in which the preconditioned
                       operator of the finished cycle is smallest (right singular vectors of its
                       Hessenberg matrix) as the first k basis vectors of the next cycle.  The
                       bound on k leaves every cycle at least as many new Krylov vectors as kept
                       ones (with only a few new ones per cycle the iteration can stagnate);
                       mgcnn_create rejects a larger k (MGCNN_E_ARG) */
  int levels;       /* network only: levels of the setup and solve networks.  0 (default) =
                       log2(n+1), coarsest grid 1 x 1; a negative value -d = log2(n+1) - d (-1 is
                       the count Sec. 4.1 uses: 4, 5, 6, ... levels for 31, 63, 127, ..., coarsest
                       3 x 3); a positive value = exactly that many levels.  The resulting count
                       must lie in [1, log2(n+1)], checked by mgcnn_setup (MGCNN_E_ARG); mgcnn_create
                       rejects values outside [-11, 12] */
  int up_post;      /* network only: 0 (default) = up smoother x + W_up * (s . x) as in Alg. 3;
                       1 = x + s . (W_up * x), the adjoint form of the down smoother: with W_up the
                       adjoint of W_dn (kernel flipped, channel axes swapped), W_T = W_R and W_out
                       the adjoint of W_in the solve network is a symmetric operator (the
                       symmetric variant of the remark in Sec. 3.3).  The recorded forward and
                       mgcnn_backward reject it (MGCNN_E_ARG) */
  int pack_pairs;   /* network, stationary method only: 0 (default); 1 = packed pairs for networks
                       of at most 8 hidden channels (Sec. 4.2 and Table 2 compare C = 4, 8, 12)
                       given in the 16-channel layout with channels 8..15 zero
                       (mgcnn_set_weights checks it: MGCNN_E_ARG otherwise).  Problems 2b and
                       2b + 1 then share one 16-channel state tensor, one in channels 0..7 and one
                       in channels 8..15, and the 16 -> 16 convolutions take the block-diagonal
                       weights diag(W8, W8): the same network per problem (up to the rounding of
                       the summation order) at half the state bytes per problem.  An odd batch
                       leaves the second half of the last pair empty.  Training entry points and
                       mgcnn_get_setup_tensor return MGCNN_E_STATE; mgcnn_create rejects it with
                       FGMRES, PCG, GMG or s_bf16 (MGCNN_E_ARG).  Groups take it too: on aligned
                       levels every size group is padded to an even count with phantom problems
                       (zero right-hand side), so that a pair never mixes two sizes */
} mgcnn_opts;

/* Default options: 16 channels, f32 state (split-bf16 matrix arithmetic), f64 u, graphs off,
 * check every 4 iterations, stationary method, FGMRES restart 30, network preconditioner
 * (GMG settings: default levels, 3 sweeps, weight 0.67). */
void mgcnn_default_opts(mgcnn_opts *opts);

/* Number of weights for `channels` hidden channels: 81 C^2 + 58 C. */
size_t mgcnn_num_weights(int channels);

/* Create a context.  `weights_host` (may be NULL: all zero) is copied.  `hip_stream` is a
 * hipStream_t (NULL = default stream).  The context owns all device workspace. */
int mgcnn_create(mgcnn_ctx **ctx, const mgcnn_opts *opts, const float *weights_host,
                 void *hip_stream);

/* Replace the weights (copied from host).  The setup tensors of the current problem set are
 * NOT recomputed: call mgcnn_setup again.  A recorded forward (mgcnn_forward, record = 1) is
 * discarded: mgcnn_backward then returns MGCNN_E_NORECORD until the next recorded forward. */
int mgcnn_set_weights(mgcnn_ctx *ctx, const float *weights_host);

/* Change the stream used by subsequent calls. */
int mgcnn_set_stream(mgcnn_ctx *ctx, void *hip_stream);

/* Setup phase (Sec. 3.2, Alg. 2) for `batch` problems of side n: a [batch][n][n] device
 * (a > 0), b [batch][2] host.  The library copies a and b; neither need outlive the call (b is
 * copied into a pinned staging buffer of the context before the call returns; a by a
 * stream-ordered device copy).  The setup network's temporaries stay allocated in the context
 * for the next setup of the same size.  A recorded forward of the previous problem set is
 * discarded (mgcnn_backward returns MGCNN_E_NORECORD until the next recorded forward).
 * Computes and keeps the per-level setup tensors.  With MGCNN_PRECOND_GMG it builds the
 * multigrid hierarchy instead: the injected coefficient of every coarse level and the f64
 * inverse of the coarsest operator (8 N^2 bytes per problem, N = coarsest nodes <= 225). */
int mgcnn_setup(mgcnn_ctx *ctx, const float *a, const float *b_host, int n, int batch);

/* Tolerance-driven solve (Sec. 2.2, Eq. (1); stop on the relative residual as in Sec. 4.1).
 * f: [batch][n][n] float32 device.  u: [batch][n][n] device, float32 or float64 per
 * opts.u_dtype; on entry the initial guess, on exit the last iterate.
 * Per problem, at iterate k: rho_k = ||f - A u_k||_2 / ||f||_2; stop with OK if rho_k <= tol
 * (iters = k), NOT_CONVERGED if k == maxit, DIVERGED if rho_k is not finite or > 1e10;
 * otherwise apply one V-cycle.  A zero f gives u = 0, iters = 0, OK.
 * With opts.method = MGCNN_METHOD_FGMRES the same stopping rule is applied to the true
 * residual at every restart (and iters counts Arnoldi steps, each applying the network
 * opts.inner_steps times); the Arnoldi estimate
 * ends a restart cycle early.
 * iters_host [batch], relres_host [batch], status_host [batch] (each may be NULL) receive the
 * per-problem results.  Return: OK if every problem converged, else E_DIVERGED if any
 * diverged, else NOT_CONVERGED.  Blocks the host until the solve has finished. */
int mgcnn_solve(mgcnn_ctx *ctx, const float *f, void *u, double tol, int maxit,
                int *iters_host, double *relres_host, int *status_host);

/* K unrolled iterations, no stopping test (training / timing): u <- K applications of
 * u + B((f - A u)/D).  If record != 0 the iterates u_0..u_{K-1} are checkpointed for
 * mgcnn_backward (state must be MGCNN_F32 and u MGCNN_U_F32). */
int mgcnn_forward(mgcnn_ctx *ctx, const float *f, void *u, int K, int record);

/* Training (loss of Sec. 3.4, Eq. (19), after K unrolled iterations, normalised per problem):
 *   L = (1/batch) sum_i ||f_i - A_i u_i||^2 / ||f_i||^2.
 * mgcnn_loss: loss_host (may be NULL) receives L; dloss_du (device [batch][n][n], may be NULL)
 * receives dL/du = -2 A^T (f - A u) / (batch ||f||^2); dloss_df (may be NULL) receives the
 * partial derivative of L in f through this expression (u held fixed).  u must be float32
 * (opts.u_dtype = MGCNN_U_F32).  Blocks the host only when loss_host is given. */
int mgcnn_loss(mgcnn_ctx *ctx, const float *f, const float *u, double *loss_host, float *dloss_du,
               float *dloss_df);

/* Reverse pass through the K iterations recorded by the last mgcnn_forward(record = 1) and
 * through the setup network: given dL_du = dL/du_K (device [batch][n][n]), writes dL/dweights
 * (device, mgcnn_num_weights(16) floats, same order as the weights) and, if dL_df != NULL,
 * ADDS dL/df through the iterations into dL_df (device [batch][n][n]).  The right-hand side
 * passed to the recorded forward must still be valid.  Returns MGCNN_E_NORECORD without a
 * recorded forward for the current problem set.  Iterations are recomputed from the
 * checkpointed iterates u_0..u_{K-1} (one iteration's activations live at a time). */
int mgcnn_backward(mgcnn_ctx *ctx, const float *dL_du, float *dL_dweights, float *dL_df);

/* Replace the weights from DEVICE memory (training loops); asynchronous on the stream.  Like
 * mgcnn_set_weights it discards a recorded forward. */
int mgcnn_set_weights_device(mgcnn_ctx *ctx, const float *weights_dev);

/* Apply the network once: z = B(r / D) for a residual r [batch][n][n] float32 device;
 * z float32 device.  This is the linear preconditioner of Sec. 2.2 for Krylov methods. */
int mgcnn_apply(mgcnn_ctx *ctx, const float *r, float *z);

/* r = f - A u (float32 device [batch][n][n]; u per opts.u_dtype, arithmetic in f64). */
int mgcnn_residual(mgcnn_ctx *ctx, const float *f, const void *u, float *r);

/* Relative residuals ||f - A u|| / ||f|| per problem (u per opts.u_dtype); relres_host
 * [batch].  Blocks the host. */
int mgcnn_residual_norms(mgcnn_ctx *ctx, const float *f, const void *u, double *relres_host);

/* Levels of the GMG cycle of the current problem set (MGCNN_PRECOND_GMG after mgcnn_setup);
 * 0 otherwise. */
int mgcnn_gmg_levels(const mgcnn_ctx *ctx);

/* Copy the level-l setup tensor (l = 1..L) into `out` [batch][n_l][n_l][16] float32 device
 * (network preconditioner only). */
int mgcnn_get_setup_tensor(mgcnn_ctx *ctx, int level, float *out);

/* Per-launch profiling of the solve loop.  Between mgcnn_profile_begin and mgcnn_profile_end
 * every kernel launched by mgcnn_solve / mgcnn_forward / mgcnn_apply is bracketed by HIP
 * events on the context stream (graph capture is bypassed while profiling).  profile_end
 * synchronises and aggregates per (kernel kind, level): launch count, total milliseconds and
 * the algorithmic bytes one launch must move (compulsory reads + writes of its operands:
 * e.g. smoother 3 x 16 x state-bytes per node of its level).  Kinds: */
enum {
  MGCNN_K_RESIDUAL = 0, MGCNN_K_FINALIZE = 1, MGCNN_K_CONV_IN = 2, MGCNN_K_SMOOTH_DOWN = 3,
  MGCNN_K_RESTRICT = 4, MGCNN_K_SMOOTH_UP = 5, MGCNN_K_PROLONG = 6, MGCNN_K_OUT_UPDATE = 7,
  MGCNN_K_SMOOTH_IN = 8,   /* finest down smoother with the reChannel-in conv folded in */
  MGCNN_K_SMOOTH_OUT = 9,  /* reserved (no longer emitted) */
  /* FGMRES vector kernels; for DOTS, ORTH and COMBINE `level` holds the number of basis
     vectors the launch reads */
  MGCNN_K_KRYLOV_APPLY_A = 10, MGCNN_K_KRYLOV_DOTS = 11, MGCNN_K_KRYLOV_ORTH = 12,
  MGCNN_K_KRYLOV_SCALE = 13, MGCNN_K_KRYLOV_COMBINE = 14, MGCNN_K_KRYLOV_RESIDUAL = 15,
  MGCNN_K_SCALE_BY_DIAG = 16, MGCNN_K_ZERO = 17,
  /* GMG preconditioner: pre-sweeps + residual + restriction of one level; prolongation +
     post-sweeps of one level; exact solve on the coarsest grid */
  MGCNN_K_GMG_DOWN = 18, MGCNN_K_GMG_UP = 19, MGCNN_K_GMG_COARSE = 20
};
typedef struct {
  int kind;                /* MGCNN_K_* */
  int level;               /* 0 = finest */
  int launches;
  double ms_total;
  double bytes_per_launch; /* algorithmic HBM bytes (compulsory reads + writes) per launch */
  double flops_per_launch; /* algorithmic floating-point operations per launch (0 if not counted) */
} mgcnn_kernel_stat;
int mgcnn_profile_begin(mgcnn_ctx *ctx);
/* stats may be NULL (then only *n_stats is set); at most max_stats entries are written. */
int mgcnn_profile_end(mgcnn_ctx *ctx, mgcnn_kernel_stat *stats, int max_stats, int *n_stats);

/* ---- Stopping-test norms without allocation ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the relative residuals of mgcnn_residual_norms,
 * relres_host[i] = ||f_i - A_i u_i||_2 / ||f_i||_2 (0 when f_i = 0), with no context and no
 * allocation.  The kernels are those of mgcnn_residual_norms (same results bit for bit); their
 * scratch memory (velocities, per-tile partial sums of r^2 in f64, per-problem sums) is one
 * fixed array of MGCNN_NOALLOC_SCRATCH_BYTES per device, held by the library until the process
 * ends, which allows tiles(n) * batch + 2 * batch doubles plus the velocities, tiles(n) =
 * ceil(n / 256) * ceil(n / 8) (e.g. batch <= 2000 at n = 1023, <= 127 at n = 4095).
 *   a, f: [batch][n][n] float32 DEVICE; u: [batch][n][n] DEVICE, float32 or float64 per u_dtype
 *   (MGCNN_U_F32 / MGCNN_U_F64; the residual arithmetic follows u_dtype, f32 or f64, as in
 *   mgcnn_residual_norms); b_host:
 *   [batch][2] HOST velocities; op_form: MGCNN_OP_DIV or MGCNN_OP_NONDIV; relres_host: [batch]
 *   HOST output; hip_stream: hipStream_t of the work (NULL = default stream), on the current
 *   device.  Blocks the host until relres_host is written.
 * Returns MGCNN_E_ARG (null pointer, unknown form or u_dtype, non-finite velocity), MGCNN_E_SIZE
 * (n not 2^L - 1 in [3, 4095], batch < 1), MGCNN_E_SCRATCH (input larger than the scratch array;
 * nothing is launched), MGCNN_E_HIP.  Calls on one device share its scratch array: calls that
 * overlap in time on the same device (several host threads or streams) race and must be
 * serialised by the caller.  Every scratch word a call reads it has written first. */
#define MGCNN_NOALLOC_SCRATCH_BYTES (8u << 20)
int mgcnn_residual_norms_noalloc(const float *a, const float *b_host, int n, int batch,
                                 int op_form, const float *f, const void *u, int u_dtype,
                                 double *relres_host, void *hip_stream);

/* ---- Tile shapes (autotuning) ------------------------------------------------------------
 * The 16 -> 16 convolutions come in tile variants that differ only in the number of output rows
 * per workgroup (variant 0 = the default); the per-pixel arithmetic and its order are the same,
 * so every variant gives the same results bit for bit.  A process-wide table selects the variant
 * per operation, storage precision and level side m (levels of equal side share an entry).
 * paper_2312_11093_amd/autotune.py times the variants on the device and stores the fastest per
 * entry in a JSON file keyed by architecture; loading it fills this table.  Not thread-safe with
 * launches in flight on other host threads. */
enum { MGCNN_TILE_SMOOTHER = 0,   /* down (coarser levels) and up smoothers (Alg. 3) */
       MGCNN_TILE_RESTRICT = 1,   /* stride-2 restriction (RCNN) */
       MGCNN_TILE_SETUP = 2,      /* tanh layers of the setup network (Alg. 2; f32 only) */
       MGCNN_TILE_SMOOTH_IN = 3,  /* finest down smoother with the reChannel-in conv folded in */
       MGCNN_TILE_PROLONG = 4 };  /* transposed-conv prolongation (TCNN), keyed by the fine side */
#define MGCNN_TILE_VARIANTS 5
/* Select `variant` (0 .. MGCNN_TILE_VARIANTS - 1) for operation `op`, state_dtype MGCNN_F32 or
 * MGCNN_BF16 and level side m (1..4095); MGCNN_E_ARG on a bad argument or a variant the operation
 * does not have (the same-size convs and the finest down smoother have five: 8, 4, 16, 10, 12
 * rows; the restriction and the prolongation three). */
int mgcnn_set_tile_variant(int op, int state_dtype, int m, int variant);
/* The selected variant, or MGCNN_E_ARG. */
int mgcnn_tile_variant(int op, int state_dtype, int m);
/* Output rows per workgroup of a variant, or MGCNN_E_ARG. */
int mgcnn_tile_rows(int op, int state_dtype, int variant);

/* Number of levels of the current problem set (0 before setup). */
int mgcnn_levels(const mgcnn_ctx *ctx);

const char *mgcnn_status_string(int status);
const char *mgcnn_last_error(const mgcnn_ctx *ctx);
void mgcnn_destroy(mgcnn_ctx *ctx);

/* ---- Uneven-size batches ---------------------------------------------------------------
 * One call for problems of different sizes n_i = 2^k - 1 (each still the method of Sec. 2.2
 * and Alg. 2 / Alg. 3 per problem).  Results per problem are identical to solving that problem
 * on its own with the same options.  Two launch structures:
 *   - aligned levels (the stationary iteration with the network preconditioner and
 *     opts.levels <= 0): every hierarchy halves its side down to a coarsest side that does not
 *     depend on n, so the levels of all problems coincide in size from the coarsest up.  With
 *     the problems sorted by decreasing n, the problems having a level of side m are a prefix,
 *     and each level size is one batched tensor: every coarse-level operation of the V-cycle is
 *     one launch over all problems having that level, the finest-level operations (residual,
 *     reChannel-in smoother, reChannel-out update, stopping test) one launch per distinct size.
 *     One HIP stream, blocks of check_every iterations captured in a hipGraph when
 *     opts.use_graph; problems that have converged are held by their flag (u unchanged) until
 *     the whole batch has stopped.  Device timestamps of every problem's stop are kept
 *     (mgcnn_group_completion_times);
 *   - buckets (every other configuration): one batched problem set per size on its own HIP
 *     stream (default priority), solved concurrently, each from its own host thread. */
typedef struct mgcnn_group mgcnn_group;

/* Create a group: options and weights as for mgcnn_create (copied).  The group's streams are
 * its own; `hip_stream` (NULL = default) is the stream the inputs were produced on: setup and
 * solve wait for it before reading them. */
int mgcnn_group_create(mgcnn_group **group, const mgcnn_opts *opts, const float *weights_host,
                       void *hip_stream);
/* Setup for `count` problems: a[i] device pointer to the n_host[i] x n_host[i] coefficients of
 * problem i (a > 0), b_host [count][2].  Coefficients are copied into per-size buckets.
 * E_SIZE if some n is not 2^k - 1 or above 4095; E_ARG for null pointers or count < 1. */
int mgcnn_group_setup(mgcnn_group *group, const float *const *a, const float *b_host,
                      const int *n_host, int count);
/* Solve every problem of the last setup: f[i] (float32) and u[i] (float32 or float64 per
 * opts.u_dtype; initial guess in, last iterate out) are device pointers of problem i.  Stopping
 * rule, per-problem outputs and return value as for mgcnn_solve.  Blocks the host. */
int mgcnn_group_solve(mgcnn_group *group, const float *const *f, void *const *u, double tol,
                      int maxit, int *iters_host, double *relres_host, int *status_host);
/* Number of distinct problem sizes of the last setup (buckets, or finest sizes of the aligned
 * levels). */
int mgcnn_group_buckets(const mgcnn_group *group);
/* 1 if the group runs on aligned levels (one stream), 0 if on per-size buckets. */
int mgcnn_group_aligned(const mgcnn_group *group);
/* Aligned levels only: per problem (caller order), the seconds from the start of the last
 * mgcnn_group_solve's iterations (after ||f|| and the solver state are initialised) to the
 * device wall clock (wall_clock64) at which the stopping test ended that problem; 0 for a zero
 * right-hand side.  seconds_host [count] host.  MGCNN_E_STATE without such a solve. */
int mgcnn_group_completion_times(const mgcnn_group *group, double *seconds_host);
const char *mgcnn_group_last_error(const mgcnn_group *group);
void mgcnn_group_destroy(mgcnn_group *group);

#ifdef __cplusplus
}
#endif

#endif /* MGCNN_H */
