// Internal declarations shared by the MGCNN HIP kernels and the C-ABI layer.
// Not part of the public interface (see include/mgcnn.h).
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mg {

constexpr int C = 16;                 // hidden channels of every state / setup tensor
constexpr int NUM_SETUP_LAYERS = 4;   // tanh ResNet layers of the setup network
constexpr int MAX_LEVELS = 12;        // levels of a 4095 x 4095 grid

// State of the solve network (x, s): storage type and matrix-core arithmetic.
//   ST_F32   float32 storage, float32 MFMA (16x16x4)
//   ST_BF16  bf16 storage, bf16 MFMA with f32 accumulation
//   ST_F32X  float32 storage, bf16 MFMA on a three-way bf16 split of both operands
//   ST_F32X2 float32 storage, bf16 MFMA on a two-way bf16 split (finest down smoother only)
//            (float32-level products at the bf16 matrix rate)
enum StateType : int { ST_F32 = 0, ST_BF16 = 1, ST_F32X = 2, ST_F32X2 = 3 };

// Offsets (in floats) of every parameter tensor inside the flat weight vector.
struct WeightOffsets {
  size_t setup_in, res_w[NUM_SETUP_LAYERS], res_b[NUM_SETUP_LAYERS], setup_restrict;
  size_t solve_in, smooth_down, smooth_up, restrict_, prolong, solve_out, total;
};
WeightOffsets weight_offsets();
namespace api {
// Packed pairs: the weights of a network with at most 8 hidden channels (16-channel layout,
// channels 8..15 unused) as block-diagonal 16-channel weights; false if channels 8..15 are used.
bool pack_pair_weights(const WeightOffsets& off, const float* w, std::vector<float>& out);
}  // namespace api

// bf16 storage: raw 16-bit pattern.
typedef uint16_t bf16_t;

// ---- launchers (all asynchronous on `st`) ------------------------------------------------
// Batch convention: `active` is either null (the launch covers problems 0..B-1) or a device
// list of B problem indices (the launch covers exactly those problems; retired problems are
// left out of the grid instead of being skipped by every workgroup).

// Operator form (`form` argument of every launcher that evaluates A): the face coefficient
// between a node and its neighbour is their harmonic mean (divergence form, Eq. (12)) or the
// node's own value (non-divergence form of Eq. (7)); public values MGCNN_OP_DIV / MGCNN_OP_NONDIV.

// Setup: stencil features F [B][n][n][4] (f32) from a [B][n][n] and b [B][2].
void launch_features(const float* a, const float* b, float* F, int n, int B, int form, hipStream_t st);

// Same-size 3x3 conv from CIN (1 or 4) channels to 16, zero padded.
//   in  [B][n][n][CIN] f32, W [16][CIN][3][3] f32, out [B][n][n][16] (f32 or bf16).
void launch_conv_in(int cin, const float* in, const float* W, void* out, StateType ot,
                    int n, int B, const int* active, hipStream_t st);

// C->C conv on MFMA.  mode: SMOOTH  y = x + W*(s.x)        (same size, s given)
//                           TANH    y = x + tanh(W*x + bias) (same size, f32 only)
//                           RESTRICT y = W *_{stride 2} x    (m -> (m-1)/2)
//                           SMOOTH_POST y = x + s . (W*x)  (same size, s given: the adjoint form)
enum ConvMode : int { CM_SMOOTH = 0, CM_TANH = 1, CM_RESTRICT = 2, CM_SMOOTH_POST = 3 };
// s_bf16: s is stored as bf16 while the state is f32 (smoother only).
void launch_conv16(ConvMode mode, StateType t, const void* x, const void* s, const float* W,
                   const float* bias, void* y, int m, int B, const int* active, hipStream_t st,
                   bool s_bf16 = false);

// Tile variants of the 16 -> 16 convolutions (process-wide table, autotuning): op = TILE_SMOOTHER
// (down / up smoothers), TILE_RESTRICT, TILE_SETUP (tanh layers), TILE_SMOOTH_IN (finest down
// smoother with reChannel-in), TILE_PROLONG (keyed by the fine side); variant 0 = the default.
enum TileOp : int { TILE_SMOOTHER = 0, TILE_RESTRICT = 1, TILE_SETUP = 2, TILE_SMOOTH_IN = 3,
                    TILE_PROLONG = 4, TILE_OPS = 5 };
constexpr int TILE_VARIANTS = 5;
int tile_variant_rows(int op, bool bf16, int variant);
int get_tile_variant(int op, bool bf16, int m);
void set_tile_variant(int op, bool bf16, int m, int variant);

// One tanh layer of the setup network on L levels in one launch: y_l = x_l + tanh(W * x_l + bias)
// for l < L, level l of side m[l] and batch B[l] (f32 storage; t = ST_F32 or ST_F32X).
void launch_tanh_levels(StateType t, const float* const* x, float* const* y, const int* m, const int* B,
                        int L, const float* W, const float* bias, hipStream_t st);

// y_fine += convT_{stride 2}(W_T, x_coarse), fine side m = 2 mc + 1, in place on y_fine.
void launch_prolong_add(StateType t, const void* xc, const float* WT, void* yf, int mc, int B,
                        const int* active, hipStream_t st);

// Finest-level down smoother with the reChannel-in conv folded in: y = x1 + W*(s.x1) with
// x1 = W_in * rt computed on the staged tile.  pairs: packed pairs (slot b = problems 2b and
// 2b + 1 in channels 0..7 / 8..15, rt [2 B][m][m], W_in's first eight rows; s in the state type).
void launch_smooth_in(StateType t, const float* rt, const void* s, const float* Win, const float* W,
                      void* y, int m, int B, const int* active, hipStream_t st, bool s_bf16 = false,
                      bool pairs = false);

// u += W_out * x (16 -> 1 same-size conv), u f32 or f64; u = W_out * x when !accumulate.
// flags (optional, indexed by problem): problems whose flag is 0 keep u unchanged.
void launch_out_update(StateType t, const void* x, const float* Wout, void* u, bool u_f64,
                       int n, int B, const int* active, hipStream_t st, bool accumulate = true,
                       const int* flags = nullptr);
// Packed pairs: `slots` slots (a list of slot indices in `active`, or all), problem 2b + h from
// channels 8h..8h+7 of slot b with W_out's first eight columns; nprob problems in u (an odd
// nprob leaves the last slot's second half unused); flags per problem.
void launch_out_update_pairs(StateType t, const void* x, const float* Wout, void* u, bool u_f64, int n,
                             int slots, int nprob, const int* active, hipStream_t st, bool accumulate,
                             const int* flags);
// Setup reChannel of packed pairs: F [nprob][n][n][4] -> out [(nprob + 1) / 2][n][n][16] (f32),
// problem 2b + h into channels 8h..8h+7 of slot b with the first eight rows of W.
void launch_conv_in_pairs(const float* in, const float* W, float* out, int n, int nprob, hipStream_t st);

// r = f - A(a,b) u ; rt = r / D (f32) ; partial[b][tile] = sum r^2 (f64).
// u == nullptr means u = 0.  mode64: u is f64 and the arithmetic is f64; otherwise u is f32 and
// the stencil arithmetic is f32 (the partial sums stay f64).
int residual_tiles(int n);
void launch_residual(const float* a, const float* b, const float* f, const void* u, bool u_f64,
                     float* rt, double* partial, int n, int B, const int* active, int form,
                     hipStream_t st);

// Per-problem stop test (one workgroup per problem).  On entry iters[b] = k of the current
// iterate.  Computes rho_k = sqrt(sum partial)/sqrt(nf2).  If nf2 is zero, rho = 0.
// Sets active/status/iters/relres following the solver's stopping rule.
// done_clock (optional): the device wall clock (wall_clock64) at which a problem stops.
void launch_finalize(const double* partial, int tiles, const double* nf2, double tol, int maxit,
                     int* active, int* status, int* iters, double* relres, int B, hipStream_t st,
                     long long* done_clock = nullptr);
// out[0] = the device wall clock (wall_clock64) when the kernel runs.
void launch_clock_stamp(long long* out, hipStream_t st);
// u = 0 for the problems whose ||f||^2 is zero.
void launch_zero_if_zero_rhs(void* u, bool u_f64, const double* nf2, int n, int B, hipStream_t st);

// nf2[b] = sum of partials (the squared norm of f), deterministic order.
void launch_sum_partials(const double* partial, int tiles, double* out, int B, hipStream_t st);
void launch_relres(const double* partial, int tiles, const double* nf2, double* relres, int B,
                   hipStream_t st);

// Convert f32 -> bf16 (round to nearest even), count elements.
void launch_f32_to_bf16(const float* in, bf16_t* out, size_t count, hipStream_t st);

// Zero fill (kernel, graph-capture safe).
void launch_zero(void* p, size_t bytes, hipStream_t st);

// Solve init: active[b] = (nf2[b] > 0), status = NOT_CONVERGED, iters = 0, relres = 0;
// problems with a zero right-hand side get u = 0 (zeroed by the caller), status OK.
void launch_solve_init(const double* nf2, int* active, int* status, int* iters, double* relres,
                       int B, hipStream_t st);

}  // namespace mg
