// Internal declarations of the reverse-mode (training) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace mg {

enum Geometry : int { GM_SAME = 0, GM_S2 = 1, GM_T2 = 2 };
enum PreMul : int { PM_NONE = 0, PM_MUL = 1, PM_TANHD = 2 };
enum Epilogue : int { EP_STORE = 0, EP_ADD = 1, EP_SKIP = 2, EP_SMOOTH_BWD = 3, EP_TANH_BIAS = 4 };

struct ConvArgs {
  const float* x = nullptr;     // input [B][mi][mi][ci]
  const float* m = nullptr;     // pre-multiplier at input pixels (PM_MUL / PM_TANHD)
  const float* W = nullptr;     // weights
  const float* bias = nullptr;  // EP_TANH_BIAS
  float* y = nullptr;           // output [B][mo][mo][co]
  const float* skip = nullptr;  // EP_SKIP / EP_SMOOTH_BWD
  const float* m2 = nullptr;    // EP_SMOOTH_BWD: multiplier of acc into y
  const float* m3 = nullptr;    // EP_SMOOTH_BWD: multiplier of acc into gs
  float* gs = nullptr;          // EP_SMOOTH_BWD accumulation target
  int mi = 0, mo = 0, ci = 0, co = 0, gm = 0, pm = 0, ep = 0, trans = 0, flip = 0;
  int tiles_x = 0, tiles_per_prob = 0;
};

struct WgradArgs {
  const float* A = nullptr;   // [B][ma][ma][ca]
  const float* Am = nullptr;  // PM_TANHD multiplier of A (t, uses 1 - t^2)
  const float* Bx = nullptr;  // [B][mb][mb][cb]
  const float* Bm = nullptr;  // PM_MUL multiplier of B
  float* partial = nullptr;   // [nblocks][ca*cb*9]
  int ma = 0, mb = 0, ca = 0, cb = 0, gm = 0, pmb = 0, pma = 0;
  int tiles_x = 0, tiles_per_prob = 0;
};

void launch_dconv(ConvArgs A, int B, hipStream_t st);
int launch_wgrad(WgradArgs G, int B, hipStream_t st);   // returns the number of partial rows
void launch_reduce_partials(const float* partial, int nblocks, int ne, float* out, bool accumulate,
                            hipStream_t st);
int launch_bias_grad(const float* g, const float* t, float* partial, size_t npx, hipStream_t st);
void launch_apply_AT(const float* a, const float* b, const float* v, const float* base,
                     const double* nf2, double alpha, bool div_by_diag, float* out, float* df_acc,
                     int n, int B, int form, hipStream_t st);
void launch_loss_finalize(const double* rr, const double* nf2, int B, double* loss, hipStream_t st);
void launch_loss_df(const float* r, const float* f, const double* rr, const double* nf2, float* df,
                    int n, int B, hipStream_t st);
void launch_residual_plain(const float* a, const float* b, const float* f, const void* u, bool u_f64,
                           float* r, int n, int B, int form, hipStream_t st);
void launch_add(const float* x, const float* z, float* y, size_t count, hipStream_t st);

}  // namespace mg
