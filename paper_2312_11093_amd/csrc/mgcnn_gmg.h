// Internal declarations of the geometric multigrid baseline (kernels_gmg.hip, mgcnn_gmg.hip).
#pragma once

#include <hip/hip_runtime.h>

struct mgcnn_ctx;

namespace mg {

constexpr int GMG_MAX_SWEEPS = 4;        // pre- and post-sweeps per level
constexpr int GMG_MAX_COARSE_SIDE = 15;  // the coarsest grid is solved exactly: at most 15 x 15
constexpr int GMG_MAX_COARSE = 256;      // >= GMG_MAX_COARSE_SIDE^2 unknowns

// Output of the finest-level kernels: f32 or f64, store or add.
enum GmgOut : int { GMG_OUT_F32 = 0, GMG_OUT_F32_ADD = 1, GMG_OUT_F64 = 2, GMG_OUT_F64_ADD = 3 };

// `form`: the operator form (harmonic face coefficients or the node's own value), as for the
// other launchers.  Right-hand sides: `scaled` means rhs holds r / D (the finest level, which receives the
// row-scaled residual); otherwise rhs holds r.  Every launch covers the problems of `active`
// (null: 0..B-1); buffers are indexed by problem.

// e = nu weighted-Jacobi sweeps from zero on A e = r (m x m grid), and
// rc = full weighting of r - A e onto the (m-1)/2 x (m-1)/2 grid.
void launch_gmg_down(int nu, const float* a, const float* b, const float* rhs, bool scaled,
                     float omega, float* e, float* rc, int m, int B, const int* active, int form,
                     hipStream_t st);

// e = nu sweeps on A e = r from e_pre + P ec, written to `out` per `mode` (GmgOut); problems
// whose flag is 0 (flags non-null) keep `out` unchanged.
void launch_gmg_up(int nu, const float* a, const float* b, const float* rhs, bool scaled,
                   float omega, const float* e_pre, const float* ec, void* out, int mode,
                   const int* flags, int m, int B, const int* active, int form, hipStream_t st);

// inv[b] = (A_b^T)^-1 (f64, [B][N][N], N = mc^2) of the rediscretised operator on the coarsest
// grid; all B problems.
void launch_gmg_coarse_inverse(const float* a, const float* b, double* inv, int mc, int B,
                               int form, hipStream_t st);

// out = A^-1 r on the coarsest grid (per `mode`, `flags` as launch_gmg_up).
void launch_gmg_coarse_solve(const double* inv, const float* a, const float* b, const float* rhs,
                             bool scaled, void* out, int mode, const int* flags, int mc, int B,
                             const int* active, int form, hipStream_t st);

// ac[b][I][J] = a[b][2I+1][2J+1] (all B problems).
void launch_gmg_inject(const float* a, float* ac, int m, int B, hipStream_t st);

namespace api {
// levels of the cycle for side n under opts.gmg_levels; 0 if the option is out of range
int gmg_levels_for(const mgcnn_ctx* c, int n);
int gmg_alloc(mgcnn_ctx* c, int n, int B);
void gmg_free(mgcnn_ctx* c);
int gmg_setup(mgcnn_ctx* c);
int gmg_cycle(mgcnn_ctx* c, void* u, bool u_f64, const int* list, int count, bool accumulate,
              const int* flags);
}  // namespace api

}  // namespace mg
