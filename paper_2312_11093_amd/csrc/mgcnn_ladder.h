// Uneven-size batches on one stream with the levels of all problems aligned by grid size.
//
// Every problem side is n = 2^p - 1 and its hierarchy halves the side (n -> (n-1)/2) down to a
// coarsest grid whose side does not depend on n (1 x 1, or 2^(d+1) - 1 with opts.levels = -d).
// So the problems of a mixed batch share their level sizes from the coarsest up: with the
// problems sorted by decreasing n, the problems that have a level of side m are a prefix of the
// sorted order, and every level size holds one batched tensor [k_m][m][m][16].  Each operation
// of a coarse level (down smoother, restriction, up smoother, prolongation) is then one batched
// launch over every problem that has that level; the finest-level operations (residual,
// reChannel-in down smoother, reChannel-out update, stopping test) are one launch per distinct
// problem size over the problems whose finest grid it is.  One stream, no host threads; blocks
// of iterations are captured in a hipGraph.
//
// Packed pairs (opts.pack_pairs, networks of at most 8 hidden channels): every size group is
// padded to an even count with phantom problems (zero right-hand side, unit coefficient, never
// copied back), so that sorted positions 2v and 2v + 1 always have the same finest size and share
// state slot v on every level they have.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mgcnn.h"
#include "mgcnn_internal.h"

namespace mg {

struct Ladder {
  mgcnn_opts opts{};
  WeightOffsets off{};
  float* d_w = nullptr;
  hipStream_t stream = nullptr;      // private, default priority
  int count = 0;                     // sorted positions (problems, plus phantoms with packed pairs)
  int real = 0;                      // the caller's problems
  bool pairs = false;                // packed pairs: two sorted positions per state slot
  std::vector<int> order;            // sorted position -> caller index (n descending, stable; -1 = phantom)
  std::vector<int> pos;              // caller index -> sorted position
  std::vector<int> nq;               // side of the problem at each sorted position
  int J = 0;                         // level sizes
  std::vector<int> m;                // side of level size j (descending)
  std::vector<int> k;                // problems that have level size j: sorted positions [0, k_j)
  std::vector<int> lo;               // first problem whose finest grid is m_j: [lo_j, k_j)
  // per level size j
  std::vector<void*> s, xin, xdn;    // [k_j][m][m][16]
  std::vector<float*> a, f, rt;      // finest fields of the problems [lo_j, k_j): [c_j][m][m]
  std::vector<void*> u;              // [c_j][m][m], f32 or f64
  std::vector<double*> partial;      // [c_j][tiles(m_j)]
  float* d_b = nullptr;              // velocities in sorted order [count][2]
  double* nf2 = nullptr;
  double* relres = nullptr;
  int *active = nullptr, *status = nullptr, *iters = nullptr;
  long long* clock = nullptr;        // [count + 1]: completion wall clock per problem, then start
  int clock_khz = 0;
  bool ready = false;
  hipGraphExec_t gexec = nullptr;    // one block of check_every iterations
  hipGraph_t graph = nullptr;
  double g_tol = -1.0;
  int g_maxit = -1, g_chunk = 0;
  std::vector<double> completion_s;  // per caller index, seconds from the start of the last solve
  float* tmp = nullptr;              // setup temporaries, kept across setups
  size_t tmp_bytes = 0;
  std::string err;

  int c(int j) const { return k[j] - lo[j]; }
  int sl(int q) const { return pairs ? q / 2 : q; }   // state slots of q sorted positions
  size_t sbytes() const;
  size_t xbytes() const;
};

// Whether the options take the aligned path: stationary iteration with the network
// preconditioner, a level count relative to the grid (opts.levels <= 0).
bool ladder_supported(const mgcnn_opts& o);
int ladder_create(Ladder* L, const mgcnn_opts& o, const float* weights_host);
int ladder_setup(Ladder* L, const float* const* a, const float* b_host, const int* n_host,
                 int count, hipStream_t user);
int ladder_solve(Ladder* L, const float* const* f, void* const* u, double tol, int maxit,
                 int* iters_host, double* relres_host, int* status_host, hipStream_t user);
void ladder_free(Ladder* L);

}  // namespace mg
