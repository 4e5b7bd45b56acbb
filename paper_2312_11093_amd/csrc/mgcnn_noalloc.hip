// mgcnn_residual_norms_noalloc: the relative residuals ||f - A u|| / ||f|| of a batch (the
// quantity of the stopping test of Sec. 4.1, on the operator of Sec. 2.5) without any device
// allocation, for callers that cannot allocate.  It runs the kernels of mgcnn_residual_norms;
// their scratch memory (the velocities, the per-tile partial sums and the two per-problem sums)
// lives in one file-scope device array instead of a context's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/mgcnn.h"
#include "mgcnn_internal.h"

using namespace mg;

namespace {

// One copy per device, held until the process ends.  In host code `scratch` names only a
// host-side stand-in of the symbol: its device address comes from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[MGCNN_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void* scratch_dev[MAX_DEVICES] = {};   // device address of `scratch` on each device

// Address of the current device's copy of `scratch`, looked up once per device (with that
// device current).
hipError_t scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[dev] = p;
  }
  *out = (unsigned char*)scratch_dev[dev];
  return hipSuccess;
}

size_t round256(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

}  // namespace

namespace mg {
namespace api {
bool valid_n(int n);
}
}  // namespace mg

extern "C" int mgcnn_residual_norms_noalloc(const float* a, const float* b_host, int n, int batch,
                                            int op_form, const float* f, const void* u,
                                            int u_dtype, double* relres_host, void* hip_stream) {
  if (!a || !b_host || !f || !u || !relres_host) return MGCNN_E_ARG;
  if (op_form != MGCNN_OP_DIV && op_form != MGCNN_OP_NONDIV) return MGCNN_E_ARG;
  if (u_dtype != MGCNN_U_F32 && u_dtype != MGCNN_U_F64) return MGCNN_E_ARG;
  if (!mg::api::valid_n(n) || batch < 1) return MGCNN_E_SIZE;
  for (int i = 0; i < 2 * batch; ++i)
    if (!std::isfinite(b_host[i])) return MGCNN_E_ARG;
  // scratch layout: velocities [batch][2] f32 | ||f||^2 [batch] | relres [batch] | partials
  const int tiles = residual_tiles(n);
  const size_t off_nf2 = round256((size_t)batch * 2 * sizeof(float));
  const size_t off_rel = off_nf2 + round256((size_t)batch * sizeof(double));
  const size_t off_par = off_rel + round256((size_t)batch * sizeof(double));
  const size_t need = off_par + (size_t)tiles * batch * sizeof(double);
  if (need > (size_t)MGCNN_NOALLOC_SCRATCH_BYTES) return MGCNN_E_SCRATCH;
  unsigned char* base = nullptr;
  if (scratch_address(&base) != hipSuccess) return MGCNN_E_HIP;
  float* d_b = (float*)base;
  double* d_nf2 = (double*)(base + off_nf2);
  double* d_rel = (double*)(base + off_rel);
  double* d_par = (double*)(base + off_par);
  hipStream_t s = (hipStream_t)hip_stream;
  // every scratch word read below is written first by this call: nothing needs clearing
  if (hipMemcpyAsync(d_b, b_host, (size_t)batch * 2 * sizeof(float), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return MGCNN_E_HIP;
  launch_residual(a, d_b, f, nullptr, true, nullptr, d_par, n, batch, nullptr, op_form, s);
  launch_sum_partials(d_par, tiles, d_nf2, batch, s);
  launch_residual(a, d_b, f, u, u_dtype == MGCNN_U_F64, nullptr, d_par, n, batch, nullptr, op_form,
                  s);
  launch_relres(d_par, tiles, d_nf2, d_rel, batch, s);
  if (hipGetLastError() != hipSuccess) return MGCNN_E_HIP;
  if (hipMemcpyAsync(relres_host, d_rel, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return MGCNN_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MGCNN_E_HIP;
  return MGCNN_OK;
}
