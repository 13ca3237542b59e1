// gg_diagnostics_noalloc: the FP64 diagnostics of gg_diagnostics with the
// reduction's partial records in a fixed device array of this file instead
// of memory the library allocates, for callers that cannot allocate.
#include <mutex>
#include <string>

#include "gg_kernels.h"
#include "gg_runtime.h"

using namespace gg;

namespace {

// Work-groups of the capped reduction: each folds every NOALLOC_GROUPS-th
// tile of the lattice, so the array holds the same number of partial
// records whatever the lattice size.
constexpr int NOALLOC_GROUPS = REDUCE_GROUPS;  // the same order of sums as gg_diagnostics
constexpr int SCRATCH_DOUBLES = 6 * NOALLOC_GROUPS + 8;  // partials, then totals

// Per device: each GPU holds its own copy at its own address until the
// process ends. In host code `scratch` names a host-side stand-in, never a
// device address: kernels and copies take the address from
// hipGetSymbolAddress (scratch_on).
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev (current when called), looked
// up once per device.
hipError_t scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = (double *)g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" gg_status gg_diagnostics_noalloc(gg_lattice *L, gg_diag *out) {
  if (!L || !out) return gg_fail(GG_ERR_ARG, "NULL argument");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return gg_fail(GG_ERR_HIP, "hipGetDevice failed");
  if (cur != L->device && hipSetDevice(L->device) != hipSuccess)
    return gg_fail(GG_ERR_HIP, "cannot make the lattice's device current");
  double *sc = nullptr;
  hipError_t e = scratch_on(L->device, &sc);
  gg_status st = GG_OK;
  if (e != hipSuccess) st = gg_fail(GG_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  double rec[8 + 2 * GG_MAX_SEGMENTS] = {};
  int64_t t = 0;
  if (st == GG_OK) {
    // every partial record of the launched groups and the totals [0..5] are
    // written by the reduction, so nothing is cleared first; acc[6..7] are
    // not used
    double *partial = sc, *acc = sc + 6 * NOALLOC_GROUPS;
    if (L->n_aux_tiles > 0)
      e = launch_reduce(L->storage, L->d_desc, L->d_aux_tiles, L->n_aux_tiles, 6, partial, acc,
                        L->stream, NOALLOC_GROUPS);
    if (e == hipSuccess && L->n_aux_tiles > 0)
      e = hipMemcpyAsync(rec, acc, 6 * sizeof(double), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(rec + 8, L->d_flux, 2 * GG_MAX_SEGMENTS * sizeof(double),
                         hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&t, L->d_t, sizeof(t), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) st = gg_fail(GG_ERR_HIP, std::string("diagnostics: ") + hipGetErrorString(e));
  }
  if (cur != L->device) (void)hipSetDevice(cur);
  if (st != GG_OK) return st;
  gg_fill_diag(L, rec, rec + 8, t, out);
  if (out->n_nonfinite > 0)
    return gg_fail(GG_ERR_NONFINITE,
                   std::to_string(out->n_nonfinite) + " fluid nodes hold non-finite populations");
  return GG_OK;
}
