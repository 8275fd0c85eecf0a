// fr_residual_noalloc: the stage residual of eq. (26) with its norms, for callers that cannot
// allocate device memory. The per-workgroup partial sums of the norm reduction, which
// fr_residual keeps in the level's workspace, live here in a file-scope device array instead;
// the call itself allocates nothing.
#include <mutex>

#include "../../include/pmgfr.h"
#include "internal.hpp"

namespace {

// partial sums of F^2: residual_blocks(L) x Nv doubles per call; 512 KiB per device, held by
// every device the library runs on until the process ends
constexpr size_t kScratchDoubles = size_t(1) << 16;
__device__ __align__(256) double scratch[kScratchDoubles];

// device address of `scratch` per device, from hipGetSymbolAddress with that device current (the
// array's name on the host is only a stand-in for the symbol)
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

pmg_status scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return pmg::set_error(PMG_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return pmg::set_error(PMG_E_HIP, "hipGetSymbolAddress of the residual scratch failed");
    g_scratch[device] = static_cast<double*>(p);
  }
  *out = g_scratch[device];
  return PMG_OK;
}

}  // namespace

extern "C" pmg_status fr_residual_noalloc(pmg_level L, const double* q, const double* src, const double* S,
                                          double c_mass, double* F, double* norms, void* stream) {
  if (!L) return pmg::set_error(PMG_E_ARG, "null level handle");
  if (!q || !F) return pmg::set_error(PMG_E_ARG, "null q or F");
  if (F == q) return pmg::set_error(PMG_E_ARG, "F must not alias q");
  const int nblk = pmg::residual_blocks(*L);
  if (norms && (size_t)nblk * (size_t)L->nv > kScratchDoubles)
    return pmg::set_error(PMG_E_ARG, "the level's norm partials exceed the 65536 doubles of fr_residual_noalloc's "
                                     "scratch; use fr_residual");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(L->device) != hipSuccess)
    return pmg::set_error(PMG_E_HIP, "cannot select the level's device");
  pmg_status status = PMG_OK;
  double* part = nullptr;
  if (norms) status = scratch_address(L->device, &part);
  if (status == PMG_OK) {
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = pmg::launch_residual(*L, q, src, S, c_mass, F, norms != nullptr, st, part);
    if (e == hipSuccess && norms) e = pmg::launch_norm_finalize_to(part, nblk, L->nv, norms, st);
    if (e != hipSuccess) status = pmg::set_error(PMG_E_HIP, hipGetErrorString(e));
  }
  (void)hipSetDevice(prev);
  return status;
}
