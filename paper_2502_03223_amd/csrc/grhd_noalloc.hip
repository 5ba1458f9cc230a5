// grhd_noalloc.hip -- grhd_rk_substep_noalloc: the Runge-Kutta stage of
// grhd_rk_substep for callers that cannot allocate device memory (code under
// graph capture, tight serving loops, harnesses that forbid allocation).  Its
// scratch -- the partial records of the diagnostics and the recovery flags
// of q_s when the caller passes none -- lives in one fixed device array of
// this library instead of a caller workspace.  The kernels are those of
// grhd_rk_substep; only where the scratch comes from differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "grhd.h"
#include "grhd_host.hpp"

namespace grhd {
int rk_substep_ws(const grhd_grid *grid, const grhd_eos *eos, const grhd_metric *metric,
                  const grhd_options *opts, const grhd_rk_stage *stage, const grhd_cons *qn,
                  const grhd_cons *qs, const grhd_cons *qout, const grhd_prim *p,
                  const grhd_cons *acc_in, const grhd_cons *acc_out, double *flux_reg, uint8_t *flags,
                  grhd_diag *diag, void *workspace, size_t workspace_bytes, void *hip_stream);
}  // namespace grhd

using namespace grhd;

// The array itself: every GPU the library runs on holds its own copy, at
// its own address, until the process ends.  Host code never passes the
// name to a kernel or a copy (on the host it is a stand-in, not a device
// address); it uses the address that hipGetSymbolAddress returns on each
// device.
static __device__ __align__(256) unsigned char scratch[GRHD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices];

// The device address of the current device's copy of the array, looked up
// once per device (with that device current) and kept.
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GRHD_ERR_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(GRHD_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(GRHD_ERR_DEVICE, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GRHD_OK;
}
}  // namespace

extern "C" int grhd_rk_substep_noalloc(const grhd_grid *grid, const grhd_eos *eos,
                                       const grhd_metric *metric, const grhd_options *opts,
                                       const grhd_rk_stage *stage, const grhd_cons *qn,
                                       const grhd_cons *qs, const grhd_cons *qout, const grhd_prim *p,
                                       const grhd_cons *acc_in, const grhd_cons *acc_out,
                                       double *flux_reg, uint8_t *flags, grhd_diag *diag,
                                       void *hip_stream) {
  int rc;
  if ((rc = check_grid(grid))) return rc;
  void *ptr = nullptr;
  if ((rc = scratch_address(&ptr))) return rc;
  rc = rk_substep_ws(grid, eos, metric, opts, stage, qn, qs, qout, p, acc_in, acc_out, flux_reg, flags, diag,
                     ptr, GRHD_NOALLOC_SCRATCH_BYTES, hip_stream);
  if (rc == GRHD_ERR_WORKSPACE)
    return fail(GRHD_ERR_WORKSPACE,
                "grid %d x %d needs more scratch than the %d bytes of grhd_rk_substep_noalloc "
                "(pass flags, drop diag, or use grhd_rk_substep with a workspace)",
                grid->nx, grid->nz, (int)GRHD_NOALLOC_SCRATCH_BYTES);
  return rc;
}
