// cr_static.hip -- cr_solve_ik_static: the two-stage IK solve (Algorithm 1) with
// its scratch in a library-owned static device buffer instead of a caller
// workspace, for callers that cannot allocate device memory.
//
// The buffer is a file-scope __device__ array; every GPU the library runs on
// holds its own copy for the life of the process.  Its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and cached;
// host code only ever passes that address, never the array's name.  The solve's
// kernels are those of cr_solve_ik, given the buffer as their workspace.  Every
// kernel writes each workspace value before any kernel reads it (stage-1
// summaries, SelectTop slots including the -1 fill, stage-2 candidates), so the
// contents left by an earlier call are never read and nothing is cleared.
#include <mutex>

#include "cr_internal.h"

namespace crk {
namespace {

static __device__ __align__(256) unsigned char scratch[CR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the buffer (the current device).
cr_status scratch_address(void** out) {
  int dev = -1;
  cr_status rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc != CR_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(CR_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc != CR_OK) return rc;
    if (!p || (uintptr_t)p % 256) return fail(CR_EDEVICE, "static scratch at %p is not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CR_OK;
}

}  // namespace
}  // namespace crk

using namespace crk;

extern "C" cr_status cr_solve_ik_static(const cr_robot* robot, const cr_spheres* spheres, int64_t P,
                                        const void* T_target, int32_t S, const void* u_seed,
                                        const cr_weights* weights, const cr_opts* opts, void* u_out, void* err_out,
                                        int32_t* status_out, cr_dtype dtype, hipStream_t stream) {
  cr_status rc;
  if ((rc = check_robot(robot)) != CR_OK || (rc = check_dtype(dtype)) != CR_OK || (rc = check_opts(opts)) != CR_OK ||
      (rc = check_weights(weights)) != CR_OK)
    return rc;
  if (P < 0 || S < 1 || S > 4096) return fail(CR_EINVAL, "need P >= 0 and 1 <= S <= 4096");
  if (P * (int64_t)S > ((int64_t)1 << 31) - 1) return fail(CR_EINVAL, "P*S too large");
  if (P == 0) return CR_OK;
  if (!T_target || !u_seed || !u_out || !err_out || !status_out) return fail(CR_EINVAL, "NULL array argument");
  if ((rc = check_spheres(spheres, P)) != CR_OK ||
      (rc = check_poly_ok(spheres, robot, true, "cr_solve_ik_static")) != CR_OK)
    return rc;
  const size_t need = ik_workspace_layout(*robot, P, S, *opts, dtype, nullptr, nullptr);
  if (need > (size_t)CR_STATIC_SCRATCH_BYTES)
    return fail(CR_ENOMEM, "these shapes need %zu bytes of scratch, more than the static %zu bytes (use cr_solve_ik)",
                need, (size_t)CR_STATIC_SCRATCH_BYTES);
  void* mem = nullptr;
  if ((rc = scratch_address(&mem)) != CR_OK) return rc;
  IkWorkspace w;
  ik_workspace_layout(*robot, P, S, *opts, dtype, (char*)mem, &w);
  const cr_spheres* sp = (spheres && (spheres->n_sph > 0 || spheres->n_poly > 0)) ? spheres : nullptr;
  return launch_solve_ik(*robot, sp, P, (const double*)T_target, S, (const double*)u_seed, *weights, *opts,
                         (double*)u_out, (double*)err_out, status_out, w, dtype, stream);
}
