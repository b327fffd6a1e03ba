// idp_dg_step_noalloc: one SSP-RK3 step of a periodic problem without a
// handle and without any allocation.  The two stage buffers that
// idp_dg_step keeps in its handle live here in one file-scope device array,
// `scratch`, held by every GPU the library runs on until the process ends.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/idp_dg.h"
#include "common.hpp"
#include "handle.hpp"

using namespace idp;

namespace {

// 64 MiB: two stage buffers of up to IDP_DG_NOALLOC_MAX_DOUBLES doubles
static_assert(2LL * 8 * IDP_DG_NOALLOC_MAX_DOUBLES <= (64LL << 20), "scratch holds two stage buffers");
static __device__ __align__(256) double scratch[2LL * IDP_DG_NOALLOC_MAX_DOUBLES];

// Device address of `scratch` on each device, resolved once per device with
// that device current.  Host code uses these addresses only: in host code
// the array's name stands for a host-side shadow, not for device memory.
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

hipError_t scratch_on(int dev, double** ptr) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *ptr = g_scratch[dev];
  return hipSuccess;
}

bool overlaps(const double* a, const double* b, long long n) { return a < b + n && b < a + n; }

}  // namespace

extern "C" int idp_dg_step_noalloc(const idp_dg_desc* desc, double* u, double dt, void* hip_stream) {
  using idp_host::fail;
  std::string why;
  if (!idp_host::desc_ok(desc, &why)) return fail(nullptr, IDP_DG_EINVAL, why);
  if (desc->bc[0] != IDP_DG_BC_PERIODIC || desc->bc[1] != IDP_DG_BC_PERIODIC)
    return fail(nullptr, IDP_DG_EINVAL, "idp_dg_step_noalloc: periodic directions only");
  if (desc->eq == IDP_DG_ADVECTION_FIELD)
    return fail(nullptr, IDP_DG_EINVAL, "idp_dg_step_noalloc: no velocity field (it needs device arrays)");
  if (!u) return fail(nullptr, IDP_DG_EINVAL, "NULL state pointer");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(nullptr, IDP_DG_EINVAL, "dt must be finite and >= 0");
  // a stack handle: host tables only, no device buffers of its own
  idp_dg h;
  idp_host::init_host(&h, desc, hip_stream);
  const long long n = (long long)h.nc * h.nn;
  if (n > IDP_DG_NOALLOC_MAX_DOUBLES)
    return fail(nullptr, IDP_DG_EINVAL,
                "idp_dg_step_noalloc: nc * Nn = " + std::to_string(n) + " exceeds the static buffers' " +
                    std::to_string((long long)IDP_DG_NOALLOC_MAX_DOUBLES) + " doubles");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
  double* buf = nullptr;
  if (e == hipSuccess) e = scratch_on(dev, &buf);
  if (e != hipSuccess)
    return fail(nullptr, IDP_DG_EHIP, std::string("idp_dg_step_noalloc: ") + hipGetErrorString(e));
  h.device = dev;
  h.buf1 = buf;
  h.buf2 = buf + n;
  if (overlaps(u, h.buf1, 2 * n)) return fail(nullptr, IDP_DG_EINVAL, "u overlaps the static buffers");
  // no diagnostics (h.diag is NULL): the kernels then skip their counters;
  // the stage buffers are written in full before they are read, so nothing
  // needs clearing
  hipStream_t s = h.stream;
  e = idp_host::launch_stage(&h, idp_host::make_stage_args(&h, nullptr, u, h.buf1, dt, nullptr, 1.0, 0), s);
  if (e == hipSuccess)
    e = idp_host::launch_stage(&h, idp_host::make_stage_args(&h, u, h.buf1, h.buf2, dt, nullptr, 1.0, 1), s);
  if (e == hipSuccess)
    e = idp_host::launch_stage(&h, idp_host::make_stage_args(&h, u, h.buf2, u, dt, nullptr, 1.0, 2), s);
  if (e != hipSuccess)
    return fail(nullptr, IDP_DG_EHIP, std::string("idp_dg_step_noalloc launch: ") + hipGetErrorString(e));
  return 0;
}
