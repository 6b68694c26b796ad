// noalloc.hip -- one time step that allocates nothing: the step of
// lbm_stefan_step (Algorithm 3, Section 4.1, with the closures of Section
// 4.2; or Algorithm 2 for EEBM) from a caller's state to a caller's
// buffer, with the per-item statistics, the energy partials and the result
// block in a fixed device array of this unit instead of a workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "host_util.hpp"
#include "kernels.hpp"
#include "lbm_stefan.h"
#include "lbm_stefan_internal.hpp"

using namespace irebm;

// Statistics slots, energy partials and the small result block of every
// call on a device.  Each device holds its own copy for the life of the
// process.  In host code `scratch` names a host-side stand-in, not device
// memory: host code uses only the address hipGetSymbolAddress returns for
// the current device (noalloc_scratch).
static __device__ __align__(256) char scratch[LBM_STEFAN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// errors go to the calling thread's handle-less error text
// (lbm_stefan_last_error(NULL))
int nfail(int code, const std::string &msg) {
  set_global_error(msg);
  return code;
}

// address of the current device's scratch (looked up once per device,
// with that device current)
hipError_t noalloc_scratch(int dev, char **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = (char *)g_ptr[dev];
  return hipSuccess;
}

// scratch layout of a lattice: [slots | partials | result block]
struct ScratchPlan {
  int64_t nslots = 0, nparts = 0;
  size_t off_parts = 0, off_small = 0, total = 0;
};

ScratchPlan plan_for(int64_t nslots, int64_t nodes) {
  ScratchPlan s;
  s.nslots = nslots;
  s.nparts = (nodes + kEnergyChunk - 1) / kEnergyChunk;
  s.off_parts = align256((size_t)nslots * sizeof(StatSlot));
  s.off_small = s.off_parts + align256((size_t)s.nparts * 8);
  s.total = s.off_small + align256(kSmallCount * 8);
  return s;
}

}  // namespace

extern "C" {

int lbm_stefan_step_noalloc(const lbm_stefan_params *p, const void *src,
                            void *dst, lbm_stefan_stats *stats,
                            void *stream) {
  std::string e = validate_params(p);
  if (!e.empty()) return nfail(LBM_STEFAN_EINVAL, e);
  if (!src || !dst) return nfail(LBM_STEFAN_EINVAL, "src or dst is NULL");
  if (src == dst) return nfail(LBM_STEFAN_EINVAL, "src and dst must differ");
  if (p->scheme == LBM_SCHEME_ILFBM)
    return nfail(LBM_STEFAN_EINVAL,
                 "the ILFBM scheme keeps liquid-fraction planes: use a handle");
  if (p->flags & LBM_FLAG_ADJOINT)
    return nfail(LBM_STEFAN_EINVAL, "the reverse mode needs a handle");
  for (int k = 0; k < 4; ++k)
    if (p->wall_profile[k])
      return nfail(LBM_STEFAN_EINVAL,
                   "wall profiles need a device copy: use a handle");
  lbm_stefan_params q = *p;
  if (q.dx == 0.0) q.dx = 1.0 / (double)(q.nx - 1);
  if (q.dim == 1) q.bc[2] = q.bc[3] = LBM_BC_PERIODIC;
  const int64_t nodes = nodes_of(q);
  // the kernel tiling and the scratch it needs (host arithmetic only:
  // oversized lattices are refused before any device call)
  int nv;
  const Variant3 *v3 = nullptr;
  const Variant *v2 = nullptr;
  ScratchPlan s;
  if (q.dim == 3) {
    v3 = &variants3(&nv)[q.variant >= 0 ? q.variant : kDefaultVariant3D];
    s = plan_for(items3_for(*v3, q.nx, q.ny, q.nz), nodes);
  } else {
    // the one-step tiling of the variant (a two-step variant's single
    // step and the resident variant's step take the defaults, as in a
    // handle)
    const Variant *vt = variants(q.q, &nv);
    int vi = q.variant;
    if (vi < 0) vi = q.dim == 1 ? kDefaultVariant1D : kDefaultVariant2D;
    if (vt[vi].tb) vi = kDefaultVariant2D;
    if (vt[vi].res) vi = kDefaultVariant1D;
    v2 = &vt[vi];
    s = plan_for(items_for(*v2, q.nx, q.ny), nodes);
  }
  if (s.total > LBM_STEFAN_NOALLOC_SCRATCH_BYTES)
    return nfail(LBM_STEFAN_EINVAL,
                 "lattice too large for the fixed scratch (" +
                     std::to_string(s.total) + " of " +
                     std::to_string(LBM_STEFAN_NOALLOC_SCRATCH_BYTES) +
                     " bytes)");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return nfail(LBM_STEFAN_EDEVICE, "no usable current device");
  char *base = nullptr;
  hipError_t he = noalloc_scratch(dev, &base);
  if (he != hipSuccess)
    return nfail(LBM_STEFAN_EDEVICE,
                 std::string("hipGetSymbolAddress: ") + hipGetErrorString(he));
  const int mode = mode_of(q);
  // the slots accumulate: clear them (a fill kernel), then the step
  he = zero_async(base, s.nslots * sizeof(StatSlot), st);
  if (q.dim == 3) {
    StepArgs3 A;
    fill_args3(q, &A);
    A.src = src;
    A.dst = dst;
    A.slots = (StatSlot *)base;
    if (he == hipSuccess) he = step3_launch(mode, q.q, q.storage, A, *v3, st);
  } else {
    StepArgs A;
    fill_args(q, nullptr, &A);
    A.src = src;
    A.dst = dst;
    A.slots = (StatSlot *)base;
    if (he == hipSuccess)
      he = step_launch(mode, q.q, q.storage, A, *v2, false, st);
  }
  if (he != hipSuccess)
    return nfail(LBM_STEFAN_EDEVICE,
                 std::string("step: ") + hipGetErrorString(he));
  if (!stats && !q.strict) return LBM_STEFAN_OK;
  // statistics of this step: the per-item slots, then the energy of dst
  double *small = (double *)(base + s.off_small);
  stats_kernel<<<1, 256, 0, st>>>((const StatSlot *)base, s.nslots, small);
  he = hipGetLastError();
  if (he == hipSuccess)
    he = energy_async(q, dst, (double *)(base + s.off_parts),
                      small + kSmallEnergy, st);
  double hs[kSmallCount];
  if (he == hipSuccess)
    he = hipMemcpyAsync(hs, small, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess)
    return nfail(LBM_STEFAN_EDEVICE,
                 std::string("statistics: ") + hipGetErrorString(he));
  lbm_stefan_stats o;
  o.steps = 1;
  o.max_newton_it = (int32_t)hs[0];
  o.reserved = 0;
  o.nonconverged = (int64_t)hs[1];
  o.max_residual = hs[2];
  o.flux_in = hs[3];
  o.flux_out = hs[4];
  o.energy = hs[kSmallEnergy];
  if (stats) *stats = o;
  if (!std::isfinite(o.energy))
    return nfail(LBM_STEFAN_ENAN, "energy is not finite");
  if (q.strict && o.nonconverged > 0)
    return nfail(LBM_STEFAN_ENOTCONV, "a Newton solve reached newton_max_it");
  return LBM_STEFAN_OK;
}

}  // extern "C"
