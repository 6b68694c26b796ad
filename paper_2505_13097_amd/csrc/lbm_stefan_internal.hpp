// lbm_stefan_internal.hpp -- the handle and helpers shared by the
// translation units of the library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "irebm_node.hpp"
#include "lattice3d.hpp"
#include "lbm_stefan.h"

namespace irebm {

// offsets into the caller's workspace
struct Layout {
  size_t buf_bytes = 0;
  size_t off_buf[2] = {0, 0};
  size_t off_prof[4] = {0, 0, 0, 0};
  size_t off_slots = 0, off_partials = 0, off_small = 0, off_adj = 0;
  size_t off_flags = 0; // 3D split step: one flag per quiet-pass item
  size_t off_lf = 0;    // ILFBM: three liquid fraction planes, the per-
                        // block pending values and the control block
  size_t total = 0;
  int64_t max_items = 0, n_partials = 0;
  bool adjoint = false;
};

// the small device result area: stats [0..5), energy, then the front
constexpr int kSmallEnergy = 8;
constexpr int kSmallCount = 9;
constexpr int kSmallFront = 16;

}  // namespace irebm

struct lbm_stefan {
  lbm_stefan_params p;
  irebm::Layout layout;
  int device = 0;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  double *prof[4] = {nullptr, nullptr, nullptr, nullptr};
  bool has_prof[4] = {false, false, false, false};
  irebm::StatSlot *slots = nullptr;
  int64_t max_items = 0;
  // 3D split step: work-item flags (valid for variant flags_variant), and
  // the stream of the front strip with the events that fork and join it
  int32_t *flags = nullptr;
  int flags_variant = -1;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  double *partials = nullptr;
  double *small = nullptr;
  char *adj = nullptr;
  int variant = 0;
  int64_t steps = 0;
  void *tape = nullptr;          // last forward tape
  int64_t tape_steps = 0, tape_interval = 0;
  // ILFBM (Algorithm 1): liquid fraction of the state, two inner-loop
  // planes, per-block pending values, device control block, and the
  // statistics of the inner loop kept on the host
  double *lf = nullptr, *lscr[2] = {nullptr, nullptr}, *pend = nullptr;
  void *ctrl = nullptr;
  int32_t ilf_max_it = 0;
  int64_t ilf_nonconv = 0;
  double ilf_max_res = 0.0, ilf_fin = 0.0, ilf_fout = 0.0;
  std::string err;
};

namespace irebm {

std::string validate_params(const lbm_stefan_params *p);
Layout layout_for(const lbm_stefan_params *p);
size_t adjoint_bytes(const lbm_stefan_params *p, int64_t max_items);
int fail(lbm_stefan_t *h, int code, const std::string &msg);
void set_global_error(const std::string &msg);
// StepArgs of a lattice from its params (prof: device wall profiles or
// NULL); src, dst, slots and the tile fields are left zero
void fill_args(const lbm_stefan_params &p, double *const prof[4],
               StepArgs *A);
void fill_step_args(const lbm_stefan_t *h, StepArgs *A);
hipError_t launch_step(const lbm_stefan_t *h, const void *src, void *dst,
                       hipStream_t stream = nullptr);
// the handle's second stream (split steps, the reverse sweep's
// recomputation) and its two events, created on first use
hipError_t handle_side(lbm_stefan_t *h);
// StepArgs3 of a 3D lattice from its params; src, dst and the tile fields
// are left zero
void fill_args3(const lbm_stefan_params &p, StepArgs3 *A);
// two steps (or one, two = false) in one launch of the two-step kernel
// (the handle's variant is a two-step variant)
hipError_t launch_step2(const lbm_stefan_t *h, const void *src, void *dst,
                        bool two);
bool two_step_variant(const lbm_stefan_t *h);
// advance the handle nsteps (pairs of steps in one launch under a two-step
// variant); updates cur and steps
hipError_t advance(lbm_stefan_t *h, int64_t nsteps);
hipError_t zero_stats_async(lbm_stefan_t *h);
int read_stats(lbm_stefan_t *h, lbm_stefan_stats *st);

// ILFBM (ilfbm.hip): workspace bytes beyond the common layout, the
// handle's pointers into it, and nsteps steps of the inner-loop scheme
size_t ilfbm_bytes(const lbm_stefan_params *p);
void ilfbm_attach(lbm_stefan_t *h, char *base);
hipError_t ilfbm_advance(lbm_stefan_t *h, int64_t nsteps);
void ilfbm_reset_stats(lbm_stefan_t *h);

// ---- kernel launches by node-update mode (launch.hpp; one translation
// unit per mode instantiates them)

struct Variant;

// one launch over a batch's table of work items
struct BatchLaunch {
  const StepArgs *descs;  // device: one descriptor per instance
  const int2 *items;      // device: (instance, item) per work item
  int64_t nitems;
  int cus, blocks_per_cu; // persistent grid of cus * blocks_per_cu blocks
                          // when blocks_per_cu > 0, else one per item
  int parity;             // 0: src -> dst of each descriptor, 1: dst -> src
  bool two;               // two steps under a two-step variant (else one)
  int split = 0;          // two-step kernels: 0 every item, 1 the quiet
                          // pass over items flagged 0, 2 the full pass over
                          // items flagged 2 (batch_step2_kernel)
  int *flags = nullptr;   // device: one flag per work item (split > 0)
  bool front = false;     // the front strips' kernel (items: instance,
                          // segment of front rows)
};

template <int MODE>
hipError_t step_launch_mode(int q, int storage, const StepArgs &A,
                            const Variant &v, bool reverse,
                            hipStream_t stream);
template <int MODE>
hipError_t step2_launch_mode(int q, int storage, const StepArgs &A,
                             const Variant &v, bool two, hipStream_t stream);
template <int MODE>
hipError_t batch_launch_mode(int q, int storage, const BatchLaunch &b,
                             const Variant &v, hipStream_t stream);
// nsteps steps of a small D1Q3 lattice in one resident workgroup
// (resident1d_kernel; the lattice passes resident_ok)
template <int MODE>
hipError_t resident_launch_mode(int storage, const StepArgs &A,
                                int32_t nsteps, hipStream_t stream);

#define IREBM_DECLARE_STEP1(M)                                             \
  extern template hipError_t step_launch_mode<M>(                          \
      int, int, const StepArgs &, const Variant &, bool, hipStream_t)
#define IREBM_DECLARE_MODE(M)                                              \
  IREBM_DECLARE_STEP1(M);                                                  \
  extern template hipError_t step2_launch_mode<M>(                         \
      int, int, const StepArgs &, const Variant &, bool, hipStream_t);     \
  extern template hipError_t resident_launch_mode<M>(                      \
      int, const StepArgs &, int32_t, hipStream_t);                       \
  extern template hipError_t batch_launch_mode<M>(                         \
      int, int, const BatchLaunch &, const Variant &, hipStream_t)
IREBM_DECLARE_MODE(kSafeguarded);
IREBM_DECLARE_MODE(kPlain);
IREBM_DECLARE_MODE(kEebm);
// lattices with a Neumann wall: one-step single-lattice kernels only
IREBM_DECLARE_STEP1(kSafeguarded | kNeumann);
IREBM_DECLARE_STEP1(kPlain | kNeumann);
IREBM_DECLARE_STEP1(kEebm | kNeumann);
#define IREBM_DECLARE_STEP3(M)                                             \
  extern template hipError_t step3_launch_mode<M>(                         \
      int, int, const StepArgs3 &, const Variant3 &, int, hipStream_t)
IREBM_DECLARE_STEP3(kSafeguarded);
IREBM_DECLARE_STEP3(kPlain);
IREBM_DECLARE_STEP3(kEebm);
IREBM_DECLARE_STEP3(kSafeguarded | kNeumann);
IREBM_DECLARE_STEP3(kPlain | kNeumann);
IREBM_DECLARE_STEP3(kEebm | kNeumann);
#undef IREBM_DECLARE_STEP3
#undef IREBM_DECLARE_MODE
#undef IREBM_DECLARE_STEP1

// does a lattice have a Neumann wall (eq. Neu_on_q)?  Its closure reads
// two cells away, so such lattices take one step per launch
inline bool has_neumann(const lbm_stefan_params &p) {
  for (int k = 0; k < (p.dim >= 2 ? 4 : 2); ++k)
    if (p.bc[k] == LBM_BC_NEUMANN) return true;
  if (p.dim == 3)
    for (int k = 0; k < 2; ++k)
      if (p.bc_z[k] == LBM_BC_NEUMANN) return true;
  return false;
}

// can the lattice run under the resident variant (resident1d_kernel)?
// D1Q3, at most kResident1D nodes, no Neumann wall, IREBM or EEBM
inline bool resident_ok(const lbm_stefan_params &p) {
  return p.dim == 1 && p.q == 3 && p.nx <= kResident1D && !has_neumann(p) &&
         p.scheme != LBM_SCHEME_ILFBM;
}

// one launch of resident1d_kernel: nsteps steps of one small 1D lattice
inline hipError_t resident_launch(int mode, int storage, const StepArgs &A,
                                  int32_t nsteps, hipStream_t stream) {
  if (mode == kEebm)
    return resident_launch_mode<kEebm>(storage, A, nsteps, stream);
  if (mode == kPlain)
    return resident_launch_mode<kPlain>(storage, A, nsteps, stream);
  return resident_launch_mode<kSafeguarded>(storage, A, nsteps, stream);
}

// nodes of a lattice, and its rows along x (one front value each)
inline int64_t nodes_of(const lbm_stefan_params &p) {
  return p.nx * p.ny * (p.dim == 3 ? p.nz : 1);
}
inline int64_t rows_of(const lbm_stefan_params &p) {
  return p.ny * (p.dim == 3 ? p.nz : 1);
}

// node-update mode of a lattice (with kNeumann when it has a Neumann wall)
inline int mode_of(const lbm_stefan_params &p) {
  const int neu = has_neumann(p) ? (int)kNeumann : 0;
  if (p.scheme == LBM_SCHEME_EEBM) return kEebm | neu;
  return (p.newton_mode == LBM_NEWTON_PLAIN ? kPlain : kSafeguarded) | neu;
}

// one step of one lattice (one-step variant v)
inline hipError_t step_launch(int mode, int q, int storage, const StepArgs &A,
                              const Variant &v, bool reverse,
                              hipStream_t stream) {
  switch (mode) {
    case kEebm:
      return step_launch_mode<kEebm>(q, storage, A, v, reverse, stream);
    case kPlain:
      return step_launch_mode<kPlain>(q, storage, A, v, reverse, stream);
    case kEebm | kNeumann:
      return step_launch_mode<kEebm | kNeumann>(q, storage, A, v, reverse,
                                                stream);
    case kPlain | kNeumann:
      return step_launch_mode<kPlain | kNeumann>(q, storage, A, v, reverse,
                                                 stream);
    case kSafeguarded | kNeumann:
      return step_launch_mode<kSafeguarded | kNeumann>(q, storage, A, v,
                                                       reverse, stream);
    default:
      return step_launch_mode<kSafeguarded>(q, storage, A, v, reverse,
                                            stream);
  }
}

// two steps (one if two = false) of one 2D lattice (two-step variant v;
// never a lattice with a Neumann wall)
inline hipError_t step2_launch(int mode, int q, int storage,
                               const StepArgs &A, const Variant &v, bool two,
                               hipStream_t stream) {
  if (mode == kEebm)
    return step2_launch_mode<kEebm>(q, storage, A, v, two, stream);
  if (mode == kPlain)
    return step2_launch_mode<kPlain>(q, storage, A, v, two, stream);
  return step2_launch_mode<kSafeguarded>(q, storage, A, v, two, stream);
}

// one step of one 3D lattice (3D variant v); split: 0 the plain kernel,
// 1 and 2 the quiet and full passes of the split step (step3_kernel)
inline hipError_t step3_launch(int mode, int q, int storage,
                               const StepArgs3 &A, const Variant3 &v,
                               hipStream_t stream, int split = 0) {
  switch (mode) {
    case kEebm:
      return step3_launch_mode<kEebm>(q, storage, A, v, split, stream);
    case kPlain:
      return step3_launch_mode<kPlain>(q, storage, A, v, split, stream);
    case kEebm | kNeumann:
      return step3_launch_mode<kEebm | kNeumann>(q, storage, A, v, split,
                                                 stream);
    case kPlain | kNeumann:
      return step3_launch_mode<kPlain | kNeumann>(q, storage, A, v, split,
                                                  stream);
    case kSafeguarded | kNeumann:
      return step3_launch_mode<kSafeguarded | kNeumann>(q, storage, A, v,
                                                        split, stream);
    default:
      return step3_launch_mode<kSafeguarded>(q, storage, A, v, split,
                                             stream);
  }
}

inline hipError_t batch_launch(int mode, int q, int storage,
                               const BatchLaunch &b, const Variant &v,
                               hipStream_t stream) {
  if (mode == kEebm) return batch_launch_mode<kEebm>(q, storage, b, v, stream);
  if (mode == kPlain) return batch_launch_mode<kPlain>(q, storage, b, v, stream);
  return batch_launch_mode<kSafeguarded>(q, storage, b, v, stream);
}

}  // namespace irebm
