// launch3.hpp -- launches of the 3D step kernel for one node-update mode;
// each mode's kernels are instantiated by a translation unit of their own
// (k_step3_<mode>.hip), reached through step3_launch (lbm_stefan_internal.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice3d.hpp"
#include "lbm_stefan.h"

namespace irebm {
namespace {

// split: 0 the plain kernel, 1 the quiet pass, 2 the full pass over
// flagged items (step3_kernel); A's x_off, x_lim and flags as set by the
// host
template <int Q, typename S, int MODE>
hipError_t launch_step3_t(const StepArgs3 &A0, const Variant3 &v, int split,
                          hipStream_t stream) {
  StepArgs3 A = A0;
  set_tiling3(&A, v);
  if (A.nitems <= 0) return hipSuccess;
  constexpr bool kNoSplit = base_mode(MODE) == kEebm || neumann_mode(MODE);
  if (split && (kNoSplit || !A.flags)) return hipErrorInvalidValue;
  dim3 grid((unsigned)(8 * A.per_xcd)), block(v.bx, v.by);
#define LAUNCH3S(NPT, NT, SP) \
  step3_kernel<Q, S, NPT, MODE, NT, SP><<<grid, block, 0, stream>>>(A)
#define LAUNCH3(NPT, NT)                                \
  do {                                                  \
    if constexpr (kNoSplit) LAUNCH3S(NPT, NT, 0);       \
    else if (split == 1) LAUNCH3S(NPT, NT, 1);          \
    else if (split == 2) LAUNCH3S(NPT, NT, 2);          \
    else LAUNCH3S(NPT, NT, 0);                          \
  } while (0)
  if (v.npt == 2) {
    if (v.nt) LAUNCH3(2, true);
    else LAUNCH3(2, false);
  } else {
    if (v.nt) LAUNCH3(1, true);
    else LAUNCH3(1, false);
  }
#undef LAUNCH3
#undef LAUNCH3S
  return hipGetLastError();
}

}  // namespace

template <int MODE>
hipError_t step3_launch_mode(int q, int storage, const StepArgs3 &A,
                             const Variant3 &v, int split,
                             hipStream_t stream) {
  const bool f32 = storage == LBM_STORE_F32;
  if (q == 7)
    return f32 ? launch_step3_t<7, float, MODE>(A, v, split, stream)
               : launch_step3_t<7, double, MODE>(A, v, split, stream);
  return f32 ? launch_step3_t<19, float, MODE>(A, v, split, stream)
             : launch_step3_t<19, double, MODE>(A, v, split, stream);
}

}  // namespace irebm

#define IREBM_INSTANTIATE_STEP3(M)                                        \
  template hipError_t irebm::step3_launch_mode<M>(                        \
      int, int, const irebm::StepArgs3 &, const irebm::Variant3 &, int,   \
      hipStream_t)
