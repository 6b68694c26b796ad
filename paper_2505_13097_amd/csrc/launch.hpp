// launch.hpp -- launches of the time-step kernels for one node-update
// mode (safeguarded or printed Newton, or the explicit scheme).  Each
// mode's kernels are instantiated by small translation units of their own
// (k_step_<mode>.hip, k_batch_<mode>.hip, and k_step_<mode>_neumann.hip for
// the one-step kernels of lattices with a Neumann wall), so the library's
// units compile in parallel; host code reaches them through step_launch,
// step2_launch and batch_launch (lbm_stefan_internal.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "host_util.hpp"
#include "kernels.hpp"
#include "lbm_stefan_internal.hpp"

namespace irebm {
namespace {

// ---------------------------------------------------------------------
// batch kernels: many lattices, one flat table of work items

// one work item of the table: items[t] = (instance, item index within
// it); the descriptor is block-uniform and read in place with scalar loads
template <int Q, typename S, int NPT, int MODE, bool NT, bool LOOP>
__device__ __forceinline__ void batch_item(const StepArgs *__restrict__ descs,
                                           const int2 *__restrict__ items,
                                           int t, int parity) {
  const int2 e = items[t];
  const int inst = __builtin_amdgcn_readfirstlane(e.x);
  const int item = __builtin_amdgcn_readfirstlane(e.y);
  const StepArgs &A = descs[inst];
  const auto src = to_global((const S *)(parity ? A.dst : A.src));
  const auto dst = to_global((S *)(parity ? A.src : A.dst));
  step_item<Q, S, NPT, MODE, NT, LOOP>(A, src, dst, item, A.slots + item);
}

// one block per work item, the blocks of XCD k taking the k-th contiguous
// chunk of the table
template <int Q, typename S, int NPT, int MODE, bool NT>
__global__ __launch_bounds__(256) void batch_step_kernel(
    const StepArgs *__restrict__ descs, const int2 *__restrict__ items,
    int32_t nitems, int32_t parity, int32_t reverse) {
  const int chunk = (nitems + 7) >> 3;
  const int b = (int)blockIdx.x;
  if ((b & 7) * chunk + (b >> 3) >= nitems) return;
  batch_item<Q, S, NPT, MODE, NT, false>(
      descs, items, xcd_item(b, chunk, nitems, reverse), parity);
}

// persistent grid sized to the machine: each block walks its XCD's chunk
// of the table with a stride
template <int Q, typename S, int NPT, int MODE, bool NT>
__global__ __launch_bounds__(256) void batch_persistent_kernel(
    const StepArgs *__restrict__ descs, const int2 *__restrict__ items,
    int32_t nitems, int32_t parity, int32_t reverse) {
  const int chunk = (nitems + 7) >> 3;
  const int per_xcd_blocks = (int)(gridDim.x >> 3);
  const int xcd = (int)(blockIdx.x & 7), lane = (int)(blockIdx.x >> 3);
  const int t_end = min(nitems, (xcd + 1) * chunk);
  for (int t = xcd * chunk + lane; t < t_end; t += per_xcd_blocks)
    batch_item<Q, S, NPT, MODE, NT, true>(descs, items,
                                          reverse ? nitems - 1 - t : t, parity);
}

// the front strips of the split schedule (front2_body): one block per
// segment of an instance's strip, XCD-contiguous chunks; the strip's
// column limits are the descriptor's x_lim and x_cnt and its statistics
// slots follow the instance's two-step items
template <int Q, typename S, int MODE>
__global__ __launch_bounds__(256) void batch_front_kernel(
    const StepArgs *__restrict__ descs, const int2 *__restrict__ items,
    int32_t nitems, int32_t parity) {
  const int chunk = (nitems + 7) >> 3;
  const int b = (int)blockIdx.x;
  if ((b & 7) * chunk + (b >> 3) >= nitems) return;
  const int2 e = items[xcd_item(b, chunk, nitems, 0)];
  const int inst = __builtin_amdgcn_readfirstlane(e.x);
  const int seg = __builtin_amdgcn_readfirstlane(e.y);
  const StepArgs &A = descs[inst];
  const auto src = to_global((const S *)(parity ? A.dst : A.src));
  const auto dst = to_global((S *)(parity ? A.src : A.dst));
  front2_body<Q, S, MODE>(A, src, dst, seg, A.slots + A.nitems + seg);
}

// two steps (or one) per launch: one block per item of the two-step
// tiling (a strip of one segment of one instance), XCD-contiguous chunks.
//
// Split schedule (SPLIT > 0, IREBM): the Newton solve is what keeps the
// two-step kernel from its memory bound (its registers cap the waves per
// SIMD, and the front's solves hold every wave of a block at the barriers
// of each pass), while nearly every node of a melting problem is quiet
// (far below the band: a closed form).  So a two-step launch is split by
// work item, with flags[t] per item of the table:
//   flags 1: a front strip, advanced by batch_front_kernel (both steps
//            per segment of rows, the first into LDS) on a stream of its
//            own, beside the quiet pass;
//   flags 0: SPLIT = 1, the kernel built for quiet nodes only (no Newton
//            code, 6 waves per SIMD in FP32 D2Q5); an item with a node
//            (halo included) that is not quiet is set to flags 2;
//   flags 2: SPLIT = 2, the full kernel, run after the quiet pass, which
//            rewrites the item's outputs and returns it to flags 0 when
//            all of its nodes were quiet.
// Every node is updated by the same arithmetic as in the one-pass kernel.
template <int Q, typename S, int MODE, int BY, int WIN, int SPLIT = 0>
__global__ __launch_bounds__(WIN * BY)
__attribute__((amdgpu_waves_per_eu(
    sizeof(S) == 4 ? (SPLIT == 1 && Q == 5 ? 6 : 4) : 1)))
void batch_step2_kernel(const StepArgs *__restrict__ descs,
                        const int2 *__restrict__ items, int32_t nitems,
                        int32_t parity, int32_t two, int *__restrict__ flags) {
  const int per_xcd = (nitems + 7) >> 3;
  const int t = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (t >= nitems) return;
  if (SPLIT > 0 &&
      __builtin_amdgcn_readfirstlane(flags[t]) != (SPLIT == 1 ? 0 : 2))
    return;
  const int2 e = items[t];
  const int inst = __builtin_amdgcn_readfirstlane(e.x);
  const int item = __builtin_amdgcn_readfirstlane(e.y);
  const StepArgs &A = descs[inst];
  const auto src = to_global((const S *)(parity ? A.dst : A.src));
  const auto dst = to_global((S *)(parity ? A.src : A.dst));
  const bool any = step2_body<Q, S, MODE, true, BY, WIN, SPLIT == 1,
                              SPLIT == 2>(A, src, dst, item % A.tiles_x,
                                          item / A.tiles_x, A.group, two != 0,
                                          A.slots + item);
  if (SPLIT > 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    if (SPLIT == 1 && any) flags[t] = 2;
    if (SPLIT == 2 && !any) flags[t] = 0;
  }
}

// ---------------------------------------------------------------------
// typed launchers

// one step of one lattice with the (one-step) tiling of v
template <int Q, typename S, int MODE>
hipError_t launch_step_t(const StepArgs &A, const Variant &v, bool reverse,
                         hipStream_t stream) {
  StepArgs B = A;
  set_tiling(&B, v);
  B.reverse = reverse;
  dim3 grid(8 * B.per_xcd), block(v.bx, v.by);
#define LAUNCH(NPT, NT) \
  step_kernel<Q, S, NPT, MODE, NT><<<grid, block, 0, stream>>>(B)
#define LAUNCH_NPT(NT)                 \
  do {                                 \
    if (v.npt == 1) LAUNCH(1, NT);     \
    else if (v.npt == 2) LAUNCH(2, NT); \
    else LAUNCH(4, NT);                \
  } while (0)
  if (v.nt) LAUNCH_NPT(true);
  else LAUNCH_NPT(false);
#undef LAUNCH_NPT
#undef LAUNCH
  return hipGetLastError();
}

// two steps (one if two = false) of one 2D lattice, two-step variant v
template <int Q, typename S, int MODE>
hipError_t launch_step2_t(const StepArgs &A, const Variant &v, bool two,
                          hipStream_t stream) {
  if constexpr (Q == 3) {
    return hipErrorInvalidValue;
  } else {
    const int32_t nstrips = (int32_t)((A.nx + v.bx - 5) / (v.bx - 4));
    const int64_t nseg = (A.ny + v.rows - 1) / v.rows;
    const int32_t nitems = (int32_t)(nstrips * nseg);
    dim3 grid((unsigned)(8 * ((nitems + 7) / 8))), block(v.bx, v.by);
#define LAUNCH2(BY, WIN)                                                  \
  step2_kernel<Q, S, MODE, true, BY, WIN><<<grid, block, 0, stream>>>(    \
      A, nstrips, v.rows, nitems, two ? 1 : 0)
    if (v.bx == 256) LAUNCH2(2, 256);
    else if (v.by == 2) LAUNCH2(2, 128);
    else LAUNCH2(4, 128);
#undef LAUNCH2
    return hipGetLastError();
  }
}

// one launch of a batch table (see BatchLaunch)
template <int Q, typename S, int MODE>
hipError_t launch_batch_t(const BatchLaunch &b, const Variant &v,
                          hipStream_t stream) {
  const int64_t chunk = (b.nitems + 7) / 8;
  const int32_t nt = (int32_t)b.nitems;
  if (b.front) {
    if constexpr (Q == 3 || MODE == kEebm) {
      return hipErrorInvalidValue;
    } else {
      dim3 grid((unsigned)(8 * std::max<int64_t>(chunk, 1))), block(256);
      batch_front_kernel<Q, S, MODE>
          <<<grid, block, 0, stream>>>(b.descs, b.items, nt, b.parity);
      return hipGetLastError();
    }
  }
  if (v.tb) {
    if constexpr (Q == 3) {
      return hipErrorInvalidValue;
    } else {
      dim3 grid((unsigned)(8 * std::max<int64_t>(chunk, 1))), block(v.bx, v.by);
      const int32_t tw = b.two ? 1 : 0;
      if (b.split && (MODE == kEebm || !b.flags || !b.two))
        return hipErrorInvalidValue;
#define B2LAUNCH_S(BY, WIN, SP)                                            \
  batch_step2_kernel<Q, S, MODE, BY, WIN, SP><<<grid, block, 0, stream>>>( \
      b.descs, b.items, nt, b.parity, tw, b.flags)
#define B2LAUNCH(BY, WIN)                                                  \
  do {                                                                     \
    if constexpr (MODE == kEebm) B2LAUNCH_S(BY, WIN, 0);                   \
    else if (b.split == 1) B2LAUNCH_S(BY, WIN, 1);                         \
    else if (b.split == 2) B2LAUNCH_S(BY, WIN, 2);                         \
    else B2LAUNCH_S(BY, WIN, 0);                                           \
  } while (0)
      if (v.bx == 256) B2LAUNCH(2, 256);
      else if (v.by == 2) B2LAUNCH(2, 128);
      else B2LAUNCH(4, 128);
#undef B2LAUNCH
#undef B2LAUNCH_S
      return hipGetLastError();
    }
  }
  int64_t g8 = chunk;  // one block per item
  if (b.blocks_per_cu > 0)
    g8 = std::min<int64_t>(((int64_t)b.cus * b.blocks_per_cu + 7) / 8, chunk);
  dim3 grid((unsigned)(8 * std::max<int64_t>(g8, 1))), block(v.bx, v.by);
  const int32_t rev = v.rev && b.parity;
  const bool pers = b.blocks_per_cu > 0;
#define BLAUNCH(NPT, NTS)                                                  \
  do {                                                                     \
    if (pers)                                                              \
      batch_persistent_kernel<Q, S, NPT, MODE, NTS>                        \
          <<<grid, block, 0, stream>>>(b.descs, b.items, nt, b.parity, rev); \
    else                                                                   \
      batch_step_kernel<Q, S, NPT, MODE, NTS>                              \
          <<<grid, block, 0, stream>>>(b.descs, b.items, nt, b.parity, rev); \
  } while (0)
#define BLAUNCH_NPT(NTS)                  \
  do {                                    \
    if (v.npt == 1) BLAUNCH(1, NTS);      \
    else if (v.npt == 2) BLAUNCH(2, NTS); \
    else BLAUNCH(4, NTS);                 \
  } while (0)
  if (v.nt) BLAUNCH_NPT(true);
  else BLAUNCH_NPT(false);
#undef BLAUNCH_NPT
#undef BLAUNCH
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------
// per-mode entry points (explicitly instantiated by the k_*.hip units)

template <int MODE>
hipError_t step_launch_mode(int q, int storage, const StepArgs &A,
                            const Variant &v, bool reverse,
                            hipStream_t stream) {
  return dispatch_qs(q, storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    return launch_step_t<Q, S, MODE>(A, v, reverse, stream);
  });
}

template <int MODE>
hipError_t step2_launch_mode(int q, int storage, const StepArgs &A,
                             const Variant &v, bool two, hipStream_t stream) {
  return dispatch_qs(q, storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    return launch_step2_t<Q, S, MODE>(A, v, two, stream);
  });
}

template <int MODE>
hipError_t resident_launch_mode(int storage, const StepArgs &A,
                                int32_t nsteps, hipStream_t stream) {
  if (storage == LBM_STORE_F32)
    resident1d_kernel<float, MODE><<<1, 1024, 0, stream>>>(A, nsteps);
  else
    resident1d_kernel<double, MODE><<<1, 1024, 0, stream>>>(A, nsteps);
  return hipGetLastError();
}

template <int MODE>
hipError_t batch_launch_mode(int q, int storage, const BatchLaunch &b,
                             const Variant &v, hipStream_t stream) {
  return dispatch_qs(q, storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    return launch_batch_t<Q, S, MODE>(b, v, stream);
  });
}

}  // namespace irebm

#define IREBM_INSTANTIATE_STEP(M)                                          \
  template hipError_t irebm::step_launch_mode<M>(                          \
      int, int, const irebm::StepArgs &, const irebm::Variant &, bool,     \
      hipStream_t);                                                        \
  template hipError_t irebm::step2_launch_mode<M>(                         \
      int, int, const irebm::StepArgs &, const irebm::Variant &, bool,     \
      hipStream_t);                                                        \
  template hipError_t irebm::resident_launch_mode<M>(                      \
      int, const irebm::StepArgs &, int32_t, hipStream_t)

#define IREBM_INSTANTIATE_STEP1(M)                                         \
  template hipError_t irebm::step_launch_mode<M>(                          \
      int, int, const irebm::StepArgs &, const irebm::Variant &, bool,     \
      hipStream_t)

#define IREBM_INSTANTIATE_BATCH(M)                                         \
  template hipError_t irebm::batch_launch_mode<M>(                         \
      int, int, const irebm::BatchLaunch &, const irebm::Variant &,        \
      hipStream_t)
