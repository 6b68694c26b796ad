// batch.hip -- many independent IREBM lattices of uneven sizes and
// parameters advanced by one persistent kernel launch per time step.
//
// Every instance gets a descriptor (its StepArgs: sizes, physics,
// boundaries, buffers, statistics base) and its work items (stacks of
// tiles, see step_item) are listed in one flat table, instance by
// instance and row by row within an instance.  A grid of one block per
// item, or a persistent grid of (compute units x blocks per CU) blocks,
// walks that table: the table is cut into eight contiguous chunks, one per
// XCD (block b runs on XCD b mod 8), so neighbouring tiles of an instance
// are swept by the same XCD and share its L2.  The node update is the one of
// the single-lattice step (step_item), so a batch member evolves exactly
// as the same lattice run alone, IREBM or EEBM alike.  Steps can be
// captured in a hipGraph; the autotuner picks the tile variant and the
// grid size.  Under a split two-step variant (tb = 2, IREBM) a launch of
// two steps is three kernels: the front strips (the first columns of each
// instance heated at x = 0) on a stream of their own, beside the quiet
// pass over the other items, then the full pass over the items the quiet
// pass flagged (see batch_step2_kernel).  This unit is the
// host side; the kernels and their launches are in launch.hpp
// (instantiated by k_batch_<mode>.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host_util.hpp"
#include "kernels.hpp"
#include "lbm_stefan.h"
#include "lbm_stefan_internal.hpp"

using namespace irebm;

struct lbm_stefan_batch {
  std::vector<lbm_stefan_params> ps;
  int count = 0, q = 0, storage = 0;
  int mode = kSafeguarded;  // node-update mode shared by the instances
  int device = 0, cus = 0;
  hipStream_t stream = nullptr, cap_stream = nullptr;
  // split schedule: the front passes run on a stream of their own, forked
  // from and joined back into the launching stream by two events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  char *ws = nullptr;
  StepArgs *descs = nullptr;
  int2 *items = nullptr;
  StatSlot *slots = nullptr;
  int *flags = nullptr;        // split schedule: one flag per work item
  int2 *fitems = nullptr;      // split schedule: front segments
  double *profs = nullptr, *partials = nullptr, *small = nullptr;
  char *state[2] = {nullptr, nullptr};
  size_t state_bytes = 0;
  bool split_ok = false;       // a split two-step schedule can run
  int64_t nslots = 0, nfitems = 0;
  std::vector<size_t> off;          // instance offset in a state region
  std::vector<size_t> prof_off;     // instance offset in the profiles
  std::vector<int64_t> first_item, nitems_inst;
  int64_t max_items = 0, nitems = 0;
  int cur = 0;
  int variant = kDefaultVariant2D, blocks_per_cu = 0, graph_steps = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int64_t steps = 0;
  std::string err;
};

namespace {

struct BLayout {
  size_t descs, items, slots, flags, fitems, profs, partials, small, stateA,
      stateB, total;
  size_t state_bytes;
  int64_t max_items, max_fitems, nslots, max_parts, small_len;
  bool split_ok;
  std::vector<size_t> off, prof_off;
};

// a split two-step schedule needs Newton solves to split off (not EEBM)
// and 2D lattices
bool split_applies(const lbm_stefan_params &p) {
  return p.q != 3 && p.scheme != LBM_SCHEME_EEBM;
}

// instances whose strip 0 runs the front pass: heated through a Dirichlet
// wall at x = 0 (a profile, or a temperature not on phi's lower plateau)
bool front_strip(const lbm_stefan_params &p) {
  return p.bc[0] == LBM_BC_DIRICHLET &&
         (p.wall_profile[0] || p.wall_T[0] >= p.t_m - 20.0 * p.delta);
}

// front segments (batch_front_kernel items) of a lattice of ny rows
int64_t front_items(const lbm_stefan_params &p) {
  const int r = p.storage == LBM_STORE_F64 ? front_rows<double>()
                                           : front_rows<float>();
  return (p.ny + r - 1) / r;
}

// columns of the front strip of an instance: the whole lattice when it is
// at most 64 columns wide (the front kernel's window), else the first
// kFrontColumns
int front_cols(const Variant &v, int64_t nx) {
  (void)v;
  return nx <= 64 ? (int)nx : kFrontColumns;
}

// two-step work items of an instance with a front strip: strips shifted
// by (bx - 4) - front_cols columns, so one more strip column at most
int64_t shifted_items(const Variant &v, int64_t nx, int64_t ny) {
  const int64_t w = v.bx - 4;
  return ((nx + w - front_cols(v, nx) + w - 1) / w) *
         ((ny + v.rows - 1) / v.rows);
}

int bfail(lbm_stefan_batch_t *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  else set_global_error(msg);
  return code;
}

#define BCHK(b, expr)                                                    \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess)                                                \
      return bfail((b), LBM_STEFAN_EDEVICE,                              \
                   std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

std::string validate_batch(const lbm_stefan_params *ps, int32_t count) {
  if (!ps) return "params is NULL";
  if (count < 1 || count > (1 << 20)) return "count must be in 1..2^20";
  for (int k = 0; k < count; ++k) {
    const std::string e = validate_params(&ps[k]);
    if (!e.empty()) return "instance " + std::to_string(k) + ": " + e;
    if (ps[k].dim == 3)
      return "instance " + std::to_string(k) +
             ": the batched form takes 1D and 2D lattices";
    if (ps[k].q != ps[0].q || ps[k].storage != ps[0].storage ||
        ps[k].newton_mode != ps[0].newton_mode ||
        ps[k].scheme != ps[0].scheme)
      return "instances must share lattice, storage, newton_mode and scheme";
    if (has_neumann(ps[k]))
      return "instance " + std::to_string(k) +
             ": the batched form has no Neumann closure";
    if (ps[k].scheme == LBM_SCHEME_ILFBM)
      return "instance " + std::to_string(k) +
             ": the batched form runs IREBM and EEBM only";
  }
  return "";
}

BLayout batch_layout(const lbm_stefan_params *ps, int32_t count) {
  BLayout L;
  const size_t s = ps[0].storage == LBM_STORE_F64 ? 8 : 4;
  int nv;
  const Variant *v = variants(ps[0].q, &nv);
  L.max_items = 0;
  L.split_ok = split_applies(ps[0]);
  for (int i = 0; i < nv; ++i) {
    int64_t t = 0;
    for (int k = 0; k < count; ++k)
      t += v[i].tb == 2 && L.split_ok && front_strip(ps[k])
               ? shifted_items(v[i], ps[k].nx, ps[k].ny)
               : items_for(v[i], ps[k].nx, ps[k].ny);
    L.max_items = std::max(L.max_items, t);
  }
  L.max_fitems = 0;
  for (int k = 0; k < count && L.split_ok; ++k)
    if (front_strip(ps[k])) L.max_fitems += front_items(ps[k]);
  L.nslots = L.max_items + L.max_fitems;
  L.state_bytes = 0;
  L.off.resize(count);
  L.prof_off.resize(count);
  size_t prof_total = 0;
  int64_t max_ny = 16;
  L.max_parts = 1;
  for (int k = 0; k < count; ++k) {
    const int64_t n = ps[k].nx * ps[k].ny;
    L.off[k] = L.state_bytes;
    L.state_bytes += align256((size_t)ps[k].q * n * s);
    L.prof_off[k] = prof_total;
    prof_total += 4 * (size_t)std::max(ps[k].nx, ps[k].ny);
    max_ny = std::max(max_ny, ps[k].ny);
    L.max_parts = std::max(L.max_parts, (n + kEnergyChunk - 1) / kEnergyChunk);
  }
  L.small_len = 16 * (int64_t)count + max_ny + 16;
  size_t o = 0;
  L.descs = o;
  o += align256(count * sizeof(StepArgs));
  L.items = o;
  o += align256(L.max_items * sizeof(int2));
  L.slots = o;
  o += align256(L.nslots * sizeof(StatSlot));
  L.flags = o;
  o += L.split_ok ? align256(L.max_items * sizeof(int)) : 0;
  L.fitems = o;
  o += align256(L.max_fitems * sizeof(int2));
  L.profs = o;
  o += align256(prof_total * 8);
  L.partials = o;
  o += align256(L.max_parts * 8);
  L.small = o;
  o += align256(L.small_len * 8);
  L.stateA = o;
  o += L.state_bytes;
  L.stateB = o;
  o += L.state_bytes;
  L.total = o;
  return L;
}

void drop_side(lbm_stefan_batch_t *b) {
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->side) (void)hipStreamDestroy(b->side);
  b->fork = b->join = nullptr;
  b->side = nullptr;
}

void drop_graphs(lbm_stefan_batch_t *b) {
  for (int k = 0; k < 2; ++k)
    if (b->graph[k]) {
      (void)hipGraphExecDestroy(b->graph[k]);
      b->graph[k] = nullptr;
    }
}

// descriptors and item table for the current variant; uploads both and
// zeroes the statistics (the item -> slot map changes with the items).
// The statistics slots of instance k are contiguous: its work items, then
// (split schedule) its front segments.
int build_schedule(lbm_stefan_batch_t *b) {
  int nv;
  const Variant *vt = variants(b->q, &nv);
  const Variant &v = vt[b->variant];
  const bool split = v.tb == 2 && b->split_ok;
  std::vector<StepArgs> d(b->count);
  std::vector<int2> t, ft;
  std::vector<int> fl;
  t.reserve(b->max_items);
  b->first_item.assign(b->count, 0);
  b->nitems_inst.assign(b->count, 0);
  int64_t sbase = 0;
  for (int k = 0; k < b->count; ++k) {
    const lbm_stefan_params &p = b->ps[k];
    double *prof[4];
    for (int w = 0; w < 4; ++w)
      prof[w] = p.wall_profile[w] ? b->profs + b->prof_off[k] +
                                        w * std::max(p.nx, p.ny)
                                  : nullptr;
    fill_args(p, prof, &d[k]);
    d[k].src = b->state[0] + b->off[k];
    d[k].dst = b->state[1] + b->off[k];
    set_tiling(&d[k], v);
    const bool front = split && front_strip(p);
    const int w = split ? front_cols(v, p.nx) : 0;  // front strip columns
    if (front) {
      // strip 0 narrowed to the front strip's w columns: step n + 1 on
      // columns [0, w + 1), step n + 2 (and the statistics) on [0, w)
      d[k].x_lim = (int32_t)std::min<int64_t>(w + 1, p.nx);
      d[k].x_cnt = (int32_t)std::min<int64_t>(w, p.nx);
      d[k].x_shift = v.bx - 4 - w;
      d[k].tiles_x = (int32_t)((p.nx + d[k].x_shift + v.bx - 5) / (v.bx - 4));
      d[k].nitems = (int32_t)shifted_items(v, p.nx, p.ny);
      d[k].per_xcd = (d[k].nitems + 7) / 8;
    }
    const int64_t nt = d[k].nitems;
    d[k].slots = b->slots + sbase;
    b->first_item[k] = sbase;
    for (int64_t i = 0; i < nt; ++i) {
      t.push_back(make_int2(k, (int)i));
      if (split) fl.push_back(front && i % d[k].tiles_x == 0 ? 1 : 0);
    }
    const int64_t nf = front ? front_items(p) : 0;
    for (int64_t i = 0; i < nf; ++i) ft.push_back(make_int2(k, (int)i));
    b->nitems_inst[k] = nt + nf;
    sbase += nt + nf;
  }
  b->nitems = (int64_t)t.size();
  b->nfitems = (int64_t)ft.size();
  BCHK(b, hipMemcpyAsync(b->descs, d.data(), d.size() * sizeof(StepArgs),
                         hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->items, t.data(), t.size() * sizeof(int2),
                         hipMemcpyHostToDevice, b->stream));
  if (split) {
    BCHK(b, hipMemcpyAsync(b->flags, fl.data(), fl.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
    if (!ft.empty())
      BCHK(b, hipMemcpyAsync(b->fitems, ft.data(), ft.size() * sizeof(int2),
                             hipMemcpyHostToDevice, b->stream));
  }
  BCHK(b, zero_async(b->slots, b->nslots * sizeof(StatSlot), b->stream));
  if (split && !b->side) {
    BCHK(b, hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    BCHK(b, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    BCHK(b, hipEventCreateWithFlags(&b->join, hipEventDisableTiming));
  }
  BCHK(b, hipStreamSynchronize(b->stream));
  drop_graphs(b);
  return LBM_STEFAN_OK;
}

// one launch from buffer `parity`: one step, or two under a two-step
// variant (one if two = false); two steps of a split schedule are the
// front kernel, the quiet pass and the full pass over flagged items
hipError_t launch_batch(const lbm_stefan_batch_t *b, hipStream_t stream,
                        int parity, bool two = true) {
  int nv;
  const Variant *vt = variants(b->q, &nv);
  const Variant &v = vt[b->variant];
  BatchLaunch L;
  L.descs = b->descs;
  L.items = b->items;
  L.nitems = b->nitems;
  L.cus = b->cus;
  L.blocks_per_cu = b->blocks_per_cu;
  L.parity = parity;
  L.two = two;
  if (!(v.tb == 2 && b->split_ok && two))
    return batch_launch(b->mode, b->q, b->storage, L, v, stream);
  // the front kernel (latency-bound: the Newton solves) on the side
  // stream, the quiet pass (bandwidth-bound) beside it; the full pass over
  // flagged items after both
  const bool fr = b->nfitems > 0;
  if (fr) {
    hipError_t e = hipEventRecord(b->fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->fork, 0);
    if (e != hipSuccess) return e;
    BatchLaunch F = L;
    F.items = b->fitems;
    F.nitems = b->nfitems;
    F.front = true;
    e = batch_launch(b->mode, b->q, b->storage, F, v, b->side);
    if (e == hipSuccess) e = hipEventRecord(b->join, b->side);
    if (e != hipSuccess) return e;
  }
  L.flags = b->flags;
  L.split = 1;
  hipError_t e = batch_launch(b->mode, b->q, b->storage, L, v, stream);
  if (e == hipSuccess && fr) e = hipStreamWaitEvent(stream, b->join, 0);
  if (e != hipSuccess) return e;
  L.split = 2;
  return batch_launch(b->mode, b->q, b->storage, L, v, stream);
}

// time steps one launch advances under the current variant
int steps_per_launch(const lbm_stefan_batch_t *b) {
  int nv;
  return variants(b->q, &nv)[b->variant].tb ? 2 : 1;
}

// graph of the launches of graph_steps steps starting at parity `par`
int ensure_graph(lbm_stefan_batch_t *b, int par) {
  if (b->graph[par]) return LBM_STEFAN_OK;
  if (!b->cap_stream)
    BCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  BCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  const int launches = b->graph_steps / steps_per_launch(b);
  for (int s = 0; s < launches && le == hipSuccess; ++s)
    le = launch_batch(b, b->cap_stream, par ^ (s & 1));
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->cap_stream, &g);
  if (le != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bfail(b, LBM_STEFAN_EDEVICE,
                 std::string("graph capture failed: ") +
                     hipGetErrorString(le != hipSuccess ? le : ee));
  }
  const hipError_t ie = hipGraphInstantiate(&b->graph[par], g, nullptr,
                                            nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    b->graph[par] = nullptr;
    return bfail(b, LBM_STEFAN_EDEVICE,
                 std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  }
  return LBM_STEFAN_OK;
}

}  // namespace

extern "C" {

const char *lbm_stefan_batch_last_error(const lbm_stefan_batch_t *b) {
  return b ? b->err.c_str() : lbm_stefan_last_error(nullptr);
}

int lbm_stefan_batch_workspace_bytes(const lbm_stefan_params *ps,
                                     int32_t count, size_t *bytes) {
  const std::string e = validate_batch(ps, count);
  if (!e.empty()) return bfail(nullptr, LBM_STEFAN_EINVAL, e);
  if (!bytes) return bfail(nullptr, LBM_STEFAN_EINVAL, "bytes is NULL");
  *bytes = batch_layout(ps, count).total;
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_init(const lbm_stefan_params *ps, int32_t count,
                          const double *const *T0, void *workspace,
                          size_t bytes, void *stream,
                          lbm_stefan_batch_t **out) {
  const std::string e = validate_batch(ps, count);
  if (!e.empty()) return bfail(nullptr, LBM_STEFAN_EINVAL, e);
  if (!out) return bfail(nullptr, LBM_STEFAN_EINVAL, "out is NULL");
  *out = nullptr;
  const BLayout L = batch_layout(ps, count);
  if (!workspace || bytes < L.total)
    return bfail(nullptr, LBM_STEFAN_EINVAL, "workspace too small");
  if ((uintptr_t)workspace % 256)
    return bfail(nullptr, LBM_STEFAN_EINVAL, "workspace not 256-byte aligned");
  lbm_stefan_batch_t *b = new (std::nothrow) lbm_stefan_batch_t();
  if (!b) return bfail(nullptr, LBM_STEFAN_EDEVICE, "out of host memory");
  auto bail = [&](int code) {
    set_global_error(b->err);
    drop_graphs(b);
    drop_side(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return code;
  };
  b->ps.assign(ps, ps + count);
  b->count = count;
  b->q = ps[0].q;
  b->storage = ps[0].storage;
  b->mode = mode_of(ps[0]);
  b->stream = (hipStream_t)stream;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount,
                            b->device) != hipSuccess)
    return bail(bfail(b, LBM_STEFAN_EDEVICE, "device query failed"));
  b->variant = b->q == 3 ? kDefaultVariant1D : kDefaultVariant2D;
  char *ws = (char *)workspace;
  b->ws = ws;
  b->descs = (StepArgs *)(ws + L.descs);
  b->items = (int2 *)(ws + L.items);
  b->slots = (StatSlot *)(ws + L.slots);
  b->split_ok = L.split_ok;
  b->nslots = L.nslots;
  if (L.split_ok) {
    b->flags = (int *)(ws + L.flags);
    b->fitems = (int2 *)(ws + L.fitems);
  }
  b->profs = (double *)(ws + L.profs);
  b->partials = (double *)(ws + L.partials);
  b->small = (double *)(ws + L.small);
  b->state[0] = ws + L.stateA;
  b->state[1] = ws + L.stateB;
  b->state_bytes = L.state_bytes;
  b->off = L.off;
  b->prof_off = L.prof_off;
  b->max_items = L.max_items;
  for (int k = 0; k < count; ++k) {
    lbm_stefan_params &p = b->ps[k];
    if (p.dx == 0.0) p.dx = 1.0 / (double)(p.nx - 1);
    if (p.dim == 1) p.bc[2] = p.bc[3] = LBM_BC_PERIODIC;
    const int64_t plen = std::max(p.nx, p.ny);
    for (int w = 0; w < 4; ++w) {
      if (!ps[k].wall_profile[w] || (p.dim == 1 && w >= 2)) {
        p.wall_profile[w] = nullptr;
        continue;
      }
      const int64_t len = w < 2 ? p.ny : p.nx;
      for (int64_t j = 0; j < len; ++j)
        if (!std::isfinite(ps[k].wall_profile[w][j]))
          return bail(bfail(b, LBM_STEFAN_EINVAL, "wall profile not finite"));
      if (hipMemcpy(b->profs + L.prof_off[k] + w * plen, ps[k].wall_profile[w],
                    len * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bail(bfail(b, LBM_STEFAN_EDEVICE, "copy of a wall profile failed"));
      p.wall_profile[w] = b->profs + L.prof_off[k] + w * plen;  // marker only
    }
  }
  if (build_schedule(b) != LBM_STEFAN_OK) return bail(LBM_STEFAN_EDEVICE);
  // initial states; T0 of instance k is staged through its B buffer
  std::vector<StepArgs> d(count);
  if (hipMemcpy(d.data(), b->descs, count * sizeof(StepArgs),
                hipMemcpyDeviceToHost) != hipSuccess)
    return bail(bfail(b, LBM_STEFAN_EDEVICE, "descriptor readback failed"));
  for (int k = 0; k < count; ++k) {
    const double *t0 = T0 ? T0[k] : nullptr;
    const int64_t n = b->ps[k].nx * b->ps[k].ny;
    double *stage = (double *)(b->state[1] + b->off[k]);
    if (t0 && hipMemcpy(stage, t0, n * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bail(bfail(b, LBM_STEFAN_EDEVICE, "copy of T0 failed"));
    StepArgs A = d[k];
    A.dst = b->state[0] + b->off[k];
    if (init_async(b->q, b->storage, A, t0 ? stage : nullptr, b->stream) !=
        hipSuccess)
      return bail(bfail(b, LBM_STEFAN_EDEVICE, "init kernel failed"));
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess)
    return bail(bfail(b, LBM_STEFAN_EDEVICE, "init failed"));
  *out = b;
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_set_schedule(lbm_stefan_batch_t *b, int32_t variant,
                                  int32_t blocks_per_cu, int32_t graph_steps) {
  if (!b) return bfail(nullptr, LBM_STEFAN_EINVAL, "batch is NULL");
  int nv;
  const Variant *vt = variants(b->q, &nv);
  if (variant < -1 || variant >= nv)
    return bfail(b, LBM_STEFAN_EINVAL, "unknown kernel variant");
  if (variant >= 0 && vt[variant].res)
    return bfail(b, LBM_STEFAN_EINVAL,
                 "the resident variant runs single lattices only");
  if (blocks_per_cu < 0 || blocks_per_cu > 32)
    return bfail(b, LBM_STEFAN_EINVAL, "blocks_per_cu must be in 0..32");
  if (graph_steps < 0 || graph_steps % 2 || graph_steps > 100000)
    return bfail(b, LBM_STEFAN_EINVAL,
                 "graph_steps must be even and in 0..100000");
  const int nvar = variant < 0 ? (b->q == 3 ? kDefaultVariant1D
                                            : kDefaultVariant2D)
                               : variant;
  DeviceGuard g(b->device);
  b->blocks_per_cu = blocks_per_cu;
  b->graph_steps = graph_steps;
  drop_graphs(b);
  if (nvar != b->variant) {
    b->variant = nvar;
    return build_schedule(b);
  }
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_step(lbm_stefan_batch_t *b, int64_t nsteps) {
  if (!b) return bfail(nullptr, LBM_STEFAN_EINVAL, "batch is NULL");
  if (nsteps < 0) return bfail(b, LBM_STEFAN_EINVAL, "nsteps < 0");
  DeviceGuard g(b->device);
  const int spl = steps_per_launch(b);
  int64_t left = nsteps;
  if (b->graph_steps > 0) {
    while (left >= b->graph_steps) {
      const int rc = ensure_graph(b, b->cur);
      if (rc) return rc;
      BCHK(b, hipGraphLaunch(b->graph[b->cur], b->stream));
      left -= b->graph_steps;
      b->steps += b->graph_steps;
      b->cur ^= (b->graph_steps / spl) & 1;
    }
  }
  for (; left > 0; left -= std::min<int64_t>(left, spl)) {
    BCHK(b, launch_batch(b, b->stream, b->cur, left >= 2));
    b->cur ^= 1;
    b->steps += std::min<int64_t>(left, spl);
  }
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_reset_stats(lbm_stefan_batch_t *b) {
  if (!b) return bfail(nullptr, LBM_STEFAN_EINVAL, "batch is NULL");
  DeviceGuard g(b->device);
  BCHK(b, zero_async(b->slots, b->nslots * sizeof(StatSlot), b->stream));
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_stats(lbm_stefan_batch_t *b, lbm_stefan_stats *out) {
  if (!b || !out) return bfail(b, LBM_STEFAN_EINVAL, "NULL argument");
  DeviceGuard g(b->device);
  std::vector<double> hs((size_t)b->count * 16);
  for (int k = 0; k < b->count; ++k) {
    const lbm_stefan_params &p = b->ps[k];
    stats_kernel<<<1, 256, 0, b->stream>>>(b->slots + b->first_item[k],
                                           b->nitems_inst[k], b->small + 16 * k);
    BCHK(b, hipGetLastError());
    BCHK(b, energy_async(p, b->state[b->cur] + b->off[k], b->partials,
                         b->small + 16 * k + 8, b->stream));
  }
  BCHK(b, hipMemcpyAsync(hs.data(), b->small, hs.size() * 8,
                         hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  bool finite = true;
  for (int k = 0; k < b->count; ++k) {
    const double *h = &hs[16 * (size_t)k];
    lbm_stefan_stats &s = out[k];
    s.steps = b->steps;
    s.max_newton_it = (int32_t)h[0];
    s.reserved = 0;
    s.nonconverged = (int64_t)h[1];
    s.max_residual = h[2];
    s.flux_in = h[3];
    s.flux_out = h[4];
    s.energy = h[8];
    finite = finite && std::isfinite(s.energy);
  }
  if (!finite) return bfail(b, LBM_STEFAN_ENAN, "an energy is not finite");
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_query_front(lbm_stefan_batch_t *b, int32_t inst,
                                 int32_t mode, double *front, double *energy) {
  if (!b) return bfail(nullptr, LBM_STEFAN_EINVAL, "batch is NULL");
  if (inst < 0 || inst >= b->count)
    return bfail(b, LBM_STEFAN_EINVAL, "instance out of range");
  if (mode != LBM_FRONT_LIQUID_INTEGRAL && mode != LBM_FRONT_ZERO_CROSSING)
    return bfail(b, LBM_STEFAN_EINVAL, "unknown front mode");
  DeviceGuard g(b->device);
  const lbm_stefan_params &p = b->ps[inst];
  const char *src = b->state[b->cur] + b->off[inst];
  double *fr = b->small + 16 * (int64_t)b->count + 16;
  if (front) {
    BCHK(b, front_async(p, src, mode, fr, b->stream));
    BCHK(b, hipMemcpyAsync(front, fr, p.ny * 8, hipMemcpyDeviceToHost,
                           b->stream));
  }
  double e = 0.0;
  if (energy) {
    BCHK(b, energy_async(p, src, b->partials,
                         b->small + 16 * (int64_t)b->count, b->stream));
    BCHK(b, hipMemcpyAsync(&e, b->small + 16 * (int64_t)b->count, 8,
                           hipMemcpyDeviceToHost, b->stream));
  }
  BCHK(b, hipStreamSynchronize(b->stream));
  if (energy) {
    *energy = e;
    if (!std::isfinite(e)) return bfail(b, LBM_STEFAN_ENAN, "energy not finite");
  }
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_get_field(lbm_stefan_batch_t *b, int32_t inst,
                               int32_t what, void *host) {
  if (!b) return bfail(nullptr, LBM_STEFAN_EINVAL, "batch is NULL");
  if (inst < 0 || inst >= b->count || !host)
    return bfail(b, LBM_STEFAN_EINVAL, "bad instance or host pointer");
  DeviceGuard g(b->device);
  const lbm_stefan_params &p = b->ps[inst];
  const int64_t n = p.nx * p.ny;
  const char *src = b->state[b->cur] + b->off[inst];
  if (what == LBM_FIELD_STATE) {
    const size_t s = b->storage == LBM_STORE_F64 ? 8 : 4;
    BCHK(b, hipMemcpyAsync(host, src, p.q * n * s, hipMemcpyDeviceToHost,
                           b->stream));
  } else if (what == LBM_FIELD_T) {
    // the instance's idle buffer holds >= 12 n bytes
    double *T = (double *)(b->state[b->cur ^ 1] + b->off[inst]);
    BCHK(b, temperature_async(p, src, T, b->stream));
    BCHK(b, hipMemcpyAsync(host, T, n * 8, hipMemcpyDeviceToHost, b->stream));
  } else {
    return bfail(b, LBM_STEFAN_EINVAL, "unknown field");
  }
  BCHK(b, hipStreamSynchronize(b->stream));
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_state_bytes(const lbm_stefan_batch_t *b, size_t *bytes) {
  if (!b || !bytes) return bfail(nullptr, LBM_STEFAN_EINVAL, "NULL argument");
  *bytes = b->state_bytes;
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_autotune(lbm_stefan_batch_t *b, void *scratch,
                              size_t scratch_bytes, int32_t steps,
                              int32_t *best_variant, int32_t *best_blocks_per_cu,
                              double *best_ms_per_step) {
  if (!b) return bfail(nullptr, LBM_STEFAN_EINVAL, "batch is NULL");
  if (!scratch || scratch_bytes < b->state_bytes)
    return bfail(b, LBM_STEFAN_EINVAL, "scratch smaller than the state");
  if (steps < 1 || steps > 10000)
    return bfail(b, LBM_STEFAN_EINVAL, "steps must be in 1..10000");
  DeviceGuard g(b->device);
  const int cur0 = b->cur;
  BCHK(b, hipMemcpyAsync(scratch, b->state[cur0], b->state_bytes,
                         hipMemcpyDeviceToDevice, b->stream));
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, LBM_STEFAN_EDEVICE, "hipEventCreate failed");
  }
  int nv;
  const Variant *vt = variants(b->q, &nv);
  const int bpcs[] = {0, 2, 4, 8};
  const int v0 = b->variant, bpc0 = b->blocks_per_cu;
  int best_v = v0, best_bpc = bpc0;
  float best_ms = -1.0f;
  int rc = LBM_STEFAN_OK;
  hipError_t err = hipSuccess;
  for (int v = 0; v < nv && rc == LBM_STEFAN_OK && err == hipSuccess; ++v) {
    if (vt[v].res) continue;  // single lattices only
    if (v != b->variant) {
      b->variant = v;
      rc = build_schedule(b);
    }
    // a two-step launch covers two steps; the persistent grid is for
    // one-step variants only
    const int spl = vt[v].tb ? 2 : 1;
    const int launches = (steps + spl - 1) / spl;
    for (int bpc : bpcs) {
      if (rc != LBM_STEFAN_OK || err != hipSuccess) break;
      if (vt[v].tb && bpc > 0) break;
      b->blocks_per_cu = bpc;
      for (int s = 0; s < launches + 2 && err == hipSuccess; ++s) {
        if (s == 2) err = hipEventRecord(e0, b->stream);
        if (err == hipSuccess) err = launch_batch(b, b->stream, b->cur);
        b->cur ^= 1;
      }
      if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      ms /= (float)(launches * spl);
      if (err == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
        best_ms = ms;
        best_v = v;
        best_bpc = bpc;
      }
      b->cur = cur0;
      if (err == hipSuccess)
        err = hipMemcpyAsync(b->state[cur0], scratch, b->state_bytes,
                             hipMemcpyDeviceToDevice, b->stream);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->cur = cur0;
  if (rc != LBM_STEFAN_OK) return rc;
  if (err != hipSuccess)
    return bfail(b, LBM_STEFAN_EDEVICE,
                 std::string("autotune: ") + hipGetErrorString(err));
  b->blocks_per_cu = best_bpc;
  if (best_v != b->variant) {
    b->variant = best_v;
    rc = build_schedule(b);
    if (rc) return rc;
  } else {
    BCHK(b, zero_async(b->slots, b->nslots * sizeof(StatSlot), b->stream));
  }
  drop_graphs(b);
  BCHK(b, hipStreamSynchronize(b->stream));
  if (best_variant) *best_variant = best_v;
  if (best_blocks_per_cu) *best_blocks_per_cu = best_bpc;
  if (best_ms_per_step) *best_ms_per_step = best_ms;
  return LBM_STEFAN_OK;
}

int lbm_stefan_batch_destroy(lbm_stefan_batch_t *b) {
  if (!b) return LBM_STEFAN_OK;
  DeviceGuard g(b->device);
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess && b->side) e = hipStreamSynchronize(b->side);
  drop_graphs(b);
  drop_side(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  if (e != hipSuccess) return bfail(nullptr, LBM_STEFAN_EDEVICE, hipGetErrorString(e));
  return LBM_STEFAN_OK;
}

}  // extern "C"
