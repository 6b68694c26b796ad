// kernels.hpp -- gfx950 kernels of the IREBM step and its reductions.
// Included by each translation unit of the library; the kernels sit in an
// anonymous namespace so every unit registers its own copies.
//
//   step_kernel      one time step, one launch; each block owns a work
//                    item of `group` tiles stacked along y (a tile is
//                    bx * npt columns by by rows).  Blocks are remapped so
//                    that each of the eight XCDs sweeps one contiguous
//                    band of tile rows: the rows a tile pulls from its
//                    neighbours then sit in that XCD's L2.  Interior tiles take a path with no bounds
//                    checks.  Per-item Newton and flux statistics are
//                    accumulated by the owning block (no atomics).
//   init_kernel      equilibrium state from a temperature field.
//   temp_kernel      T = sum_i Omega_i (EEBM: Theta of that enthalpy).
//   energy_*         E = sum [T + phi(T)/Ste] (EEBM: sum H), two
//                    fixed-order passes.
//   front_*          per-row front position.
//   stats_kernel     fixed-order reduction of per-item slots.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "irebm_node.hpp"

namespace irebm {

constexpr int kEnergyChunk = 2048;  // nodes per energy partial

// Statistics of one block (already reduced over the node loop of each
// thread), combined across the block and added by thread 0 to the item's
// slot, whose previous value `pre` thread 0 loaded (blocks of up to 1024
// threads).  LOOP: the block goes on to another item, so the shared arrays
// are fenced again.
template <bool LOOP>
__device__ __forceinline__ void block_stats_to_slot(const NodeStats &st,
                                                    bool fast,
                                                    const StatSlot &pre,
                                                    StatSlot *sl) {
  __shared__ int s_it[16], s_nc[16];
  __shared__ double s_res[16], s_fin[16], s_fout[16];
  const int lin = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int wid = lin >> 6, nw = (int)(blockDim.x * blockDim.y) >> 6;
  const int it = wave_max_i(st.max_it);
  const int nc = wave_sum_i(st.nonconv);
  const double res = wave_max(st.max_res);
  double fin = 0.0, fout = 0.0;
  if (!fast) {
    fin = wave_sum(st.flux_in);
    fout = wave_sum(st.flux_out);
  }
  if ((lin & 63) == 0) {
    s_it[wid] = it;
    s_nc[wid] = nc;
    s_res[wid] = res;
    s_fin[wid] = fin;
    s_fout[wid] = fout;
  }
  __syncthreads();
  if (lin == 0) {
    int bit = s_it[0], bnc = s_nc[0];
    double bres = s_res[0], bfin = s_fin[0], bfout = s_fout[0];
    for (int w = 1; w < nw; ++w) {
      bit = max(bit, s_it[w]);
      bnc += s_nc[w];
      bres = fmax(bres, s_res[w]);
      bfin += s_fin[w];
      bfout += s_fout[w];
    }
    StatSlot out = pre;
    out.max_it = max(pre.max_it, bit);
    out.nonconv = pre.nonconv + bnc;
    out.max_res = fmax(pre.max_res, bres);
    if (!fast) {
      out.flux_in = pre.flux_in + bfin;
      out.flux_out = pre.flux_out + bfout;
    }
    *sl = out;
  }
  if (LOOP) __syncthreads();
}

// One tile (tx, ty) of the lattice described by A, from state src to
// state dst: on interior tiles all loads of the thread's nodes first
// (memory-level parallelism), then the updates.  Statistics go into st;
// returns whether the tile took the interior path.
template <int Q, typename S, int NPT, int MODE, bool NT>
__device__ __forceinline__ bool step_tile(const StepArgs &A,
                                          gptr<const S> __restrict__ src,
                                          gptr<S> __restrict__ dst, int tx,
                                          int ty, NodeStats &st) {
  const int bx = blockDim.x, by = blockDim.y;
  const int TW = bx * NPT;
  const int x0 = tx * TW, y0 = ty * by;
  const bool fast = x0 >= 1 && x0 + TW <= A.nx - 1 &&
                    (Q == 3 || (y0 >= 1 && y0 + by <= A.ny - 1));
  // a wave lies in one row of the tile (bx is a multiple of 64)
  const int y = y0 + __builtin_amdgcn_readfirstlane((int)threadIdx.y);
  if (fast) {
    NodeLoad<Q, S> L[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      load_node<Q, S, true>(A, src, x0 + (int)threadIdx.x + k * bx, y, L[k]);
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      update_node<Q, S, MODE, true, NT>(A, dst, x0 + (int)threadIdx.x + k * bx,
                                         y, L[k], st);
  } else {
    // boundary tiles: one node at a time keeps the register count of the
    // interior path; the loads of a node are still issued together.  At
    // the x = 0 wall (where the workloads heat, so where their melting
    // front starts) the first bx columns of the tile are dealt out column
    // by column: the by nodes of a column side by side in a wave, 64 / by
    // columns per wave.  The front then falls into the first wave of the
    // tile instead of into one wave per row, so by times fewer waves run
    // the Newton solve of the nodes in and near the band.  Other nodes
    // keep one row per wave (whole-row loads).  (by is a power of two.)
    const int tid = (int)threadIdx.x + (int)threadIdx.y * bx;
    const int lb = __builtin_ctz((unsigned)by);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const bool cm = k == 0 && x0 == 0;
      const int x = cm ? (tid >> lb) : x0 + (int)threadIdx.x + k * bx;
      const int yj = cm ? y0 + (tid & (by - 1)) : y;
      if (x < A.nx && yj < A.ny) {
        NodeLoad<Q, S> L;
        load_node<Q, S, false, neumann_mode(MODE)>(A, src, x, yj, L);
        update_node<Q, S, MODE, false, NT>(A, dst, x, yj, L, st);
      }
    }
  }
  return fast;
}

// One work item: tile rows ty0 .. ty0 + group - 1 of tile column tx
// (fewer at the top of the lattice), swept upward by one block, so the
// rows a tile pulls from below were just read by the same block, and the
// block's start-up (descriptor and slot reads) and statistics reduction
// are paid once per item.  One statistics slot per item.
template <int Q, typename S, int NPT, int MODE, bool NT = false,
          bool LOOP = false>
__device__ __forceinline__ void step_item(const StepArgs &A,
                                          gptr<const S> __restrict__ src,
                                          gptr<S> __restrict__ dst, int item,
                                          StatSlot *slot) {
  const int tx = item % A.tiles_x;
  const int ty0 = (item / A.tiles_x) * A.group;
  const int rows = min(A.group, A.tiles_y - ty0);
  NodeStats st;
  bool fast = true;
  for (int r = 0; r < rows; ++r) {
    // Re-read the (uniform) arguments in every pass: an index the compiler
    // cannot see through keeps it from hoisting all of them out of the
    // loop, which would hold ~80 more scalar registers live across it and
    // spill them into vector registers (lower occupancy).
    int z = 0;
    asm volatile("" : "+s"(z));
    fast &= step_tile<Q, S, NPT, MODE, NT>((&A)[z], src, dst, tx, ty0 + r,
                                           st);
  }
  // read after the loop: a prefetched slot would stay live across it
  StatSlot pre{};
  if (threadIdx.x == 0 && threadIdx.y == 0) pre = *slot;
  block_stats_to_slot<LOOP>(st, fast, pre, slot);
}

// work item of block b: the blocks of XCD k (b mod 8 = k) take the k-th
// contiguous chunk of the item order, optionally swept backwards
__device__ __forceinline__ int xcd_item(int b, int per_xcd, int nitems,
                                        int reverse) {
  const int t = (b & 7) * per_xcd + (b >> 3);
  return reverse ? nitems - 1 - t : t;
}

// The same chunks, each XCD taking the x = 0 tiles of its chunk first (the
// items t with t mod tiles_x = 0, where a heated x = 0 wall puts the
// melting front), then the others in order: the tiles whose Newton solves
// make them the longest start first, and their latency hides under the
// rest of the chunk instead of ending it.  A permutation of the items
// within each chunk (the caller has checked that block b has an item).
__device__ __forceinline__ int xcd_item_front_first(int b, int per_xcd,
                                                    int nitems, int tiles_x) {
  const int c0 = (b & 7) * per_xcd, j = b >> 3;
  const int c1 = min(c0 + per_xcd, nitems);
  const int base = (c0 / tiles_x) * tiles_x, r0 = c0 - base;
  const int f0 = r0 == 0 ? c0 : base + tiles_x;   // first x = 0 item
  const int nf = f0 < c1 ? (c1 - 1 - f0) / tiles_x + 1 : 0;
  if (j < nf) return f0 + j * tiles_x;
  // the (j - nf)-th item with x > 0: items with x > 0 counted from base
  const int w = tiles_x - 1;
  const int rk = (r0 == 0 ? 0 : r0 - 1) + (j - nf);
  return base + (rk / w) * tiles_x + rk % w + 1;
}

namespace {


// one time step of one lattice, one block per work item (XCD-aware order)
template <int Q, typename S, int NPT, int MODE, bool NT>
__global__ __launch_bounds__(256) void step_kernel(StepArgs A) {
  const int b = blockIdx.x;
  if ((b & 7) * A.per_xcd + (b >> 3) >= A.nitems) return;
  const int t = A.front_first && !A.reverse
                    ? xcd_item_front_first(b, A.per_xcd, A.nitems, A.tiles_x)
                    : xcd_item(b, A.per_xcd, A.nitems, A.reverse);
  step_item<Q, S, NPT, MODE, NT>(A, to_global((const S *)A.src),
                                  to_global((S *)A.dst), t, A.slots + t);
}

// ---------------------------------------------------------------------
// two time steps per launch (temporal blocking)
//
// Each block owns a strip of WIN - 4 columns and a segment of rows of the
// output, and sweeps the segment upward with a window of WIN columns (2
// halo columns on each side).  Per pass it loads BY new rows of the state
// at step n into a ring in LDS, computes BY rows of step n + 1 from that
// ring into a second ring (a halo of one row and one column around the
// block's part is recomputed by the neighbours as well), and BY rows of
// step n + 2 from the second ring, which it writes.  So a node pair of
// steps moves q s bytes in and q s bytes out, half of two single steps,
// and every node update is the same code (update_values) on the same
// operands, so the result equals two single steps bit for bit.
// Statistics count each node once per step: only the nodes of the
// block's own part, at both levels.
//
// Loads and stores share one counter on this chip, and a wait for the
// prefetched rows waits for every store issued before them as well; so
// the rows of step n + 2 are stored at the top of the next pass, right
// after the wait and before the next prefetch, which leaves a whole pass
// for both to complete.

// NodeLoad of node (x, y) (lattice coordinates) from a ring of rows in
// LDS: column t of the window, ring slot of row r at (r - base) % RING.
// INNER: every pull source is a lattice node and nothing leaves (no masks).
// The Neumann closure reads two cells away, beyond the ring's reach, so
// lattices with a Neumann wall never take the two-step kernel (host).
template <int Q, typename S, int RING, int WIN, bool INNER>
__device__ __forceinline__ void load_ring(const StepArgs &A,
                                          const S (*ring)[Q][WIN],
                                          int x, int y, int t, int r, int base,
                                          NodeLoad<Q, S> &L) {
  if (INNER) {
    L.known = (1u << Q) - 1u;
    L.out = 0u;
  } else {
    node_masks<Q>(A, x, y, L.known, L.out);
  }
  L.mirror = 0.0;
  const unsigned so = (unsigned)(r - base) % RING;
#pragma unroll
  for (int j = 0; j < Q; ++j) L.own[j] = ring[so][j][t];
  L.pull[0] = L.own[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int ex = cx<Q>(i), ey = cy<Q>(i);
    const S v = ring[(unsigned)(r - ey - base) % RING][i][t - ex];
    L.pull[i] = (INNER || (L.known >> i & 1u)) ? v : (S)0;
  }
}

// the update of node (x, y) of a window from a ring: the interior form
// (no masks, no closures) when every neighbour is a lattice node
template <int Q, typename S, int MODE, int RING, int WIN, bool QUIET = false>
__device__ __forceinline__ void ring_update(const StepArgs &A,
                                            const S (*ring)[Q][WIN], int x,
                                            int y, int t, int r, int base,
                                            bool inner, NodeStats &st, S v[Q]) {
  NodeLoad<Q, S> L;
  if (inner) {
    load_ring<Q, S, RING, WIN, true>(A, ring, x, y, t, r, base, L);
    update_values<Q, S, MODE, true, QUIET>(A, x, y, L, st, v);
  } else {
    load_ring<Q, S, RING, WIN, false>(A, ring, x, y, t, r, base, L);
    update_values<Q, S, MODE, false, QUIET>(A, x, y, L, st, v);
  }
}

// One block: strip `strip` of segment `seg` (seg_rows rows) of the lattice
// described by A, from state src to state dst, two steps (two = true) or
// one (the rows of step n + 1 are then written out directly).
// QUIET: node updates of quiet nodes only (no Newton code); when any node
// of the window, halo included, is not quiet, the item's statistics are
// not added (its outputs are then rewritten by a full kernel).  Returns,
// for QUIET and FLAGGED (a full kernel over flagged items), whether any
// node of the window took (or needed) the Newton path.
template <int Q, typename S, int MODE, bool NT, int BY, int WIN,
          bool QUIET = false, bool FLAGGED = false>
__device__ __forceinline__ bool step2_body(const StepArgs &A,
                                           gptr<const S> __restrict__ src,
                                           gptr<S> __restrict__ dst, int strip,
                                           int seg, int seg_rows, bool two,
                                           StatSlot *slot) {
  constexpr int RING = BY + 2;
  __shared__ S l0[RING][Q][WIN];
  __shared__ S l1[RING][Q][WIN];
  // a wave lies in one row of threads (WIN is a multiple of 64)
  const int t = (int)threadIdx.x;
  const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
  const int s0 = seg * seg_rows;
  const int s1 = min(s0 + seg_rows, A.ny);       // output rows [s0, s1)
  const int x = strip * (WIN - 4) - 2 + t - A.x_shift;  // window column
  const int nx = A.nx, ny = A.ny;
  const int64_t P = A.plane;
  const bool px = A.periodic_x != 0, py = A.periodic_y != 0;
  // lattice column of this window column (wrapped on a periodic axis)
  int gx = x;
  bool col = x >= 0 && x < nx;
  if (!col && px) {
    gx = (x % nx + nx) % nx;
    col = true;
  }
  // every neighbour of the node at window column t is a lattice node along x
  const bool inner_x = px || (x >= 1 && x <= nx - 2);
  const bool own_col = t >= 2 && t < WIN - 2 && x >= 0 && x < nx;
  // ring slots: (row - base) % RING with base a multiple of RING below
  // every row touched (rows >= s0 - 4)
  const int base = s0 - 12;
  // lattice row of row r (wrapped on a periodic axis), or -1
  auto lrow = [&](int r) -> int {
    if (r >= 0 && r < ny) return r;
    return py ? (r % ny + ny) % ny : -1;
  };
  const int iters = (s1 - s0 + 4 + BY - 1) / BY;
  S pf[Q];
  {
    const int gr = lrow(s0 - 2 + ty);
    const int64_t o = (int64_t)(gr < 0 ? 0 : gr) * nx + (col ? gx : 0);
#pragma unroll
    for (int j = 0; j < Q; ++j) pf[j] = src[j * P + o];
  }
  S w[Q];            // a row of output waiting to be stored
  int64_t wo = -1;   // its offset, or -1
  NodeStats st;
  for (int i = 0; i < iters; ++i) {
    // arguments re-read in every pass (see step_item)
    int z = 0;
    asm volatile("" : "+s"(z));
    const StepArgs &Ai = (&A)[z];
    const int a = s0 - 2 + i * BY;
    // rows a .. a + BY - 1 of step n into the first ring
#pragma unroll
    for (int j = 0; j < Q; ++j)
      l0[(unsigned)(a + ty - base) % RING][j][t] = pf[j];
    if (wo >= 0) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        if (NT) __builtin_nontemporal_store(w[j], dst + j * P + wo);
        else dst[j * P + wo] = w[j];
      }
      wo = -1;
    }
    if (i + 1 < iters) {
      const int gr = lrow(a + BY + ty);
      const int64_t o = (int64_t)(gr < 0 ? 0 : gr) * nx + (col ? gx : 0);
#pragma unroll
      for (int j = 0; j < Q; ++j) pf[j] = src[j * P + o];
    }
    __syncthreads();
    // step n + 1 at row b (needed rows s0 - 1 .. s1; for one step only
    // the block's own rows, stored in the next pass)
    if (!two) {
      const int b = a - 1 + ty;
      if (own_col && b >= s0 && b < s1) {
        const bool inner = inner_x && (py || (b >= 1 && b <= ny - 2));
        ring_update<Q, S, MODE, RING, WIN, QUIET>(Ai, l0, x, b, t, b, base,
                                                   inner, st, w);
        wo = (int64_t)b * nx + x;
      }
    } else {
      const int b = a - 1 + ty;
      const int gb = lrow(b);
      if (t >= 1 && t < WIN - 1 && col && gb >= 0 && b >= s0 - 1 && b <= s1) {
        S v[Q];
        NodeStats one;
        const bool inner = inner_x && (py || (gb >= 1 && gb <= ny - 2));
        ring_update<Q, S, MODE, RING, WIN, QUIET>(Ai, l0, gx, gb, t, b, base,
                                                   inner, one, v);
        if (own_col && b >= s0 && b < s1) {
          st.max_it = max(st.max_it, one.max_it);
          st.nonconv += one.nonconv;
          st.max_res = fmax(st.max_res, one.max_res);
          st.flux_in += one.flux_in;
          st.flux_out += one.flux_out;
        }
        st.solves += one.solves;   // halo nodes too: own nodes use them
#pragma unroll
        for (int j = 0; j < Q; ++j) l1[(unsigned)(b - base) % RING][j][t] = v[j];
      }
    }
    __syncthreads();
    // step n + 2 at row c (stored in the next pass)
    if (two) {
      const int c = a - 2 + ty;
      if (own_col && c >= s0 && c < s1) {
        const bool inner = inner_x && (py || (c >= 1 && c <= ny - 2));
        ring_update<Q, S, MODE, RING, WIN, QUIET>(Ai, l1, x, c, t, c, base,
                                                   inner, st, w);
        wo = (int64_t)c * nx + x;
      }
    }
  }
  if (wo >= 0) {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      if (NT) __builtin_nontemporal_store(w[j], dst + j * P + wo);
      else dst[j * P + wo] = w[j];
    }
  }
  bool any = false;
  if constexpr (QUIET || FLAGGED)
    any = __syncthreads_or(st.solves > 0) != 0;
  if (!QUIET || !any) {
    StatSlot pre{};
    if (t == 0 && ty == 0) pre = *slot;
    block_stats_to_slot<false>(st, false, pre, slot);
  }
  return any;
}

// ---------------------------------------------------------------------
// front strips of the split two-step schedule (batched form)

template <int Q, typename S, bool NT>
__device__ __forceinline__ void store_values(const StepArgs &A,
                                             gptr<S> __restrict__ dst, int x,
                                             int y, const S v[Q]) {
  const gptr<S> row = dst + (int64_t)y * A.nx;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const gptr<S> p = (row + i * A.plane) + (uint32_t)x;
    if (NT) __builtin_nontemporal_store(v[i], p);
    else *p = v[i];
  }
}

__device__ __forceinline__ void merge_stats(NodeStats &st,
                                            const NodeStats &one) {
  st.max_it = max(st.max_it, one.max_it);
  st.nonconv += one.nonconv;
  st.max_res = fmax(st.max_res, one.max_res);
  st.flux_in += one.flux_in;
  st.flux_out += one.flux_out;
}

// rows of a front segment: R + 2 rows of step n + 1 fill 256 threads
// evenly (4 rows of 64 columns per pass)
template <typename S>
constexpr int front_rows() { return sizeof(S) == 4 ? 10 : 6; }

// Two steps of segment `seg` (front_rows<S>() rows) of an instance's front
// strip, one block of 256 threads: step n + 1 of the segment's rows and of
// one halo row on each side (recomputed by the neighbouring segments as
// well) on columns [0, A.x_lim), from the global state into LDS, then,
// after one barrier, step n + 2 of the segment's rows on columns
// [0, A.x_cnt) from LDS into dst.  One node per thread at a time (the slow
// path's loads), whole rows per wave.  No third state and no wait for the
// other segments between the two steps.  The strip lies at the x = 0 wall
// of a lattice that is not periodic along x and is at most 64 columns
// wide (both checked by the host), so LDS column x is lattice column x
// and the masked pulls from x = -1 (and from x = nx when the strip is the
// whole lattice) are the only reads outside the columns computed.
// Statistics count each node once per step (own rows, columns below
// x_cnt).
template <int Q, typename S, int MODE>
__device__ __forceinline__ void front2_body(const StepArgs &A,
                                            gptr<const S> __restrict__ src,
                                            gptr<S> __restrict__ dst, int seg,
                                            StatSlot *slot) {
  constexpr int R = front_rows<S>(), RR = R + 2, W = 64;
  __shared__ S buf[RR][Q][W];
  const int tid = (int)threadIdx.x;
  const int ny = A.ny;
  const bool py = A.periodic_y != 0;
  const int y0 = seg * R, y1 = min(y0 + R, ny);
  NodeStats st;
  // step n + 1: LDS row r holds lattice row y0 - 1 + r
  for (int n = tid; n < RR * W; n += 256) {
    int z = 0;
    asm volatile("" : "+s"(z));
    const StepArgs &Ai = (&A)[z];
    const int r = n >> 6, x = n & (W - 1);
    const int yy = y0 - 1 + r;
    int gy = yy;
    if (yy < 0 || yy >= ny) gy = py ? (yy % ny + ny) % ny : -1;
    if (x < Ai.x_lim && gy >= 0 && yy <= y1) {
      NodeLoad<Q, S> L;
      load_node<Q, S, false>(Ai, src, x, gy, L);
      NodeStats one;
      S v[Q];
      update_values<Q, S, MODE, false>(Ai, x, gy, L, one, v);
#pragma unroll
      for (int j = 0; j < Q; ++j) buf[r][j][x] = v[j];
      if (yy >= y0 && yy < y1 && x < Ai.x_cnt) merge_stats(st, one);
    }
  }
  __syncthreads();
  // step n + 2 from LDS
  for (int n = tid; n < R * W; n += 256) {
    int z = 0;
    asm volatile("" : "+s"(z));
    const StepArgs &Ai = (&A)[z];
    const int r = n >> 6, x = n & (W - 1);
    const int y = y0 + r;
    if (x < Ai.x_cnt && y < y1) {
      NodeLoad<Q, S> L;
      node_masks<Q>(Ai, x, y, L.known, L.out);
      L.mirror = 0.0;
#pragma unroll
      for (int j = 0; j < Q; ++j) L.own[j] = buf[r + 1][j][x];
      L.pull[0] = L.own[0];
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int ex = cx<Q>(i), ey = cy<Q>(i);
        const S v = buf[r + 1 - ey][i][(x - ex) & (W - 1)];
        L.pull[i] = (L.known >> i & 1u) ? v : (S)0;
      }
      NodeStats one;
      S v[Q];
      update_values<Q, S, MODE, false>(Ai, x, y, L, one, v);
      store_values<Q, S, true>(Ai, dst, x, y, v);
      merge_stats(st, one);
    }
  }
  StatSlot pre{};
  if (tid == 0) pre = *slot;
  block_stats_to_slot<false>(st, false, pre, slot);
}

// Blocks are numbered strip-fastest within a segment of rows, and each
// XCD takes one contiguous chunk of that order, so neighbouring strips run
// on the same XCD and share the halo lines (and the cache lines that
// straddle two strips) in its L2.
template <int Q, typename S, int MODE, bool NT, int BY, int WIN>
// FP32 states: at most 128 VGPRs (4 waves per SIMD); FP64 rings fill the
// LDS first
__global__ __launch_bounds__(WIN * BY)
__attribute__((amdgpu_waves_per_eu(sizeof(S) == 4 ? 4 : 1)))
void step2_kernel(StepArgs A, int32_t nstrips, int32_t seg_rows,
                  int32_t nitems, int32_t two) {
  const int per_xcd = (nitems + 7) >> 3;
  const int item = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (item >= nitems) return;
  step2_body<Q, S, MODE, NT, BY, WIN>(A, to_global((const S *)A.src),
                                       to_global((S *)A.dst),
                                       item % nstrips, item / nstrips,
                                       seg_rows, two != 0, A.slots + item);
}

// ---------------------------------------------------------------------
// small 1D lattices: many steps in one resident workgroup

// Largest D1Q3 lattice the resident kernel takes: both states of 2048
// nodes fit in LDS (96 KB in FP64).
constexpr int kResident1D = 2048;

// nsteps steps of a D1Q3 lattice of at most kResident1D nodes with no
// Neumann wall, in one workgroup of 1024 threads: the state at A.src is
// loaded once into LDS, each step reads one LDS state and writes the
// other (the same per-node code as step_kernel), a barrier separates the
// steps, and at the end the two LDS
// states go back to the two global buffers exactly as nsteps one-step
// launches would leave them: the last state in A.src when nsteps is even
// (A.dst otherwise), the one before it in the other buffer.  Statistics
// of all nsteps go to slot 0.
template <typename S, int MODE>
__global__ __launch_bounds__(1024) void resident1d_kernel(StepArgs A,
                                                          int32_t nsteps) {
  constexpr int Q = 3;
  __shared__ S st_lds[2][Q][kResident1D];
  const int n = A.nx;
  if (n > kResident1D) return;  // the host never launches such a lattice
  const int t = (int)threadIdx.x;
  const gptr<S> b0 = to_global((S *)A.src);
  const gptr<S> b1 = to_global((S *)A.dst);
  const int64_t P = A.plane;
  for (int x = t; x < n; x += 1024) {
#pragma unroll
    for (int j = 0; j < Q; ++j) st_lds[0][j][x] = b0[j * P + x];
  }
  __syncthreads();
  const bool px = A.periodic_x != 0;
  NodeStats st;
  for (int s = 0; s < nsteps; ++s) {
    const int c = s & 1;
    // arguments read in place each step (see step_item); a by-value copy
    // would index the wall arrays from private memory
    int k0 = 0;
    asm volatile("" : "+s"(k0));
    const StepArgs &B = (&A)[k0];
    for (int x = t; x < n; x += 1024) {
      NodeLoad<Q, S> L;
      // directions +x (1) and -x (2): the pull source x - 1 (x + 1) is a
      // lattice node, or the destination x + 1 (x - 1) leaves the lattice
      // (node_masks for D1Q3, written out)
      const bool vm = x >= 1 || px, vp = x + 1 < n || px;
      L.known = 1u | (vm ? 2u : 0u) | (vp ? 4u : 0u);
      L.out = (vp ? 0u : 2u) | (vm ? 0u : 4u);
      L.mirror = 0.0;
      // pull sources wrapped on a periodic axis, clamped otherwise (then
      // masked)
      const int xm = x >= 1 ? x - 1 : (px ? n - 1 : 0);
      const int xp = x + 1 < n ? x + 1 : (px ? 0 : n - 1);
#pragma unroll
      for (int j = 0; j < Q; ++j) L.own[j] = st_lds[c][j][x];
      L.pull[0] = L.own[0];
      L.pull[1] = (L.known >> 1 & 1u) ? st_lds[c][1][xm] : (S)0;
      L.pull[2] = (L.known >> 2 & 1u) ? st_lds[c][2][xp] : (S)0;
      // the closures run only where a direction is unknown or leaves
      S v[Q];
      update_values<Q, S, MODE, false>(B, x, 0, L, st, v);
#pragma unroll
      for (int i = 0; i < Q; ++i) st_lds[c ^ 1][i][x] = v[i];
    }
    __syncthreads();
  }
  // state k lies in LDS state k % 2, as in global buffer k % 2
  for (int x = t; x < n; x += 1024) {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      b1[j * P + x] = st_lds[1][j][x];
      b0[j * P + x] = st_lds[0][j][x];
    }
  }
  StatSlot pre{};
  if (t == 0) pre = A.slots[0];
  block_stats_to_slot<false>(st, false, pre, A.slots);
}

// ---------------------------------------------------------------------
// init, temperature, zero fill

// IREBM and ILFBM: Omega_i = w_i T (and, when lf is given, the ILFBM
// liquid fraction l = 1 above T_m, else 0).  EEBM: the equilibrium of the
// enthalpy H = T + l(T)/Ste, which collision keeps.
template <int Q, typename S>
__global__ void init_kernel(StepArgs A, const double *T0, double *lf) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.plane) return;
  const int x = (int)(k % A.nx), y = (int)(k / A.nx);
  const int wall = dirichlet_wall<Q>(A, x, y);
  const double T = wall >= 0 ? wall_value(A, wall, x, y) : (T0 ? T0[k] : 0.0);
  S *dst = (S *)A.dst;
  if (lf) lf[k] = T > A.tm ? 1.0 : 0.0;
  if (A.scheme == SCHEME_EEBM) {
    const double H = T + (T > A.tm ? A.inv_ste : 0.0);
    const double th = eebm_theta(H, A.tm, A.inv_ste);
    dst[k] = (S)(H - (1.0 - wt<Q>(0)) * th);
#pragma unroll
    for (int i = 1; i < Q; ++i) dst[i * A.plane + k] = (S)(wt<Q>(i) * th);
    return;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[i * A.plane + k] = (S)(wt<Q>(i) * T);
}

template <int Q, typename S>
__global__ void temp_kernel(const S *src, int64_t plane, int eebm, double tm,
                            double inv_ste, double *T) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= plane) return;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) s += (double)src[j * plane + k];
  T[k] = eebm ? eebm_theta(s, tm, inv_ste) : s;
}

// liquid fraction of every node: phi(T) (IREBM), l(H) (EEBM) or the lf
// plane (ILFBM)
template <int Q, typename S>
__global__ void liquid_kernel(const S *src, int64_t plane, int eebm,
                              double tm, double inv_delta, double ste,
                              const double *lf, double *out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= plane) return;
  if (lf) {
    out[k] = lf[k];
    return;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) s += (double)src[j * plane + k];
  out[k] = eebm ? eebm_lf(s, tm, ste) : phi_only(s, tm, inv_delta);
}

__global__ void zero_kernel(uint64_t *p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

// ---------------------------------------------------------------------
// fixed-order reductions

__device__ __forceinline__ double block_sum_256(double v) {
  __shared__ double s[4];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s[w] = v;
  __syncthreads();
  double r = s[0] + s[1] + s[2] + s[3];
  __syncthreads();
  return r;
}

// partial[b] = sum over nodes [b*chunk, (b+1)*chunk) of T + phi(T)/Ste,
// of the enthalpy M0 itself (eebm), or of T + lf/Ste (lf given: ILFBM)
template <int Q, typename S>
__global__ __launch_bounds__(256) void energy_partial_kernel(
    const S *src, int64_t plane, int eebm, double tm, double inv_delta,
    double inv_ste, const double *lf, double *partial) {
  const int64_t base = (int64_t)blockIdx.x * kEnergyChunk;
  double acc = 0.0;
  for (int j = 0; j < kEnergyChunk / 256; ++j) {
    const int64_t k = base + j * 256 + threadIdx.x;
    if (k < plane) {
      double T = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) T += (double)src[i * plane + k];
      acc += lf ? T + lf[k] * inv_ste
                : (eebm ? T : T + phi_only(T, tm, inv_delta) * inv_ste);
    }
  }
  const double s = block_sum_256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_kernel(const double *partial,
                                                  int64_t n, double *out) {
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) acc += partial[k];
  const double s = block_sum_256(acc);
  if (threadIdx.x == 0) *out = s;
}

// out: max_it, nonconv, max_res, flux_in, flux_out (as doubles)
__global__ __launch_bounds__(256) void stats_kernel(const StatSlot *slots,
                                                    int64_t n, double *out) {
  int it = 0;
  double nc = 0.0, res = 0.0, fin = 0.0, fout = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) {
    const StatSlot s = slots[k];
    it = max(it, s.max_it);
    nc += (double)s.nonconv;
    res = fmax(res, s.max_res);
    fin += s.flux_in;
    fout += s.flux_out;
  }
  __shared__ int s_it[4];
  __shared__ double s_res[4];
  it = wave_max_i(it);
  res = wave_max(res);
  if ((threadIdx.x & 63) == 0) {
    s_it[threadIdx.x >> 6] = it;
    s_res[threadIdx.x >> 6] = res;
  }
  const double snc = block_sum_256(nc);
  const double sfin = block_sum_256(fin);
  const double sfout = block_sum_256(fout);
  if (threadIdx.x == 0) {
    out[0] = (double)max(max(s_it[0], s_it[1]), max(s_it[2], s_it[3]));
    out[1] = snc;
    out[2] = fmax(fmax(s_res[0], s_res[1]), fmax(s_res[2], s_res[3]));
    out[3] = sfin;
    out[4] = sfout;
  }
}

// front of row blockIdx.x: dx * trapezoid sum of phi(T), of the sharp
// liquid fraction l(H) (eebm), or of the liquid fraction plane lf (ILFBM)
template <int Q, typename S>
__global__ __launch_bounds__(256) void front_integral_kernel(
    const S *src, int64_t plane, int nx, int eebm, double tm, double inv_delta,
    double ste, const double *lf, double dx, double *out) {
  const int64_t row = (int64_t)blockIdx.x * nx;
  double acc = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) {
    double T = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) T += (double)src[i * plane + row + x];
    const double ph = lf ? lf[row + x]
                         : (eebm ? eebm_lf(T, tm, ste)
                                 : phi_only(T, tm, inv_delta));
    acc += (x == 0 || x == nx - 1) ? 0.5 * ph : ph;
  }
  const double s = block_sum_256(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = dx * s;
}

// temperature of node k: M0 of the state, or Theta of it (eebm)
template <int Q, typename S>
__device__ __forceinline__ double temp_at(const S *src, int64_t plane,
                                          int64_t k, int eebm, double tm,
                                          double inv_ste) {
  double T = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) T += (double)src[i * plane + k];
  return eebm ? eebm_theta(T, tm, inv_ste) : T;
}

// first x (from x = 0) with T(x) - tm > 0 >= T(x+1) - tm, interpolated
template <int Q, typename S>
__global__ __launch_bounds__(256) void front_crossing_kernel(
    const S *src, int64_t plane, int nx, int eebm, double tm, double inv_ste,
    double dx, double *out) {
  const int64_t row = (int64_t)blockIdx.x * nx;
  auto rel = [&](int64_t k) {
    return temp_at<Q, S>(src, plane, k, eebm, tm, inv_ste) - tm;
  };
  const int chunk = (nx + 255) / 256;
  const int xa = threadIdx.x * chunk;
  int first = INT32_MAX;
  for (int x = xa; x < xa + chunk && x + 1 < nx; ++x) {
    const double t0 = rel(row + x);
    const double t1 = rel(row + x + 1);
    if (t0 > 0.0 && t1 <= 0.0) {
      first = x;
      break;
    }
  }
  __shared__ int s_min[4];
  int m = first;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = min(min(s_min[0], s_min[1]), min(s_min[2], s_min[3]));
    const double T0 = rel(row);
    double pos;
    if (T0 <= 0.0) {
      pos = 0.0;
    } else if (m == INT32_MAX) {
      pos = (nx - 1) * dx;
    } else {
      const double t0 = rel(row + m);
      const double t1 = rel(row + m + 1);
      pos = dx * (m + t0 / (t0 - t1));
    }
    out[blockIdx.x] = pos;
  }
}

}  // namespace
}  // namespace irebm
