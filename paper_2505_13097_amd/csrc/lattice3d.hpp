// lattice3d.hpp -- the IREBM step (Algorithm 3) and the explicit scheme
// (Algorithm 2) on the 3D lattices D3Q7 and D3Q19, for gfx950.
//
// Same state as the 2D kernels (the post-collision populations Omega_i,
// planes [q][nz][ny][nx], x fastest), the same per-node arithmetic
// (irebm_node.hpp: newton, phi, eebm_theta) and the same closures of
// Section 4.2, taken over the six faces in the order x-, x+, y-, y+, z-,
// z+ (the first Dirichlet face holding a node gives its temperature).
//
// Weights: the tau relation of Section 5 needs a second moment of T/3
// times the identity: D3Q19 1/3 (rest), 1/18 (faces), 1/36 (edges); D3Q7
// 1/6 per face and 0 at rest.  Velocity order: rest, +x, +y, +z, -x, -y,
// -z, then (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1), (0,1,-1) and
// their negatives in the same order (D3Q7 is the first seven).
//
// Tiling: a block of bx x by threads (waves along x) owns a column of
// (bx * npt) x by nodes of the xy plane and sweeps cz consecutive z slices
// of it: the slice its nodes pull from below was read by the same block in
// the iteration before, the slice above is read in the next one, so those
// reads come from the L2.  A work item is one such column chunk; items are
// ordered by bands of rows, each band through all its z chunks (kBand3Rows),
// and the blocks of XCD k take the k-th contiguous part of that order, so
// the columns beside a block share its L2.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "kernels.hpp"

namespace irebm {

// velocity component a (0: x, 1: y, 2: z) of direction i
__host__ __device__ constexpr int e3(int i, int a) {
  if (i == 0) return 0;
  if (i <= 6) return ((i - 1) % 3 == a) ? (i <= 3 ? 1 : -1) : 0;
  const int j = i <= 12 ? i - 7 : i - 13;  // edge pair: xy, xy, xz, xz, yz, yz
  const int s = i <= 12 ? 1 : -1;
  const int p = j / 2;
  const int first = p == 2 ? 1 : 0;
  const int second = p == 0 ? 1 : 2;
  const int sg = (j & 1) ? -1 : 1;
  return s * (a == first ? 1 : (a == second ? sg : 0));
}
__host__ __device__ constexpr int opp3(int i) {
  return i == 0 ? 0 : (i <= 6 ? (i <= 3 ? i + 3 : i - 3)
                              : (i <= 12 ? i + 6 : i - 6));
}
template <int Q>
__host__ __device__ constexpr double wt3(int i) {
  return Q == 7 ? (i == 0 ? 0.0 : 1.0 / 6.0)
                : (i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0));
}
// weight class: 0 rest, 1 face, 2 edge
__host__ __device__ constexpr int wclass3(int i) {
  return i == 0 ? 0 : (i <= 6 ? 1 : 2);
}

// Everything one step of one 3D lattice needs; passed by value.
struct StepArgs3 {
  const void *src;
  void *dst;
  int32_t nx, ny, nz, cz;  // node counts; z slices per work item
  int64_t plane;           // nx * ny * nz
  int32_t tiles_x, tiles_y, tiles_z;
  int32_t nitems, per_xcd;
  int32_t periodic[3];
  int32_t neu;             // bit k: face k (x-, x+, y-, y+, z-, z+) Neumann
  int32_t max_it;
  int32_t bc[6];
  double wall_T[6];
  double a, inv_tau;
  double wtau[3], wste[3]; // w/tau and w/Ste per weight class
  double inv_ste, tm, inv_delta, tol;
  StatSlot *slots;
  // split step (quiet and full passes, front strip): tiles start at column
  // x_off, columns from x_lim on are not updated; flags: one per work item
  int32_t x_off, x_lim;
  int32_t *flags;
  int32_t front_first;  // each XCD takes the x = 0 tiles of its chunk first
  // rows off the y and z faces take the in-register x-face closure
  // (close_xface3): both x faces Dirichlet or bounce-back, nx >= 3
  int32_t xrow;
  // item order: bands of `band` tile rows, each swept through all its
  // z chunks before the next band (0: z-chunk major over all rows)
  int32_t band;
};

template <int Q, typename S>
struct NodeLoad3 {
  S own[Q];
  S pull[Q];
  uint32_t known;  // bit i: pull source of direction i is a lattice node
  uint32_t out;    // bit i: destination x + e_i leaves the lattice
  double mirror;   // on a Neumann face: M0 of the pulls at the mirror node
};

// coordinates of the neighbours one cell below (m) and above (p) along each
// axis, wrapped on periodic axes and clamped elsewhere, with validity flags
struct Nbr3 {
  int m[3], p[3];
  bool vm[3], vp[3];
};

template <bool FAST>
__device__ __forceinline__ void neighbours3(const StepArgs3 &A, int x, int y,
                                            int z, Nbr3 &N) {
  const int c[3] = {x, y, z};
  const int n[3] = {A.nx, A.ny, A.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    N.m[a] = c[a] - 1;
    N.p[a] = c[a] + 1;
    N.vm[a] = N.vp[a] = true;
    if (!FAST) {
      if (N.m[a] < 0) {
        N.vm[a] = A.periodic[a] != 0;
        N.m[a] = N.vm[a] ? N.m[a] + n[a] : 0;
      }
      if (N.p[a] >= n[a]) {
        N.vp[a] = A.periodic[a] != 0;
        N.p[a] = N.vp[a] ? N.p[a] - n[a] : n[a] - 1;
      }
    }
  }
}

// mirror node of (x, y, z) across the Neumann faces it lies on (eq.
// Neu_on_q): one cell inward across each; false when on none
__device__ __forceinline__ bool neumann_mirror3(const StepArgs3 &A, int x,
                                                int y, int z, int m[3]) {
  const int c[3] = {x, y, z};
  const int n[3] = {A.nx, A.ny, A.nz};
  bool on = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m[a] = c[a];
    if ((A.neu >> (2 * a) & 1) && c[a] == 0) {
      m[a] = 1;
      on = true;
    }
    if ((A.neu >> (2 * a + 1) & 1) && c[a] == n[a] - 1) {
      m[a] = n[a] - 2;
      on = true;
    }
  }
  return on;
}

// M0 of the pulled populations at node m: sum_i Omega_i(m - e_i).  The host
// admits no bounce-back face beside a Neumann one, so every source is a
// lattice node (periodic axes wrap); indices are clamped all the same.
template <int Q, typename S>
__device__ __forceinline__ double mirror_m0_3(const StepArgs3 &A,
                                              const S *__restrict__ src,
                                              const int m[3]) {
  const int n[3] = {A.nx, A.ny, A.nz};
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = m[a] - e3(i, a);
      if (c[a] < 0) c[a] = A.periodic[a] ? c[a] + n[a] : 0;
      if (c[a] >= n[a]) c[a] = A.periodic[a] ? c[a] - n[a] : n[a] - 1;
    }
    s += (double)src[i * A.plane + ((int64_t)c[2] * A.ny + c[1]) * A.nx + c[0]];
  }
  return s;
}

// Loads of one node: own populations (for T) and the pulled ones.  FAST:
// every source and destination is a lattice node without wrapping.
// Otherwise the sources are wrapped or clamped so that every load is
// issued, and unknown directions are zeroed for the closure.
template <int Q, typename S, bool FAST, bool NEU>
__device__ __forceinline__ void load3(const StepArgs3 &A,
                                      const S *__restrict__ src, int x, int y,
                                      int z, NodeLoad3<Q, S> &L) {
  const int64_t P = A.plane;
  Nbr3 N;
  neighbours3<FAST>(A, x, y, z, N);
  // row pointers of the nine (y, z) source rows: wave-uniform when y and z
  // are, so each load is a scalar base plus a lane offset
  auto row = [&](int ey, int ez) {
    const int yy = ey == 1 ? N.m[1] : (ey == -1 ? N.p[1] : y);
    const int zz = ez == 1 ? N.m[2] : (ez == -1 ? N.p[2] : z);
    return src + ((int64_t)zz * A.ny + yy) * A.nx;
  };
  const S *r0 = row(0, 0);
#pragma unroll
  for (int j = 0; j < Q; ++j) L.own[j] = (r0 + j * P)[(uint32_t)x];
  L.pull[0] = L.own[0];
  L.known = 1u;
  L.out = 0u;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int ex = e3(i, 0), ey = e3(i, 1), ez = e3(i, 2);
    const int sx = ex == 1 ? N.m[0] : (ex == -1 ? N.p[0] : x);
    L.pull[i] = (row(ey, ez) + i * P)[(uint32_t)sx];
    if (!FAST) {
      bool ok = true, leaves = false;
      const int e[3] = {ex, ey, ez};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ok = ok && (e[a] == 1 ? N.vm[a] : (e[a] == -1 ? N.vp[a] : true));
        leaves = leaves || (e[a] == 1 ? !N.vp[a] : (e[a] == -1 ? !N.vm[a] : false));
      }
      if (ok) L.known |= 1u << i;
      else L.pull[i] = (S)0;
      if (leaves) L.out |= 1u << i;
    } else {
      L.known |= 1u << i;
    }
  }
  L.mirror = 0.0;
  if (!FAST && NEU) {
    int m[3];
    if (neumann_mirror3(A, x, y, z, m)) L.mirror = mirror_m0_3<Q, S>(A, src, m);
  }
}

// Loads of a node of a row off the y and z faces (the xrow path): as
// load3<FAST>, with the x sources clamped into the row so that an x-face
// node's unknown directions read a lattice node (their values are replaced
// by close_xface3).  OWN false (EEBM, whose update reads the own
// populations only for the face fluxes): own populations past the rest one
// loaded on face nodes only.
template <int Q, typename S, bool OWN>
__device__ __forceinline__ void load_row3(const StepArgs3 &A,
                                          const S *__restrict__ src, int x,
                                          int y, int z, bool face,
                                          NodeLoad3<Q, S> &L) {
  const int64_t P = A.plane;
  auto row = [&](int ey, int ez) {
    return src + ((int64_t)(z - ez) * A.ny + (y - ey)) * A.nx;
  };
  const S *r0 = row(0, 0);
  L.own[0] = r0[(uint32_t)x];
#pragma unroll
  for (int j = 1; j < Q; ++j)
    L.own[j] = (OWN || face) ? (r0 + j * P)[(uint32_t)x] : (S)0;
  L.pull[0] = L.own[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int ex = e3(i, 0), ey = e3(i, 1), ez = e3(i, 2);
    const int sx = ex == 0 ? x : min(max(x - ex, 0), A.nx - 1);
    L.pull[i] = (row(ey, ez) + i * P)[(uint32_t)sx];
  }
  L.known = (1u << Q) - 1u;
  L.out = 0u;
  L.mirror = 0.0;
}

// does the source of unknown direction i of node (x, y, z) lie beyond
// bounce-back faces only?  (a periodic axis wraps and is never left)
__device__ __forceinline__ bool leaves_by_bounceback3(const StepArgs3 &A,
                                                      int x, int y, int z,
                                                      int i) {
  const int c[3] = {x, y, z};
  const int n[3] = {A.nx, A.ny, A.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int s = c[a] - e3(i, a);
    if (A.periodic[a]) continue;
    if (s < 0 && A.bc[2 * a] != BC_BOUNCEBACK) return false;
    if (s >= n[a] && A.bc[2 * a + 1] != BC_BOUNCEBACK) return false;
  }
  return true;
}

// the first Dirichlet face (x-, x+, y-, y+, z-, z+) holding the node, or -1
__device__ __forceinline__ int dirichlet_face3(const StepArgs3 &A, int x,
                                               int y, int z) {
  const int c[3] = {x, y, z};
  const int n[3] = {A.nx, A.ny, A.nz};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int a = k >> 1;
    if (A.bc[k] == BC_DIRICHLET && c[a] == ((k & 1) ? n[a] - 1 : 0)) return k;
  }
  return -1;
}

// The zeroth moment a Dirichlet closure gives a node at wall temperature
// TD: IREBM eq. Dir_on_q (TD plus the latent term's jump between the wall
// and the node's temperature th), EEBM the wall enthalpy.  PLATEAU (the
// quiet pass): phi only where it is exactly 0 or 1, *near set when the
// wall or the node lies nearer the band (see close_node)
template <bool EEBM, bool PLATEAU>
__device__ __forceinline__ double dirichlet_deficit3(const StepArgs3 &A,
                                                     double TD, double th,
                                                     int *near) {
  if constexpr (PLATEAU && !EEBM) {
    const double ud = (TD - A.tm) * A.inv_delta;
    const double ut = (th - A.tm) * A.inv_delta;
    if (!(fabs(ud) > 20.0 && fabs(ut) > 20.0)) *near = 1;
    return TD + ((ud > 20.0 ? 1.0 : 0.0) - (ut > 20.0 ? 1.0 : 0.0)) *
                    A.inv_ste;
  } else {
    return EEBM ? TD + (TD > A.tm ? A.inv_ste : 0.0)
                : TD + (phi_only(TD, A.tm, A.inv_delta) -
                        phi_only(th, A.tm, A.inv_delta)) * A.inv_ste;
  }
}

// Closure of the unknown pulled populations (Section 4.2), as close_node:
// bounce-back from a known opposite; Dirichlet deficit (IREBM eq.
// Dir_on_q, EEBM the wall enthalpy) shared by weight; Neumann deficit to
// M0 of the mirror's pulls (eq. Neu_on_q) shared by weight; own
// Omega_opp for anything left.  Returns the sum of the closed values.
// PLATEAU (the quiet pass): phi only where it is exactly 0 or 1, *near set
// when the wall or the node lies nearer the band (see close_node)
template <int Q, bool EEBM, bool NEU, bool PLATEAU = false, typename S>
__device__ __forceinline__ double close3(const StepArgs3 &A, int x, int y,
                                         int z, double th, const S *om,
                                         double *q, uint32_t known,
                                         double mirror, int *near = nullptr) {
  // the bounce-back set first, then its values: compiled from the
  // in-place form (test, copy and mark in one loop), the D3Q7 step kernel
  // lost the copies on gfx950 while keeping the marks (the same source was
  // right on the host and in a kernel without the z loop)
  uint32_t bb = 0u;
  double fill = 0.0;
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (!(known >> i & 1u) && (known >> opp3(i) & 1u) &&
        leaves_by_bounceback3(A, x, y, z, i))
      bb |= 1u << i;
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (bb >> i & 1u) {
      q[i] = q[opp3(i)];
      fill += q[i];
    }
  uint32_t set = known | bb;
  const int face = dirichlet_face3(A, x, y, z);
  bool share = false;
  double D = 0.0;
  if (face >= 0) {
    D = dirichlet_deficit3<EEBM, PLATEAU>(A, A.wall_T[face], th, near);
    share = true;
  } else if (NEU) {
    int m[3];
    if (neumann_mirror3(A, x, y, z, m)) {
      D = mirror;
      share = true;
    }
  }
  if (share) {
    double wu = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (set >> i & 1u) D -= q[i];
      else wu += wt3<Q>(i);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (!(set >> i & 1u)) {
        q[i] = D * (wt3<Q>(i) / wu);
        fill += q[i];
      }
    set = (1u << Q) - 1u;
  }
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (!(set >> i & 1u)) {
      q[i] = (double)om[opp3(i)];
      fill += q[i];
    }
  return fill;
}

// close3 for a node on an x face (side 0: x = 0, whose unknown directions
// have e_x = +1; side 1: x = nx - 1, e_x = -1) of a row off the y and z
// faces, the x faces being Dirichlet or bounce-back (xrow): there close3
// copies every unknown direction from its known opposite (bounce-back) or
// shares the Dirichlet deficit by weight, and this does the same
// operations in the same order, from the direction masks of the face.
template <int Q, bool EEBM, bool PLATEAU>
__device__ __forceinline__ double close_xface3(const StepArgs3 &A, int side,
                                               double th, double *q,
                                               int *near) {
  const int eu = side == 0 ? 1 : -1;
  double fill = 0.0;
  if (A.bc[side] == BC_BOUNCEBACK) {
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if (e3(i, 0) == eu) {
        q[i] = q[opp3(i)];
        fill += q[i];
      }
    return fill;
  }
  double D = dirichlet_deficit3<EEBM, PLATEAU>(A, A.wall_T[side], th, near);
  double wu = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (e3(i, 0) != eu) D -= q[i];
    else wu += wt3<Q>(i);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    if (e3(i, 0) == eu) {
      q[i] = D * (wt3<Q>(i) / wu);
      fill += q[i];
    }
  return fill;
}

// The update of one node from its loads into v (storage type): the same
// arithmetic as update_values (irebm_node.hpp) on the 3D lattice.  QUIET:
// the quiet pass's form (no Newton code): a node that is not quiet is
// counted in st.solves and v is left meaningless.
template <int Q, typename S, int MODE, bool FAST, bool QUIET = false,
          bool XROW = false>
__device__ __forceinline__ void update3(const StepArgs3 &A, int x, int y,
                                        int z, const NodeLoad3<Q, S> &L,
                                        NodeStats &st, S v[Q],
                                        int side = -1) {
  constexpr bool PLAIN = base_mode(MODE) == kPlain;
  constexpr bool EEBM = base_mode(MODE) == kEebm;
  constexpr bool NEU = neumann_mode(MODE);
  // own populations stay in storage precision until used (fewer
  // registers than an FP64 copy held across the closure)
  double q[Q];
  double th = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) th += (double)L.own[j];
#pragma unroll
  for (int i = 0; i < Q; ++i) q[i] = (double)L.pull[i];
  int near = 0;
  if (!FAST) {
    if (L.known != (1u << Q) - 1u)
      st.flux_in += close3<Q, EEBM, NEU, QUIET>(A, x, y, z, th, L.own, q,
                                                L.known, L.mirror, &near);
    if (L.out) {
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (L.out >> i & 1u) st.flux_out += (double)L.own[i];
    }
  }
  if constexpr (XROW) {
    // an x-face node of an interior row (side >= 0): its closure, and the
    // populations leaving through the face
    if (side >= 0) {
      st.flux_in += close_xface3<Q, EEBM, QUIET>(A, side, th, q, &near);
      const int eo = side == 0 ? -1 : 1;
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (e3(i, 0) == eo) st.flux_out += (double)L.own[i];
    }
  }
  double m0 = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) m0 += q[i];
  if constexpr (EEBM) {
    // Algorithm 2: H = m0, explicit temperature, BGK collision
    const double tq = eebm_theta(m0, A.tm, A.inv_ste);
    v[0] = (S)(A.a * q[0] + A.inv_tau * (m0 - (1.0 - wt3<Q>(0)) * tq));
#pragma unroll
    for (int i = 1; i < Q; ++i)
      v[i] = (S)(A.a * q[i] + A.wtau[wclass3(i)] * tq);
    return;
  }
  // quiet node (see update_values): far below the melting band before and
  // after, the Newton solve in closed form, f~ = q
  {
    const double u = (th - A.tm) * A.inv_delta;
    const double um = (m0 - A.tm) * A.inv_delta;
    const double d = th - m0;
    const double dx0 = m0 - (m0 - A.inv_ste);
    if (u < -20.0 && um < -20.0 && th - d == m0 && !near &&
        (PLAIN || 2.0 * fabs(d) <= fabs(dx0))) {
      const bool one = fabs(d) <= A.tol;
      const int it = (one || A.max_it < 2) ? 1 : 2;
      st.max_it = it > st.max_it ? it : st.max_it;
      st.nonconv += (one || A.max_it >= 2) ? 0 : 1;
#pragma unroll
      for (int i = 0; i < Q; ++i)
        v[i] = (S)(A.a * q[i] + A.wtau[wclass3(i)] * m0);
      return;
    }
  }
  ++st.solves;
  if constexpr (QUIET) {
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = (S)q[i];
    return;
  }
  double pth, dpth;
  phi_dphi(th, A.tm, A.inv_delta, pth, dpth);
  int it;
  bool conv;
  PhiAt at;
  const double tn = newton<PLAIN>(m0, th, pth, dpth, A, it, conv, at);
  const double pnew = at.ok ? at.ph : phi_only(tn, A.tm, A.inv_delta);
  const double dphi_s = pth - pnew;
  double f[Q];
  double tsum = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    f[i] = q[i] + A.wste[wclass3(i)] * dphi_s;
    tsum += f[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    v[i] = (S)(A.a * f[i] + A.wtau[wclass3(i)] * tsum);
  const double res = fabs(tn + pnew * A.inv_ste - (m0 + pth * A.inv_ste));
  st.max_it = it > st.max_it ? it : st.max_it;
  st.nonconv += conv ? 0 : 1;
  st.max_res = res > st.max_res ? res : st.max_res;
}

template <int Q, typename S, int MODE, bool FAST, bool NT, bool QUIET = false,
          bool XROW = false>
__device__ __forceinline__ void update_store3(const StepArgs3 &A,
                                              S *__restrict__ dst, int x,
                                              int y, int z,
                                              const NodeLoad3<Q, S> &L,
                                              NodeStats &st, int side = -1) {
  S v[Q];
  update3<Q, S, MODE, FAST, QUIET, XROW>(A, x, y, z, L, st, v, side);
  S *row = dst + ((int64_t)z * A.ny + y) * A.nx;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    S *p = (row + i * A.plane) + (uint32_t)x;
    if (NT) __builtin_nontemporal_store(v[i], p);
    else *p = v[i];
  }
}

// waves per SIMD the 3D step asks of the compiler: the occupancy its
// register count gives without the interior-row path, which would
// otherwise cost D3Q19 a wave
constexpr int step3_waves(int q, int bytes, int npt) {
  return q == 19 ? (bytes == 4 || npt == 1 ? 3 : 2) : (npt == 1 ? 5 : 4);
}

namespace {

// One step of a 3D lattice: one block per work item (a column chunk of
// cz slices), items in bands of rows (set_tiling3), XCD-contiguous item
// order; interior slices of interior
// columns take the path with no bounds checks, and so do the rows off the
// y and z faces of the other columns when both x faces are Dirichlet or
// bounce-back (xrow), an x-face node closed in registers; the rest take
// the bounds-checked path, a node at a time.  Per-item statistics slots
// as in step_kernel.
//
// Split step (variants ".../s", IREBM, a lattice heated through the x = 0
// face): the Newton solve is rare (the front lies in the first cells of
// every x row) but its code sets the register count of every wave and its
// iterations hold whole 64-lane waves.  So the step is split by columns:
// the front strip [0, A.x_lim) by this kernel as it stands (SPLIT 0) on a
// stream of its own, and the rest (tiles from column A.x_off) by SPLIT 1,
// built for quiet nodes only (no Newton code), beside it; an item of the
// quiet pass with a node (in or near the band) that is not quiet adds no
// statistics and sets its flag to 2, and SPLIT 2, after both, redoes the
// flagged items with the full update and clears the flag of an item with
// no solve left (the quiet pass skips items flagged 2).  Same per-node
// arithmetic either way.
template <int Q, typename S, int NPT, int MODE, bool NT, int SPLIT = 0>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(step3_waves(Q, sizeof(S), NPT))))
void step3_kernel(StepArgs3 A) {
  const int b = (int)blockIdx.x;
  if ((b & 7) * A.per_xcd + (b >> 3) >= A.nitems) return;
  const int t = A.front_first
                    ? xcd_item_front_first(b, A.per_xcd, A.nitems, A.tiles_x)
                    : xcd_item(b, A.per_xcd, A.nitems, 0);
  if (SPLIT > 0 &&
      __builtin_amdgcn_readfirstlane(A.flags[t]) != (SPLIT == 1 ? 0 : 2))
    return;
  const int tx = t % A.tiles_x;
  const int r = t / A.tiles_x;
  int ty, tz;
  if (A.band > 0) {
    const int per = A.band * A.tiles_z;
    const int bi = r / per, rr = r - bi * per;
    const int bw = min(A.band, A.tiles_y - bi * A.band);
    ty = bi * A.band + rr % bw;
    tz = rr / bw;
  } else {
    ty = r % A.tiles_y;
    tz = r / A.tiles_y;
  }
  const int bx = (int)blockDim.x, by = (int)blockDim.y;
  const int TW = bx * NPT;
  const int x0 = A.x_off + tx * TW, y0 = ty * by;
  const int z0 = tz * A.cz, z1 = min(z0 + A.cz, A.nz);
  const bool fxy = x0 >= 1 && x0 + TW <= A.nx - 1 && x0 + TW <= A.x_lim &&
                   y0 >= 1 && y0 + by <= A.ny - 1;
  // a wave lies in one row of the column (bx is a multiple of 64)
  const int y = y0 + __builtin_amdgcn_readfirstlane((int)threadIdx.y);
  const S *src = (const S *)A.src;
  S *dst = (S *)A.dst;
  NodeStats st;
  bool fast_all = true;
  for (int z = z0; z < z1; ++z) {
    // re-read the uniform arguments each pass (see step_item)
    int k0 = 0;
    asm volatile("" : "+s"(k0));
    const StepArgs3 &B = (&A)[k0];
    const bool fast = fxy && z >= 1 && z <= B.nz - 2;
    fast_all = fast_all && fast;
    if (fast) {
      NodeLoad3<Q, S> L[NPT];
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        load3<Q, S, true, false>(B, src, x0 + (int)threadIdx.x + k * bx, y, z,
                                 L[k]);
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        update_store3<Q, S, MODE, true, NT, SPLIT == 1>(
            B, dst, x0 + (int)threadIdx.x + k * bx, y, z, L[k], st);
    } else if (B.xrow && z >= 1 && z <= B.nz - 2 && y >= 1 &&
               y <= B.ny - 2) {
      // a row off the y and z faces in a tile holding an x face or a
      // ragged end: both nodes' loads in flight as above, an x-face node
      // closed in registers (close_xface3), lanes past the row idle
      constexpr bool OWN = base_mode(MODE) != kEebm;
      NodeLoad3<Q, S> L[NPT];
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int x = x0 + (int)threadIdx.x + k * bx;
        load_row3<Q, S, OWN>(B, src, min(x, B.nx - 1), y, z,
                             x == 0 || x == B.nx - 1, L[k]);
      }
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int x = x0 + (int)threadIdx.x + k * bx;
        if (x < B.nx && x < B.x_lim)
          update_store3<Q, S, MODE, true, NT, SPLIT == 1, true>(
              B, dst, x, y, z, L[k], st,
              x == 0 ? 0 : (x == B.nx - 1 ? 1 : -1));
      }
    } else {
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int x = x0 + (int)threadIdx.x + k * bx;
        if (x < B.x_lim && y < B.ny) {
          NodeLoad3<Q, S> L;
          load3<Q, S, false, neumann_mode(MODE)>(B, src, x, y, z, L);
          update_store3<Q, S, MODE, false, NT, SPLIT == 1>(B, dst, x, y, z,
                                                          L, st);
        }
      }
    }
  }
  bool any = false;
  if constexpr (SPLIT > 0) any = __syncthreads_or(st.solves > 0) != 0;
  if (SPLIT != 1 || !any) {
    StatSlot pre{};
    if (threadIdx.x == 0 && threadIdx.y == 0) pre = A.slots[t];
    block_stats_to_slot<false>(st, fast_all, pre, A.slots + t);
  }
  if (SPLIT > 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    if (SPLIT == 1 && any) A.flags[t] = 2;
    if (SPLIT == 2 && !any) A.flags[t] = 0;
  }
}

// equilibrium initial state (as init_kernel): IREBM Omega_i = w_i T, EEBM
// the equilibrium of H = T + l(T)/Ste; Dirichlet nodes at their face's
// temperature
template <int Q, typename S>
__global__ void init3_kernel(StepArgs3 A, int eebm, const double *T0) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.plane) return;
  const int x = (int)(k % A.nx);
  const int64_t r = k / A.nx;
  const int y = (int)(r % A.ny), z = (int)(r / A.ny);
  const int face = dirichlet_face3(A, x, y, z);
  const double T = face >= 0 ? A.wall_T[face] : (T0 ? T0[k] : 0.0);
  S *dst = (S *)A.dst;
  if (eebm) {
    const double H = T + (T > A.tm ? A.inv_ste : 0.0);
    const double th = eebm_theta(H, A.tm, A.inv_ste);
    dst[k] = (S)(H - (1.0 - wt3<Q>(0)) * th);
#pragma unroll
    for (int i = 1; i < Q; ++i) dst[i * A.plane + k] = (S)(wt3<Q>(i) * th);
    return;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[i * A.plane + k] = (S)(wt3<Q>(i) * T);
}

}  // namespace
}  // namespace irebm

namespace irebm {

// ---------------------------------------------------------------------
// host side: kernel variants of the 3D step

// A 3D variant: blocks of bx x by threads (bx a multiple of 64, at most
// 256 threads: the kernel's launch bound), npt nodes per thread bx apart
// along x, cz z slices per work item; nt: non-temporal stores.
// split: the split step (see step3_kernel) on lattices heated through the
// x = 0 face, IREBM; the plain kernel otherwise
struct Variant3 {
  int bx, by, npt, cz, nt, split;
};

inline const Variant3 *variants3(int *n) {
  static const Variant3 v[] = {
      {64, 4, 1, 8, 1},  {64, 4, 1, 8, 0},  {64, 4, 1, 32, 1},
      {64, 4, 1, 1, 1},  {128, 2, 1, 16, 1}, {256, 1, 1, 16, 1},
      {64, 2, 2, 16, 1}, {64, 4, 2, 8, 1},  {128, 1, 2, 16, 1},
      {64, 2, 1, 8, 1},  {128, 1, 2, 4, 1},  {128, 1, 2, 8, 1},
      {128, 1, 2, 32, 1}, {128, 1, 2, 16, 0}, {64, 1, 2, 16, 1},
      {64, 2, 2, 8, 1},
      {128, 1, 2, 4, 1, 1}, {128, 1, 2, 8, 1, 1}, {64, 4, 1, 8, 1, 1},
      {64, 2, 2, 8, 1, 1},  {64, 4, 1, 16, 1, 1}};
  *n = (int)(sizeof(v) / sizeof(Variant3));
  return v;
}
constexpr int kDefaultVariant3D = 0;
// split step: the front strip is the first kFront3Columns columns, run
// with the tiling of variant kFront3Variant (64 x 4, 32 slices per item:
// fewer, longer front blocks beside the quiet pass; on the 512^3 D3Q7
// cube 8 slices per item gave 1652 us per step, 16 gave 1638, 32 and 64
// 1577, 128 1593)
constexpr int kFront3Columns = 64;
constexpr int kFront3Variant = 2;
// item order: bands of about kBand3Rows lattice rows, each swept through
// its z chunks in turn, so that an XCD's blocks in flight share y
// neighbours and the slices at the chunk boundaries are still in its L2
// when the next chunk pulls them (512^3 D3Q19 cube: 4407 us per step
// z-chunk major, 4229 with bands of 128 rows, 4241-4257 with 96-256)
constexpr int kBand3Rows = 128;

inline int64_t tiles3_x(const Variant3 &v, int64_t nx) {
  return (nx + (int64_t)v.bx * v.npt - 1) / ((int64_t)v.bx * v.npt);
}
inline int64_t tiles3_y(const Variant3 &v, int64_t ny) {
  return (ny + v.by - 1) / v.by;
}
inline int64_t tiles3_z(const Variant3 &v, int64_t nz) {
  return (nz + v.cz - 1) / v.cz;
}
inline int64_t items3_for(const Variant3 &v, int64_t nx, int64_t ny,
                          int64_t nz) {
  return tiles3_x(v, nx) * tiles3_y(v, ny) * tiles3_z(v, nz);
}
// tiles over the columns [x_off, x_lim) (the whole row unless split)
inline void set_tiling3(StepArgs3 *A, const Variant3 &v) {
  const int64_t w = (int64_t)A->x_lim - A->x_off;
  A->cz = v.cz;
  A->tiles_x = (int32_t)tiles3_x(v, w);
  A->tiles_y = (int32_t)tiles3_y(v, A->ny);
  A->tiles_z = (int32_t)tiles3_z(v, A->nz);
  A->nitems = (int32_t)items3_for(v, w, A->ny, A->nz);
  A->per_xcd = (A->nitems + 7) / 8;
  A->band = std::max(1, kBand3Rows / v.by);
}

// one step of a 3D lattice for one node-update mode (instantiated by the
// k_step3_<mode>.hip units)
template <int MODE>
hipError_t step3_launch_mode(int q, int storage, const StepArgs3 &A,
                             const Variant3 &v, int split,
                             hipStream_t stream);

}  // namespace irebm
