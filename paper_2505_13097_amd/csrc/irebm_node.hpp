// irebm_node.hpp -- device-side pieces of the IREBM step for gfx950:
// lattice constants, the regularized liquid fraction, the local Newton
// solve and the per-node update on the post-collision state.
//
// Method: Luddens, Lothode, Danaila, arXiv 2505.13097, Algorithm 3
// (Section 4.1) with the boundary closures of Section 4.2.
//
// State: Omega_i(x) = (1 - 1/tau) f_i(x) + (w_i/tau) T(x) (eq.
// def_qi_omegai), stored as q planes.  One step for node x reads
//   T(x)   = sum_j Omega_j(x)            (collision conserves M0),
//   q_i(x) = Omega_i(x - e_i)            (pull streaming),
// solves the local equation for the new temperature T~, forms
//   f~_i = q_i + (w_i/Ste)(phi(T) - phi(T~))   (source and update),
// and writes the next state Omega'_i = (1 - 1/tau) f~_i + (w_i/tau) M0(f~).
// Storing Omega instead of f makes the pull read one direction per
// neighbour, so a step moves the minimum 2 q s bytes per node.
//
// The same kernels run the explicit enthalpy based method (EEBM, Section
// 3.4, Algorithm 2) on the same post-collision state: the pulled q_i are
// the streamed f~_i, H = M0(f~) is the enthalpy, theta = Theta(H) its
// temperature, and the next state is the BGK collision
//   Omega'_i = (1 - 1/tau) f~_i + f_i^eq / tau,
//   f_i^eq = w_i theta (i != 0),  f_0^eq = H - (1 - w_0) theta.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace irebm {

// ---- lattices (Section 3.2): rest, +x, +y, -x, -y, (1,1), (-1,1),
// (-1,-1), (1,-1); D1Q3 is rest, +x, -x.
template <int Q>
__host__ __device__ constexpr int cx(int i) {
  return Q == 3 ? (i == 1 ? 1 : (i == 2 ? -1 : 0))
                : ((i == 1 || i == 5 || i == 8) ? 1
                   : (i == 3 || i == 6 || i == 7) ? -1 : 0);
}
template <int Q>
__host__ __device__ constexpr int cy(int i) {
  return Q == 3 ? 0
                : ((i == 2 || i == 5 || i == 6) ? 1
                   : (i == 4 || i == 7 || i == 8) ? -1 : 0);
}
template <int Q>
__host__ __device__ constexpr double wt(int i) {
  return Q == 3 ? (i == 0 ? 2.0 / 3.0 : 1.0 / 6.0)
       : Q == 5 ? (i == 0 ? 1.0 / 3.0 : 1.0 / 6.0)
                : (i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0));
}
// the first direction with the weight of direction i: equal weights give
// equal w_i/tau and w_i/Ste, so kernels read one value per weight class
template <int Q>
__host__ __device__ constexpr int wclass(int i) {
  return i == 0 ? 0 : (Q == 9 && i >= 5 ? 5 : 1);
}
template <int Q>
__host__ __device__ constexpr int opp(int i) {
  return Q == 3 ? (i == 0 ? 0 : 3 - i)
       : i == 0 ? 0
       : i < 5  ? (i + 1) % 4 + 1
                : (i - 3) % 4 + 5;
}

enum { BC_DIRICHLET = 0, BC_BOUNCEBACK = 1, BC_PERIODIC = 2, BC_NEUMANN = 3 };

// Pointers into global memory (address space 1).  The node loads and
// stores take them, so that a pointer the kernel reads from memory (a
// batch descriptor) still gives global loads and stores with a scalar base
// and a 32-bit lane offset; through a generic pointer every access would
// be a flat instruction with a 64-bit address computed per lane.  Every
// state buffer the library hands its kernels lies in global memory.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p) {
  return (gptr<T>)p;
}

// node update of a kernel instance: IREBM with the safeguarded or the
// printed Newton update (Algorithm 3), or the explicit scheme (Algorithm 2);
// kNeumann added to a mode compiles the Neumann closure (one-step kernels
// of lattices with a Neumann wall; every other kernel is built without it)
enum Mode : int { kSafeguarded = 0, kPlain = 1, kEebm = 2, kNeumann = 4 };
constexpr int base_mode(int m) { return m & 3; }
constexpr bool neumann_mode(int m) { return (m & kNeumann) != 0; }
enum { SCHEME_IREBM = 0, SCHEME_EEBM = 1, SCHEME_ILFBM = 2 };

// Per-tile statistics slot, accumulated across steps by the one block
// that owns the tile (no atomics; deterministic).
struct StatSlot {
  int32_t max_it;
  int32_t nonconv;
  double max_res;
  double flux_in;
  double flux_out;
};

// Everything one step of one lattice needs; passed by value.
struct StepArgs {
  const void *src;      // current state planes
  void *dst;            // next state planes
  int32_t nx, ny;
  int32_t x_lim, x_cnt; // kernels built with LIM (the batched two-step
                        // front pass): columns x < x_lim are computed, and
                        // those with x < x_cnt counted in the statistics
  int64_t plane;        // nx * ny
  int32_t tiles_x, tiles_y;  // tile grid
  int32_t group;             // tile rows per work item (one block each)
  int32_t nitems, per_xcd;   // work items; items per XCD chunk
  int32_t reverse;      // sweep the tiles in reverse order
  int32_t front_first;  // each XCD takes the x = 0 tiles of its chunk first
  int32_t periodic_x, periodic_y;
  int32_t scheme;       // SCHEME_IREBM or SCHEME_EEBM
  int32_t neu;          // bit k: wall k (x-, x+, y-, y+) is a Neumann wall
  int32_t x_shift;      // two-step kernels: strip s covers the columns from
                        // s (bx - 4) - x_shift on (a narrow first strip)
  double a;             // 1 - 1/tau
  double inv_tau;       // 1/tau
  double wtau[9];       // w_i / tau
  double wste[9];       // w_i / Ste
  double inv_ste, tm, inv_delta, tol;
  int32_t max_it;
  int32_t bc[4];
  double wall_T[4];
  const double *prof[4];
  StatSlot *slots;
};

// ---- regularized liquid fraction (Section 4.1)
// phi(T) = (1 + tanh(u))/2 = 1/(1 + exp(-2u)), u = (T - T_m)/delta, and
// phi'(T) = (1 - tanh^2 u)/(2 delta) = 2 e/(1 + e)^2 / delta with
// e = exp(-2u).  Past |u| > 20, tanh(u) rounds to +-1 in double, so
// phi is exactly 0 or 1 there and phi' is 0.
__device__ __forceinline__ void phi_dphi(double t, double tm, double inv_delta,
                                double &ph, double &dph) {
  const double u = (t - tm) * inv_delta;
  if (u > 20.0) {
    ph = 1.0;
    dph = 0.0;
  } else if (u < -20.0) {
    ph = 0.0;
    dph = 0.0;
  } else {
    const double e = exp(-2.0 * u);
    const double r = 1.0 / (1.0 + e);
    ph = r;
    dph = 2.0 * inv_delta * e * r * r;
  }
}

__device__ __forceinline__ double phi_only(double t, double tm, double inv_delta) {
  const double u = (t - tm) * inv_delta;
  if (u > 20.0) return 1.0;
  if (u < -20.0) return 0.0;
  return 1.0 / (1.0 + exp(-2.0 * u));
}

// ---- temperature of an enthalpy in the explicit scheme (Section 3.4):
// H below T_m, T_m on the band [T_m, T_m + 1/Ste], H - 1/Ste above it
__host__ __device__ __forceinline__ double eebm_theta(double H, double tm,
                                                      double inv_ste) {
  return H < tm ? H : (H <= tm + inv_ste ? tm : H - inv_ste);
}
// its sharp liquid fraction l(H) = clamp(Ste (H - T_m), 0, 1)
__host__ __device__ __forceinline__ double eebm_lf(double H, double tm,
                                                   double ste) {
  const double l = ste * (H - tm);
  return l < 0.0 ? 0.0 : (l > 1.0 ? 1.0 : l);
}

// phi and phi' at the value a Newton solve returns, when the solve
// already evaluated them there (ok); the caller then needs no evaluation
struct PhiAt {
  double ph = 0.0, dph = 0.0;
  bool ok = false;
};

// ---- local Newton solve of eq. rhs_fl_2:
//   F(t) = t + phi(t)/Ste - c = 0,  c = m0 + phi(T)/Ste,
// started from t = T (Algorithm 3); pth and dpth are phi(T) and phi'(T),
// which the caller has (they are the first iterate's values).  PLAIN takes
// the printed update.
// The safeguarded form keeps the same step inside the rtsafe rule
// (Press et al., Numerical Recipes, sec. 9.4): bracket [c - 1/Ste, c]
// (F' >= 1 and 0 <= phi <= 1 make it valid), bisect when the step leaves
// the bracket or fails to halve the step before the last.  Stops when
// |t_{k+1} - t_k| <= tol, then takes one more Newton step (below).
// AR: any argument block with inv_ste, tm, inv_delta, tol and max_it.
template <bool PLAIN, class AR>
__device__ __forceinline__ double newton(double m0, double th, double pth,
                                         double dpth, const AR &A, int &iters,
                                         bool &conv, PhiAt &at) {
  const double s = A.inv_ste;
  const double c = m0 + pth * s;
  double lo = c - s, hi = c;
  double dx = hi - lo, dxold = dx;
  // Solid node far from the melting band (phi(T) = 0 and phi(m0) = 0
  // exactly, phi' = 0): then c = m0, the first iterate is T - (T - m0),
  // and when that equals m0 (the difference is exact) the second iterate
  // and the final step change nothing.  Evaluate those iterations in closed
  // form: same result (up to the sign of a zero, which only enters phi),
  // same iteration count and convergence flag.  The guard also checks
  // that the safeguard's step test would have kept the first step.
  if (pth == 0.0 && (m0 - A.tm) * A.inv_delta < -20.0) {
    const double d = th - m0;
    if (th - d == m0 && (PLAIN || 2.0 * fabs(d) <= fabs(dx))) {
      const bool one = fabs(d) <= A.tol;
      conv = one || A.max_it >= 2;
      iters = (one || A.max_it < 2) ? 1 : 2;
      at.ph = at.dph = 0.0;  // m0 lies below the band too
      at.ok = true;
      return m0;
    }
  }
  double cur = th, cand = th;
  // phi and phi' at the current iterate: evaluated once per iterate, at
  // the end of the iteration that produced it, so the final step below
  // reuses the converged iterate's values
  double ph = pth, dph = dpth;
  int k = 0;
  conv = false;
  while (k < A.max_it) {
    if (PLAIN) {
      cand = (m0 + pth * s + dph * cur * s - ph * s) / (1.0 + dph * s);
    } else {
      const double F = cur + ph * s - c;
      if (F < 0.0) lo = cur;
      else if (F > 0.0) hi = cur;
      const double stp = (dph == 0.0) ? F : F / (1.0 + dph * s);
      cand = cur - stp;
      if (cand < lo || cand > hi || 2.0 * fabs(stp) > fabs(dxold)) {
        cand = 0.5 * (lo + hi);
        dxold = dx;
        dx = 0.5 * (hi - lo);
      } else {
        dxold = dx;
        dx = stp;
      }
    }
    ++k;
    phi_dphi(cand, A.tm, A.inv_delta, ph, dph);
    if (fabs(cand - cur) <= A.tol) {
      conv = true;
      break;
    }
    cur = cand;
  }
  iters = k;
  // one more Newton step from the converged iterate: a solve that stopped
  // on a bisection step is then the root to rounding, not any point within
  // tol of it, so the result does not depend on the safeguard's path.
  // ph, dph belong to cand; they still do when the step changes nothing
  // (or when the solve stopped at the cap)
  at.ph = ph;
  at.dph = dph;
  at.ok = true;
  if (conv) {
    const double F = cand + ph * s - c;
    const double next = cand - ((dph == 0.0) ? F : F / (1.0 + dph * s));
    at.ok = next == cand;
    cand = next;
  }
  return cand;
}

struct NodeStats {
  int max_it = 0;
  int nonconv = 0;
  double max_res = 0.0;
  double flux_in = 0.0;
  double flux_out = 0.0;
  int solves = 0;  // node updates that took the Newton path (not quiet)
};

// Raw loads of one node: own populations (for T) and pulled ones.
template <int Q, typename S>
struct NodeLoad {
  S own[Q];
  S pull[Q];
  uint32_t known;   // bit i: pull source of direction i is a lattice node
  uint32_t out;     // bit i: destination x + e_i leaves the lattice
  double mirror;    // on a Neumann wall: M0 of the pulls at the mirror node
};

// Mirror node of (x, y) across the Neumann walls it lies on (eq.
// Neu_on_q): one cell inward across each, the diagonal neighbour at the
// corner of two.  Returns false when the node lies on no Neumann wall.
template <int Q>
__device__ __forceinline__ bool neumann_mirror(const StepArgs &A, int x, int y,
                                               int &mx, int &my) {
  mx = x;
  my = y;
  const int neu = A.neu;
  if (!neu) return false;
  bool on = false;
  if ((neu & 1) && x == 0) { mx = 1; on = true; }
  if ((neu & 2) && x == A.nx - 1) { mx = A.nx - 2; on = true; }
  if (Q > 3 && (neu & 4) && y == 0) { my = 1; on = true; }
  if (Q > 3 && (neu & 8) && y == A.ny - 1) { my = A.ny - 2; on = true; }
  return on;
}

// M0 of the pulled populations at the mirror node (mx, my), sum_i
// Omega_i(m - e_i).  The host admits no bounce-back wall beside a Neumann
// one, so every source is a lattice node (periodic axes wrap); the
// indices are clamped all the same so that no load leaves the planes.
template <int Q, typename S>
__device__ __forceinline__ double mirror_m0(const StepArgs &A,
                                            gptr<const S> __restrict__ src,
                                            int mx, int my) {
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int sx = mx - cx<Q>(i), sy = my - cy<Q>(i);
    if (sx < 0) sx = A.periodic_x ? sx + A.nx : 0;
    if (sx >= A.nx) sx = A.periodic_x ? sx - A.nx : A.nx - 1;
    if (sy < 0) sy = A.periodic_y ? sy + A.ny : 0;
    if (sy >= A.ny) sy = A.periodic_y ? sy - A.ny : A.ny - 1;
    m += (double)src[i * A.plane + (int64_t)sy * A.nx + sx];
  }
  return m;
}

// FAST: every pull source and destination of the node lies inside the
// lattice without wrapping (interior tile); no checks are compiled.
// Otherwise sources are wrapped on periodic axes and clamped into the
// lattice elsewhere, so every load is issued unconditionally (no branch
// around a load); the values of unknown directions are then zeroed and
// left to the closure.
template <int Q, typename S, bool FAST, bool NEU = false>
__device__ __forceinline__ void load_node(const StepArgs &A,
                                          gptr<const S> __restrict__ src,
                                          int x, int y, NodeLoad<Q, S> &L) {
  const int64_t P = A.plane;
  const int nx = A.nx;
  int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
  bool vxm = true, vxp = true, vym = true, vyp = true;
  if (!FAST) {
    if (xm < 0) {
      vxm = A.periodic_x != 0;
      xm = vxm ? xm + nx : 0;
    }
    if (xp >= nx) {
      vxp = A.periodic_x != 0;
      xp = vxp ? xp - nx : nx - 1;
    }
    if (Q > 3) {
      if (ym < 0) {
        vym = A.periodic_y != 0;
        ym = vym ? ym + A.ny : 0;
      }
      if (yp >= A.ny) {
        vyp = A.periodic_y != 0;
        yp = vyp ? yp - A.ny : A.ny - 1;
      }
    }
  }
  // row pointers and unsigned column offsets: when the caller's y is
  // wave-uniform the row pointers are scalar and each load takes a scalar
  // base plus a 32-bit lane offset
  const gptr<const S> r0 = src + (int64_t)y * nx;
  const gptr<const S> rm = src + (int64_t)ym * nx;
  const gptr<const S> rp = src + (int64_t)yp * nx;
#pragma unroll
  for (int j = 0; j < Q; ++j) L.own[j] = (r0 + j * P)[(uint32_t)x];
  L.known = 1u;
  L.out = 0u;
  L.pull[0] = L.own[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int ex = cx<Q>(i), ey = cy<Q>(i);
    const int sx = ex == 1 ? xm : (ex == -1 ? xp : x);
    const gptr<const S> sr = ey == 1 ? rm : (ey == -1 ? rp : r0);
    L.pull[i] = (sr + i * P)[(uint32_t)sx];
    if (!FAST) {
      const bool ok = (ex == 1 ? vxm : (ex == -1 ? vxp : true)) &&
                      (ey == 1 ? vym : (ey == -1 ? vyp : true));
      const bool leaves = (ex == 1 ? !vxp : (ex == -1 ? !vxm : false)) ||
                          (ey == 1 ? !vyp : (ey == -1 ? !vym : false));
      if (ok) L.known |= 1u << i;
      else L.pull[i] = (S)0;
      if (leaves) L.out |= 1u << i;
    } else {
      L.known |= 1u << i;
    }
  }
  L.mirror = 0.0;
  if (!FAST && NEU) {
    int mx, my;
    if (neumann_mirror<Q>(A, x, y, mx, my))
      L.mirror = mirror_m0<Q, S>(A, src, mx, my);
  }
}

// Does the unknown direction i of node (x, y) leave the lattice only
// through bounce-back walls?  (A periodic axis wraps and is never left.)
template <int Q>
__device__ __forceinline__ bool leaves_by_bounceback(const StepArgs &A, int x, int y,
                                            int i) {
  const int sx = x - cx<Q>(i), sy = y - cy<Q>(i);
  if (sx < 0 && A.bc[0] != BC_BOUNCEBACK && !A.periodic_x) return false;
  if (sx >= A.nx && A.bc[1] != BC_BOUNCEBACK && !A.periodic_x) return false;
  if (Q > 3 && sy < 0 && A.bc[2] != BC_BOUNCEBACK && !A.periodic_y)
    return false;
  if (Q > 3 && sy >= A.ny && A.bc[3] != BC_BOUNCEBACK && !A.periodic_y)
    return false;
  return true;
}

template <int Q>
__device__ __forceinline__ int dirichlet_wall(const StepArgs &A, int x, int y) {
  if (x == 0 && A.bc[0] == BC_DIRICHLET) return 0;
  if (x == A.nx - 1 && A.bc[1] == BC_DIRICHLET) return 1;
  if (Q > 3 && y == 0 && A.bc[2] == BC_DIRICHLET) return 2;
  if (Q > 3 && y == A.ny - 1 && A.bc[3] == BC_DIRICHLET) return 3;
  return -1;
}

__device__ __forceinline__ double wall_value(const StepArgs &A, int wall, int x,
                                    int y) {
  const double *p = A.prof[wall];
  return p ? to_global(p)[wall < 2 ? y : x] : A.wall_T[wall];
}

// Closure of the unknown pulled populations (Section 4.2):
// 1. bounce-back q_i = q_opp(i) for unknowns beyond bounce-back walls
//    only, when the opposite is known;
// 2. on a Dirichlet node, the zeroth moment is fixed to
//    T_D + (phi(T_D) - phi(T))/Ste (eq. Dir_on_q), so that the new
//    temperature is T_D; the deficit is shared by weight among the
//    remaining unknowns.  EEBM: the zeroth moment is the wall enthalpy
//    T_D + l(T_D)/Ste (l = 1 above T_m, else 0), whose Theta is T_D;
//    ILFBM (M0 = theta): T_D itself;
// 3. on a Neumann node (not Dirichlet), M0(q) is set to M0 of the pulls
//    at the mirror node (eq. Neu_on_q; `mirror`), the deficit shared by
//    weight among the remaining unknowns (one on flat D2Q5/D1Q3 walls);
// 4. anything left (corner of two bounce-back walls): own Omega_opp(i).
// Masks of how each unknown was closed (for the reverse mode).
struct CloseInfo {
  uint32_t bb = 0;     // bounce-back from a known opposite
  uint32_t share = 0;  // Dirichlet deficit share
  uint32_t own = 0;    // own post-collision opposite population
  int wall = -1;       // Dirichlet wall of the node
  double TD = 0.0, wu = 0.0;
};

// PLATEAU (quiet-only kernels): phi is taken only where it is exactly 0
// or 1 (|T - T_m| > 20 delta), with no exp in the code; a Dirichlet node
// whose wall or own temperature lies nearer the band sets *near instead
// (its update is then left to a full kernel).
template <int Q, int SCH = SCHEME_IREBM, bool NEU = true,
          bool PLATEAU = false>
__device__ __forceinline__ double close_node(const StepArgs &A, int x, int y,
                                    double th, const double *om, double *q,
                                    uint32_t known, double mirror,
                                    CloseInfo *ci = nullptr,
                                    int *near = nullptr) {
  uint32_t set = known;
  double fill = 0.0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int o = opp<Q>(i);
    if (!(known >> i & 1u) && (known >> o & 1u) &&
        leaves_by_bounceback<Q>(A, x, y, i)) {
      q[i] = q[o];
      set |= 1u << i;
      fill += q[i];
      if (ci) ci->bb |= 1u << i;
    }
  }
  const int wall = dirichlet_wall<Q>(A, x, y);
  if (ci) ci->wall = wall;
  if (wall >= 0) {
    const double TD = wall_value(A, wall, x, y);
    double D;
    if constexpr (PLATEAU && SCH == SCHEME_IREBM) {
      const double ud = (TD - A.tm) * A.inv_delta;
      const double ut = (th - A.tm) * A.inv_delta;
      if (!(fabs(ud) > 20.0 && fabs(ut) > 20.0)) *near = 1;
      D = TD + ((ud > 20.0 ? 1.0 : 0.0) - (ut > 20.0 ? 1.0 : 0.0)) *
                   A.inv_ste;
    } else {
      D = SCH == SCHEME_EEBM    ? TD + (TD > A.tm ? A.inv_ste : 0.0)
          : SCH == SCHEME_ILFBM ? TD
                                : TD + (phi_only(TD, A.tm, A.inv_delta) -
                                        phi_only(th, A.tm, A.inv_delta)) *
                                           A.inv_ste;
    }
    double wu = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (set >> i & 1u) D -= q[i];
      else wu += wt<Q>(i);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (!(set >> i & 1u)) {
        q[i] = D * (wt<Q>(i) / wu);
        fill += q[i];
        if (ci) ci->share |= 1u << i;
      }
    if (ci) {
      ci->TD = TD;
      ci->wu = wu;
    }
    set = (1u << Q) - 1u;
  } else if (NEU) {
    int mx, my;
    if (neumann_mirror<Q>(A, x, y, mx, my)) {
      double D = mirror, wu = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (set >> i & 1u) D -= q[i];
        else wu += wt<Q>(i);
      }
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (!(set >> i & 1u)) {
          q[i] = D * (wt<Q>(i) / wu);
          fill += q[i];
        }
      set = (1u << Q) - 1u;
    }
  }
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (!(set >> i & 1u)) {
      q[i] = om[opp<Q>(i)];
      fill += q[i];
      if (ci) ci->own |= 1u << i;
    }
  return fill;
}

// Which pull sources of node (x, y) are lattice nodes (bit i of known,
// wrapping periodic axes) and which destinations x + e_i leave the lattice
// (bit i of out): the masks load_node computes, from coordinates only.
template <int Q>
__device__ __forceinline__ void node_masks(const StepArgs &A, int x, int y,
                                           uint32_t &known, uint32_t &out) {
  const bool vxm = x - 1 >= 0 || A.periodic_x != 0;
  const bool vxp = x + 1 < A.nx || A.periodic_x != 0;
  const bool vym = Q == 3 || y - 1 >= 0 || A.periodic_y != 0;
  const bool vyp = Q == 3 || y + 1 < A.ny || A.periodic_y != 0;
  known = 1u;
  out = 0u;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int ex = cx<Q>(i), ey = cy<Q>(i);
    const bool ok = (ex == 1 ? vxm : (ex == -1 ? vxp : true)) &&
                    (ey == 1 ? vym : (ey == -1 ? vyp : true));
    const bool leaves = (ex == 1 ? !vxp : (ex == -1 ? !vxm : false)) ||
                        (ey == 1 ? !vyp : (ey == -1 ? !vym : false));
    if (ok) known |= 1u << i;
    if (leaves) out |= 1u << i;
  }
}

// The update of one node from its loads: the next state's populations
// into v (rounded to the storage type).  QUIET: a kernel built for quiet
// nodes only (no Newton code, so fewer registers); a node that is not
// quiet is counted in st.solves, v is left meaningless, and the caller
// hands its work item to a full kernel.
template <int Q, typename S, int MODE, bool FAST, bool QUIET = false>
__device__ __forceinline__ void update_values(const StepArgs &A, int x, int y,
                                              const NodeLoad<Q, S> &L,
                                              NodeStats &st, S v[Q]) {
  constexpr bool PLAIN = base_mode(MODE) == kPlain;
  constexpr bool EEBM = base_mode(MODE) == kEebm;
  constexpr bool NEU = neumann_mode(MODE);
  double om[Q], q[Q];
  double th = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    om[j] = (double)L.own[j];
    th += om[j];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) q[i] = (double)L.pull[i];
  int near = 0;
  if (!FAST) {
    if (L.known != (1u << Q) - 1u)
      st.flux_in +=
          close_node<Q, EEBM ? SCHEME_EEBM : SCHEME_IREBM, NEU, QUIET>(
              A, x, y, th, om, q, L.known, L.mirror, nullptr, &near);
    if (L.out) {
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (L.out >> i & 1u) st.flux_out += om[i];
    }
  }
  double m0 = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) m0 += q[i];
  if constexpr (EEBM) {
    // Algorithm 2: H = m0, explicit temperature, BGK collision
    const double tq = eebm_theta(m0, A.tm, A.inv_ste);
    v[0] = (S)(A.a * q[0] + A.inv_tau * (m0 - (1.0 - wt<Q>(0)) * tq));
#pragma unroll
    for (int i = 1; i < Q; ++i)
      v[i] = (S)(A.a * q[i] + A.wtau[wclass<Q>(i)] * tq);
    return;
  }
  // Quiet node: far below the melting band before and after (phi = 0 and
  // phi' = 0 exactly) and the Newton solve is the closed form of newton()
  // (T~ = m0, same iteration count).  Then f~ = q exactly and M0(f~) = m0
  // (the same sum in the same order), so the update reduces to
  // Omega' = a q + (w/tau) m0 with the same rounding.
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
        v[i] = (S)(A.a * q[i] + A.wtau[wclass<Q>(i)] * m0);
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
    f[i] = q[i] + A.wste[wclass<Q>(i)] * dphi_s;
    tsum += f[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    v[i] = (S)(A.a * f[i] + A.wtau[wclass<Q>(i)] * tsum);
  const double res = fabs(tn + pnew * A.inv_ste - (m0 + pth * A.inv_ste));
  st.max_it = it > st.max_it ? it : st.max_it;
  st.nonconv += conv ? 0 : 1;
  st.max_res = res > st.max_res ? res : st.max_res;
}

// The update of one node from its loads; writes the next state.
template <int Q, typename S, int MODE, bool FAST, bool NT = false>
__device__ __forceinline__ void update_node(const StepArgs &A,
                                            gptr<S> __restrict__ dst, int x,
                                            int y, const NodeLoad<Q, S> &L,
                                            NodeStats &st) {
  S v[Q];
  update_values<Q, S, MODE, FAST>(A, x, y, L, st, v);
  const gptr<S> row = dst + (int64_t)y * A.nx;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const gptr<S> p = (row + i * A.plane) + (uint32_t)x;
    if (NT) __builtin_nontemporal_store(v[i], p);
    else *p = v[i];
  }
}

// ---- wave and block reductions (wave64)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace irebm
