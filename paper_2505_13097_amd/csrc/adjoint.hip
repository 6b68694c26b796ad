// adjoint.hip -- reverse mode of the IREBM step on the post-collision
// state, and a checkpointed driver (tape) for front-misfit gradients.
//
// Forward step at node x (Algorithm 3 in the Omega form of this library):
//   T = sum_j Omega_j(x),  q_i = Omega_i(x - e_i) (or a closure),
//   m0 = sum q_i,  T~ solves R = T~ + phi(T~)/Ste - m0 - phi(T)/Ste = 0,
//   s = (phi(T) - phi(T~))/Ste,  f~_i = q_i + w_i s,
//   T' = sum f~_i,  Omega'_i = a f~_i + (w_i/tau) T'      (a = 1 - 1/tau).
// Reverse, given Omega'bar at x:
//   T'bar = sum (w_i/tau) Omega'bar_i,  f~bar_i = a Omega'bar_i + T'bar,
//   sbar = sum w_i f~bar_i,  qbar_i = f~bar_i,
//   source: Tbar += sbar phi'(T)/Ste,  T~bar = -sbar phi'(T~)/Ste,
//   Newton root by the implicit-function theorem (J = 1 + phi'(T~)/Ste,
//   exact at converged nodes): m0bar = T~bar/J,
//   Tbar += T~bar (phi'(T)/Ste)/J, plus the Ste and delta terms,
//   qbar_i += m0bar, then the closures in reverse order,
// and the transposes of the pull and of T = sum Omega:
//   Omegabar_i(y) = qbar_i(y + e_i) + Tbar(y).
// The pull transpose is again a radius-1 stencil, so a reverse step is two
// kernels: adj_local (per node: recompute the forward, write qbar and
// Tbar) and adj_pull (gather).  Parameter gradients are summed per block
// in a fixed order and accumulated across steps in per-block slots;
// Dirichlet wall-temperature gradients are accumulated per wall node by
// the one thread owning it.  Adjoint arrays are FP64 in every storage mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_util.hpp"
#include "kernels.hpp"
#include "lbm_stefan.h"
#include "lbm_stefan_internal.hpp"

using namespace irebm;

namespace {

struct AdjArgs {
  StepArgs A;              // A.src: the forward state at step n
  const double *abar_in;   // Omega'bar (q planes) / abar_0 for the init term
  const double *qbar_in;   // qbar, Tbar of the later step (gather input)
  const double *tbar_in;
  double *qbar;            // q planes (node-local output)
  double *tbar;            // n
  double *abar_out;        // q planes
  int32_t nblocks, per_xcd;  // node blocks of 256, blocks per XCD chunk
  double *gS, *gD;         // per-block partial sums (accumulated)
  double *gwall[4];        // per wall node (accumulated)
  const double *r;         // dL/dfront per row (front vjp)
  double dx, delta, ste;
};

__device__ __forceinline__ double dphi_ddelta(double t, double tm, double delta,
                                     double dph) {
  return -((t - tm) / delta) * dph;
}

// block sums of a and b (fixed order) added to the block's slots *ga, *gb
__device__ __forceinline__ void block_add2(double a, double b, double *ga, double *gb) {
  __shared__ double s[8];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s[w] = a;
    s[4 + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *ga += (s[0] + s[1]) + (s[2] + s[3]);
    *gb += (s[4] + s[5]) + (s[6] + s[7]);
  }
}

__device__ __forceinline__ int wall_index(int wall, int x, int y) {
  return wall < 2 ? y : x;
}

// Node of block-local thread `tid` in 1-D blocks of 256 nodes, blocks
// remapped so that each XCD (block b runs on XCD b mod 8) sweeps one
// contiguous band of rows; `blk` is the block's slot index.
__device__ __forceinline__ int64_t adj_node(const AdjArgs &G, int &blk) {
  blk = (int)((blockIdx.x & 7) * G.per_xcd + (blockIdx.x >> 3));
  return (int64_t)blk * 256 + threadIdx.x;
}

// per node: recompute the forward step at (x, y) from the state in G.A.src,
// then reverse it from ab = Omega'bar(x) down to qbar and Tbar (written to
// qbar_out, tbar_out) and the parameter and wall-temperature gradients
template <int Q, typename S, bool PLAIN>
__device__ __forceinline__ void local_reverse(const AdjArgs &G, int x, int y,
                                             int64_t k, const double ab[Q],
                                             double *qbar_out, double *tbar_out,
                                             double &accS, double &accD) {
  const StepArgs &A = G.A;
  NodeLoad<Q, S> L;
  load_node<Q, S, false>(A, to_global((const S *)A.src), x, y, L);
  double om[Q], q[Q], th = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    om[j] = (double)L.own[j];
    th += om[j];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) q[i] = (double)L.pull[i];
  CloseInfo ci;
  if (L.known != (1u << Q) - 1u)
    close_node<Q>(A, x, y, th, om, q, L.known, 0.0, &ci);
  double m0 = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) m0 += q[i];
  const double is = A.inv_ste, tm = A.tm, dl = G.delta;
  double P, d;
  phi_dphi(th, tm, A.inv_delta, P, d);
  int it;
  bool conv;
  PhiAt at;
  const double tn = newton<PLAIN>(m0, th, P, d, A, it, conv, at);
  double Pt = at.ph, dt = at.dph;
  if (!at.ok) phi_dphi(tn, tm, A.inv_delta, Pt, dt);
  const double dP = dphi_ddelta(th, tm, dl, d);
  const double dPt = dphi_ddelta(tn, tm, dl, dt);
  // reverse of Omega' = a f~ + (w/tau) sum f~
  double qb[Q];
  double tpb = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) tpb += A.wtau[wclass<Q>(i)] * ab[i];
  double sb = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    qb[i] = A.a * ab[i] + tpb;
    sb += wt<Q>(i) * qb[i];
  }
  // source s = (P - Pt)/Ste
  double thl = sb * d * is;
  const double tnb = -sb * dt * is;
  double Sb = -sb * (P - Pt) * is * is;
  double Db_ = sb * (dP - dPt) * is;
  // Newton root (implicit-function theorem)
  const double J = 1.0 + dt * is;
  const double m0b = tnb / J;
  thl += tnb * (d * is) / J;
  Sb += tnb * (Pt - P) * is * is / J;
  Db_ += -tnb * (dPt - dP) * is / J;
#pragma unroll
  for (int i = 0; i < Q; ++i) qb[i] += m0b;
  // closures, reversed: Dirichlet share, then bounce-back
  if (ci.share) {
    double Db = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (ci.share >> i & 1u) Db += qb[i] * (wt<Q>(i) / ci.wu);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (!(ci.share >> i & 1u) && !(ci.own >> i & 1u)) qb[i] -= Db;
    double PD, dPD;
    phi_dphi(ci.TD, tm, A.inv_delta, PD, dPD);
    G.gwall[ci.wall][wall_index(ci.wall, x, y)] += Db * (1.0 + dPD * is);
    thl += -Db * d * is;
    Sb += -Db * (PD - P) * is * is;
    Db_ += Db * (dphi_ddelta(ci.TD, tm, dl, dPD) - dP) * is;
  }
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (ci.bb >> i & 1u) qb[opp<Q>(i)] += qb[i];
#pragma unroll
  for (int i = 0; i < Q; ++i) qbar_out[i * A.plane + k] = qb[i];
  tbar_out[k] = thl;
  accS = Sb;
  accD = Db_;
}

// Omegabar_i(y) = qbar_i(y + e_i) (where that node pulls direction i from
// y) + Tbar(y) + own-population closures at y, from the qbar and Tbar a
// node-local reverse left
template <int Q>
__device__ __forceinline__ void pull_reverse(const AdjArgs &G,
                                             const double *qbar,
                                             const double *tbar, int x, int y,
                                             int64_t k, double out[Q]) {
  const StepArgs &A = G.A;
  const double tb = tbar[k];
#pragma unroll
  for (int i = 0; i < Q; ++i) out[i] = tb;
  uint32_t known = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int ex = cx<Q>(i), ey = cy<Q>(i);
    // destination z = y + e_i
    int zx = x + ex, zy = y + ey;
    bool ok = true;
    if (zx < 0 || zx >= A.nx) {
      if (A.periodic_x) zx = (zx + A.nx) % A.nx; else ok = false;
    }
    if (zy < 0 || zy >= A.ny) {
      if (A.periodic_y) zy = (zy + A.ny) % A.ny; else ok = false;
    }
    if (ok) out[i] += qbar[i * A.plane + (int64_t)zy * A.nx + zx];
    // source x - e_i of this node (for its own closures)
    int sx = x - ex, sy = y - ey;
    bool sk = true;
    if (sx < 0 || sx >= A.nx) sk = A.periodic_x != 0;
    if (sy < 0 || sy >= A.ny) sk = sk && A.periodic_y != 0;
    if (sk) known |= 1u << i;
  }
  if (known != (1u << Q) - 1u && dirichlet_wall<Q>(A, x, y) < 0) {
    // unknowns closed by the node's own Omega_opp (both directions unknown)
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int o = opp<Q>(i);
      const bool bb = (known >> o & 1u) && leaves_by_bounceback<Q>(A, x, y, i);
      if (!(known >> i & 1u) && !bb) out[o] += qbar[i * A.plane + k];
    }
  }
}

// node-local half of a reverse step: Omega'bar from G.abar_in
template <int Q, typename S, bool PLAIN>
__global__ __launch_bounds__(256) void adj_local_kernel(AdjArgs G) {
  int blk;
  const int64_t k = adj_node(G, blk);
  double accS = 0.0, accD = 0.0;
  if (blk < G.nblocks && k < G.A.plane) {
    const int x = (int)(k % G.A.nx), y = (int)(k / G.A.nx);
    double ab[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) ab[i] = G.abar_in[i * G.A.plane + k];
    local_reverse<Q, S, PLAIN>(G, x, y, k, ab, G.qbar, G.tbar, accS, accD);
  }
  if (blk < G.nblocks) block_add2(accS, accD, G.gS + blk, G.gD + blk);
}

// gather half of a reverse step: Omegabar into G.abar_out
template <int Q>
__global__ __launch_bounds__(256) void adj_pull_kernel(AdjArgs G) {
  int blk;
  const int64_t k = adj_node(G, blk);
  if (blk >= G.nblocks || k >= G.A.plane) return;
  const int x = (int)(k % G.A.nx), y = (int)(k / G.A.nx);
  double out[Q];
  pull_reverse<Q>(G, G.qbar_in, G.tbar_in, x, y, k, out);
#pragma unroll
  for (int i = 0; i < Q; ++i) G.abar_out[i * G.A.plane + k] = out[i];
}

// the gather half of reverse step n + 1 fused with the node-local half of
// reverse step n: Omega'bar(x) for step n is formed in registers from the
// qbar/Tbar of step n + 1 (G.qbar_in, G.tbar_in) and never stored
template <int Q, typename S, bool PLAIN>
__global__ __launch_bounds__(256) void adj_fused_kernel(AdjArgs G) {
  int blk;
  const int64_t k = adj_node(G, blk);
  double accS = 0.0, accD = 0.0;
  if (blk < G.nblocks && k < G.A.plane) {
    const int x = (int)(k % G.A.nx), y = (int)(k / G.A.nx);
    double ab[Q];
    pull_reverse<Q>(G, G.qbar_in, G.tbar_in, x, y, k, ab);
    local_reverse<Q, S, PLAIN>(G, x, y, k, ab, G.qbar, G.tbar, accS, accD);
  }
  if (blk < G.nblocks) block_add2(accS, accD, G.gS + blk, G.gD + blk);
}

// seed: Omegabar_j(x, y) = r(y) dx w_x phi'(T(x, y)) for every j, and the
// delta-dependence of the front itself
template <int Q, typename S>
__global__ __launch_bounds__(256) void front_vjp_kernel(AdjArgs G) {
  const StepArgs &A = G.A;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double accD = 0.0;
  if (k < A.plane) {
    const int x = (int)(k % A.nx), y = (int)(k / A.nx);
    const S *src = (const S *)A.src;
    double T = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) T += (double)src[j * A.plane + k];
    double P, d;
    phi_dphi(T, A.tm, A.inv_delta, P, d);
    const double wx = (x == 0 || x == A.nx - 1) ? 0.5 : 1.0;
    const double c = G.r[y] * G.dx * wx;
#pragma unroll
    for (int j = 0; j < Q; ++j) G.abar_out[j * A.plane + k] = c * d;
    accD = c * dphi_ddelta(T, A.tm, G.delta, d);
  }
  block_add2(0.0, accD, G.gS + blockIdx.x, G.gD + blockIdx.x);
}

// initial state: Omega_i = w_i T_D at Dirichlet nodes
template <int Q>
__global__ __launch_bounds__(256) void init_term_kernel(AdjArgs G) {
  const StepArgs &A = G.A;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= A.plane) return;
  const int x = (int)(k % A.nx), y = (int)(k / A.nx);
  const int wall = dirichlet_wall<Q>(A, x, y);
  if (wall < 0) return;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) s += wt<Q>(i) * G.abar_in[i * A.plane + k];
  G.gwall[wall][wall_index(wall, x, y)] += s;
}

struct AdjLayout {
  size_t abar0, abar1, qbar[2], tbar[2], gS, gD, gwall, r, out, total;
  int64_t nblocks, wlen;
};

AdjLayout adj_layout(const lbm_stefan_params *p) {
  AdjLayout L;
  const int64_t n = p->nx * p->ny;
  L.nblocks = (n + 255) / 256;
  L.wlen = std::max(p->nx, p->ny);
  size_t o = 0;
  L.abar0 = o;
  o += align256((size_t)p->q * n * 8);
  L.abar1 = o;
  o += align256((size_t)p->q * n * 8);
  for (int c = 0; c < 2; ++c) {
    L.qbar[c] = o;
    o += align256((size_t)p->q * n * 8);
    L.tbar[c] = o;
    o += align256((size_t)n * 8);
  }
  L.gS = o;
  o += align256((size_t)L.nblocks * 8);
  L.gD = o;
  o += align256((size_t)L.nblocks * 8);
  L.gwall = o;
  o += align256((size_t)4 * L.wlen * 8);
  L.r = o;
  o += align256((size_t)p->ny * 8);
  L.out = o;
  o += 256;
  L.total = o;
  return L;
}

int check_adj(lbm_stefan_t *h) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  if (!h->layout.adjoint)
    return fail(h, LBM_STEFAN_EINVAL,
                "handle was created without LBM_FLAG_ADJOINT");
  return LBM_STEFAN_OK;
}

AdjArgs make_args(lbm_stefan_t *h) {
  const AdjLayout L = adj_layout(&h->p);
  AdjArgs G;
  std::memset(&G, 0, sizeof(G));
  fill_step_args(h, &G.A);
  char *base = h->adj;
  G.qbar = (double *)(base + L.qbar[0]);
  G.tbar = (double *)(base + L.tbar[0]);
  G.qbar_in = G.qbar;
  G.tbar_in = G.tbar;
  G.nblocks = (int32_t)L.nblocks;
  G.per_xcd = (int32_t)((L.nblocks + 7) / 8);
  G.gS = (double *)(base + L.gS);
  G.gD = (double *)(base + L.gD);
  for (int w = 0; w < 4; ++w) G.gwall[w] = (double *)(base + L.gwall) + w * L.wlen;
  G.r = (const double *)(base + L.r);
  G.dx = h->p.dx;
  G.delta = h->p.delta;
  G.ste = h->p.ste;
  return G;
}

unsigned node_blocks(const lbm_stefan_t *h) {
  return (unsigned)((h->p.nx * h->p.ny + 255) / 256);
}

// grid of the remapped node kernels: eight XCD chunks of per_xcd blocks
unsigned remapped_grid(const AdjArgs &G) { return 8u * (unsigned)G.per_xcd; }

// node-local half of reverse step n: state_n and Omega'bar (abar_in) ->
// qbar/Tbar buffer c
hipError_t local_async(lbm_stefan_t *h, const void *state,
                       const double *abar_in, int c) {
  const AdjLayout L = adj_layout(&h->p);
  AdjArgs G = make_args(h);
  G.A.src = state;
  G.abar_in = abar_in;
  G.qbar = (double *)(h->adj + L.qbar[c]);
  G.tbar = (double *)(h->adj + L.tbar[c]);
  const bool plain = h->p.newton_mode == LBM_NEWTON_PLAIN;
  return dispatch_qs(h->p.q, h->p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    if (plain)
      adj_local_kernel<Q, S, true><<<remapped_grid(G), 256, 0, h->stream>>>(G);
    else
      adj_local_kernel<Q, S, false><<<remapped_grid(G), 256, 0, h->stream>>>(G);
    return hipGetLastError();
  });
}

// gather half of a reverse step: qbar/Tbar buffer c -> Omegabar (abar_out)
hipError_t pull_async(lbm_stefan_t *h, int c, double *abar_out) {
  const AdjLayout L = adj_layout(&h->p);
  AdjArgs G = make_args(h);
  G.qbar_in = (const double *)(h->adj + L.qbar[c]);
  G.tbar_in = (const double *)(h->adj + L.tbar[c]);
  G.abar_out = abar_out;
  return dispatch_qs(h->p.q, h->p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    (void)sizeof(S);
    adj_pull_kernel<Q><<<remapped_grid(G), 256, 0, h->stream>>>(G);
    return hipGetLastError();
  });
}

// gather half of reverse step n + 1 (qbar/Tbar buffer c) fused with the
// node-local half of reverse step n (state_n) -> buffer c ^ 1
hipError_t fused_async(lbm_stefan_t *h, const void *state, int c) {
  const AdjLayout L = adj_layout(&h->p);
  AdjArgs G = make_args(h);
  G.A.src = state;
  G.qbar_in = (const double *)(h->adj + L.qbar[c]);
  G.tbar_in = (const double *)(h->adj + L.tbar[c]);
  G.qbar = (double *)(h->adj + L.qbar[c ^ 1]);
  G.tbar = (double *)(h->adj + L.tbar[c ^ 1]);
  const bool plain = h->p.newton_mode == LBM_NEWTON_PLAIN;
  return dispatch_qs(h->p.q, h->p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    if (plain)
      adj_fused_kernel<Q, S, true><<<remapped_grid(G), 256, 0, h->stream>>>(G);
    else
      adj_fused_kernel<Q, S, false><<<remapped_grid(G), 256, 0, h->stream>>>(G);
    return hipGetLastError();
  });
}

// one whole reverse step: Omega'bar of step n + 1 -> Omegabar of step n
hipError_t adjoint_step_async(lbm_stefan_t *h, const void *state,
                              const double *abar_in, double *abar_out) {
  hipError_t e = local_async(h, state, abar_in, 0);
  if (e != hipSuccess) return e;
  return pull_async(h, 0, abar_out);
}

hipError_t front_vjp_async(lbm_stefan_t *h, const void *state,
                           const double *dL_dfront_host, double *abar) {
  const AdjLayout L = adj_layout(&h->p);
  hipError_t e = hipMemcpyAsync(h->adj + L.r, dL_dfront_host, h->p.ny * 8,
                                hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return e;
  AdjArgs G = make_args(h);
  G.A.src = state;
  G.abar_out = abar;
  const unsigned nb = node_blocks(h);
  return dispatch_qs(h->p.q, h->p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    front_vjp_kernel<Q, S><<<nb, 256, 0, h->stream>>>(G);
    return hipGetLastError();
  });
}

hipError_t init_term_async(lbm_stefan_t *h, const double *abar0) {
  AdjArgs G = make_args(h);
  G.abar_in = abar0;
  const unsigned nb = node_blocks(h);
  return dispatch_qs(h->p.q, h->p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    (void)sizeof(S);
    init_term_kernel<Q><<<nb, 256, 0, h->stream>>>(G);
    return hipGetLastError();
  });
}

hipError_t reset_async(lbm_stefan_t *h) {
  const AdjLayout L = adj_layout(&h->p);
  hipError_t e = zero_async(h->adj + L.gS, L.nblocks * 8, h->stream);
  if (e == hipSuccess) e = zero_async(h->adj + L.gD, L.nblocks * 8, h->stream);
  if (e == hipSuccess)
    e = zero_async(h->adj + L.gwall, 4 * L.wlen * 8, h->stream);
  return e;
}

// gradients to host: g_wall (x-, x+ of length ny, then y-, y+ of length
// nx; nullable), dL/dSte and dL/ddelta (nullable)
int read_gradients(lbm_stefan_t *h, double *g_wall, double *g_ste,
                   double *g_delta) {
  const AdjLayout L = adj_layout(&h->p);
  double *out = (double *)(h->adj + L.out);
  sum_kernel<<<1, 256, 0, h->stream>>>((const double *)(h->adj + L.gS),
                                       L.nblocks, out);
  sum_kernel<<<1, 256, 0, h->stream>>>((const double *)(h->adj + L.gD),
                                       L.nblocks, out + 1);
  HIPCHK(h, hipGetLastError());
  double sd[2];
  HIPCHK(h, hipMemcpyAsync(sd, out, 16, hipMemcpyDeviceToHost, h->stream));
  std::vector<double> gw;
  if (g_wall) {
    gw.resize(4 * L.wlen);
    HIPCHK(h, hipMemcpyAsync(gw.data(), h->adj + L.gwall, gw.size() * 8,
                             hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (g_ste) *g_ste = sd[0];
  if (g_delta) *g_delta = sd[1];
  if (g_wall) {
    const int64_t nx = h->p.nx, ny = h->p.ny;
    std::copy(gw.begin(), gw.begin() + ny, g_wall);
    std::copy(gw.begin() + L.wlen, gw.begin() + L.wlen + ny, g_wall + ny);
    std::copy(gw.begin() + 2 * L.wlen, gw.begin() + 2 * L.wlen + nx,
              g_wall + 2 * ny);
    std::copy(gw.begin() + 3 * L.wlen, gw.begin() + 3 * L.wlen + nx,
              g_wall + 2 * ny + nx);
  }
  if (!std::isfinite(sd[0]) || !std::isfinite(sd[1]))
    return fail(h, LBM_STEFAN_ENAN, "a gradient is not finite");
  return LBM_STEFAN_OK;
}

size_t state_bytes(const lbm_stefan_params &p) {
  return (size_t)p.q * p.nx * p.ny * (p.storage == LBM_STORE_F64 ? 8 : 4);
}

}  // namespace

size_t irebm::adjoint_bytes(const lbm_stefan_params *p, int64_t max_items) {
  (void)max_items;
  return adj_layout(p).total;
}

extern "C" {

int lbm_stefan_adjoint_reset(lbm_stefan_t *h) {
  if (int rc = check_adj(h)) return rc;
  DeviceGuard g(h->device);
  HIPCHK(h, reset_async(h));
  return LBM_STEFAN_OK;
}

int lbm_stefan_front_vjp(lbm_stefan_t *h, const void *state,
                         const double *dL_dfront, double *abar) {
  if (int rc = check_adj(h)) return rc;
  if (!state || !dL_dfront || !abar)
    return fail(h, LBM_STEFAN_EINVAL, "NULL argument");
  DeviceGuard g(h->device);
  HIPCHK(h, front_vjp_async(h, state, dL_dfront, abar));
  // dL_dfront is host memory read by an asynchronous copy
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return LBM_STEFAN_OK;
}

int lbm_stefan_adjoint_step(lbm_stefan_t *h, const void *state_n,
                            const double *abar_np1, double *abar_n) {
  if (int rc = check_adj(h)) return rc;
  if (!state_n || !abar_np1 || !abar_n || abar_np1 == abar_n)
    return fail(h, LBM_STEFAN_EINVAL, "NULL or aliased argument");
  DeviceGuard g(h->device);
  HIPCHK(h, adjoint_step_async(h, state_n, abar_np1, abar_n));
  return LBM_STEFAN_OK;
}

int lbm_stefan_adjoint_initial_state(lbm_stefan_t *h, const double *abar_0) {
  if (int rc = check_adj(h)) return rc;
  if (!abar_0) return fail(h, LBM_STEFAN_EINVAL, "NULL argument");
  DeviceGuard g(h->device);
  HIPCHK(h, init_term_async(h, abar_0));
  return LBM_STEFAN_OK;
}

int lbm_stefan_adjoint_gradients(lbm_stefan_t *h, double *g_wall,
                                 double *g_ste, double *g_delta) {
  if (int rc = check_adj(h)) return rc;
  DeviceGuard g(h->device);
  return read_gradients(h, g_wall, g_ste, g_delta);
}

int lbm_stefan_tape_bytes(const lbm_stefan_params *p, int64_t nsteps,
                          int64_t interval, size_t *bytes) {
  const std::string e = validate_params(p);
  if (!e.empty()) return fail(nullptr, LBM_STEFAN_EINVAL, e);
  if (nsteps < 1 || interval < 1 || !bytes)
    return fail(nullptr, LBM_STEFAN_EINVAL, "nsteps and interval must be >= 1");
  const int64_t I = std::min(interval, nsteps);
  const int64_t K = (nsteps + I - 1) / I;
  // checkpoints 0..K, then two segments' recomputed states (the reverse
  // sweep of one segment overlaps the recomputation of the next)
  *bytes = (size_t)(K + 1 + 2 * I) * align256(state_bytes(*p));
  return LBM_STEFAN_OK;
}

int lbm_stefan_forward_tape(lbm_stefan_t *h, int64_t nsteps, int64_t interval,
                            void *tape, size_t bytes) {
  if (int rc = check_adj(h)) return rc;
  size_t need;
  if (lbm_stefan_tape_bytes(&h->p, nsteps, interval, &need))
    return fail(h, LBM_STEFAN_EINVAL, lbm_stefan_last_error(nullptr));
  if (!tape || bytes < need || (uintptr_t)tape % 256)
    return fail(h, LBM_STEFAN_EINVAL, "tape too small or misaligned");
  DeviceGuard g(h->device);
  const int64_t I = std::min(interval, nsteps);
  const int64_t K = (nsteps + I - 1) / I;
  const size_t sb = state_bytes(h->p), slot = align256(sb);
  char *t = (char *)tape;
  HIPCHK(h, hipMemcpyAsync(t, h->buf[h->cur], sb, hipMemcpyDeviceToDevice,
                           h->stream));
  // segment k starts from checkpoint k - 1 and its last step writes
  // checkpoint k directly; the steps between use the handle's two buffers
  for (int64_t k = 1; k <= K; ++k) {
    const int64_t n = std::min(I, nsteps - (k - 1) * I);
    const void *src = t + (k - 1) * slot;
    for (int64_t s = 0; s < n; ++s) {
      void *dst = s == n - 1 ? (void *)(t + k * slot) : h->buf[s & 1];
      HIPCHK(h, launch_step(h, src, dst));
      h->steps++;
      src = dst;
    }
  }
  h->cur = 0;
  HIPCHK(h, hipMemcpyAsync(h->buf[0], t + K * slot, sb,
                           hipMemcpyDeviceToDevice, h->stream));
  h->tape = tape;
  h->tape_steps = nsteps;
  h->tape_interval = I;
  return LBM_STEFAN_OK;
}

int lbm_stefan_backward_tape(lbm_stefan_t *h, const double *dL_dfront,
                             void *tape, size_t bytes, double *g_wall,
                             double *g_ste, double *g_delta) {
  if (int rc = check_adj(h)) return rc;
  if (!tape || tape != h->tape || !dL_dfront)
    return fail(h, LBM_STEFAN_EINVAL,
                "tape is not the one of the last lbm_stefan_forward_tape");
  const int64_t N = h->tape_steps, I = h->tape_interval;
  const int64_t K = (N + I - 1) / I;
  const size_t sb = state_bytes(h->p), slot = align256(sb);
  if (bytes < (size_t)(K + 1 + 2 * I) * slot)
    return fail(h, LBM_STEFAN_EINVAL, "tape too small");
  DeviceGuard g(h->device);
  HIPCHK(h, handle_side(h));
  const AdjLayout L = adj_layout(&h->p);
  double *ab[2] = {(double *)(h->adj + L.abar0), (double *)(h->adj + L.abar1)};
  char *t = (char *)tape;
  char *seg[2] = {t + (K + 1) * slot, t + (K + 1 + I) * slot};
  HIPCHK(h, reset_async(h));
  HIPCHK(h, front_vjp_async(h, t + K * slot, dL_dfront, ab[0]));
  // Segment k's states are recomputed from checkpoint k into seg[k & 1] on
  // the handle's second stream, while this stream runs the reverse sweep
  // of segment k + 1 from seg[(k + 1) & 1]: both are chains of small,
  // latency-bound launches, so they overlap.  Event `join` (recorded on the
  // second stream) marks a segment recomputed, event `fork` (recorded
  // here) a sweep done, after which its buffer may be overwritten.
  auto states_of = [&](int64_t k) -> const void * {
    return (const void *)(t + k * slot);
  };
  // (a tape of every state, interval 1, has nothing to recompute: no
  // second stream then)
  const bool overlap = I > 1;
  auto recompute = [&](int64_t k) -> hipError_t {
    const int64_t n = std::min(I, N - k * I);
    char *sg = seg[k & 1];
    hipError_t e = hipStreamWaitEvent(h->side, h->fork, 0);
    for (int64_t j = 1; j < n && e == hipSuccess; ++j)
      e = launch_step(h, j == 1 ? states_of(k) : sg + (j - 1) * slot,
                      sg + j * slot, h->side);
    if (e == hipSuccess) e = hipEventRecord(h->join, h->side);
    return e;
  };
  if (overlap) {
    HIPCHK(h, hipEventRecord(h->fork, h->stream));
    HIPCHK(h, recompute(K - 1));
  }
  // reverse steps N-1 .. 0: the last one node-local only (its Omega'bar is
  // the front seed), then gather-of-(n+1) fused with local-of-n, then the
  // final gather; qbar/Tbar alternate between two buffers
  int c = -1;
  for (int64_t k = K - 1; k >= 0; --k) {
    const int64_t n = std::min(I, N - k * I);
    // states of segment k: the checkpoint itself, then recomputed ones
    auto state = [&](int64_t j) -> const void * {
      return j == 0 ? states_of(k) : (const void *)(seg[k & 1] + j * slot);
    };
    if (overlap) {
      HIPCHK(h, hipStreamWaitEvent(h->stream, h->join, 0));
      if (k >= 1) HIPCHK(h, recompute(k - 1));
    }
    for (int64_t j = n - 1; j >= 0; --j) {
      if (c < 0) {
        HIPCHK(h, local_async(h, state(j), ab[0], 0));
        c = 0;
      } else {
        HIPCHK(h, fused_async(h, state(j), c));
        c ^= 1;
      }
    }
    if (overlap) HIPCHK(h, hipEventRecord(h->fork, h->stream));
  }
  HIPCHK(h, pull_async(h, c, ab[1]));
  HIPCHK(h, init_term_async(h, ab[1]));
  return read_gradients(h, g_wall, g_ste, g_delta);
}

int lbm_stefan_adjoint_buffers(lbm_stefan_t *h, double **abar0,
                               double **abar1) {
  if (int rc = check_adj(h)) return rc;
  const AdjLayout L = adj_layout(&h->p);
  if (abar0) *abar0 = (double *)(h->adj + L.abar0);
  if (abar1) *abar1 = (double *)(h->adj + L.abar1);
  return LBM_STEFAN_OK;
}

}  // extern "C"
