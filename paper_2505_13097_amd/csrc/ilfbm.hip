// ilfbm.hip -- the implicit liquid fraction based method (ILFBM, Section
// 3.3, Algorithm 1) on gfx950, the inner-loop scheme the paper compares
// IREBM with.
//
// The state is the post-collision population planes Omega0 (collision
// without source, as for the other schemes) and the liquid fraction plane
// l.  One step runs the inner loop of Algorithm 1: iteration k pulls
//   f_i^(k)(x) = Omega0_i(x - e_i) + (w_i/Ste)(l - l^(k-1))(x - e_i)
// (the collision with source of the upstream node, then streaming),
// closes the unknown populations (Section 4.2 on the streamed populations,
// Dirichlet target T_D), and forms H^(k) = M0(f^(k)) + l^(k-1)/Ste and
// l^(k) = clamp(Ste (H^(k) - T_m), 0, 1).  The source term reaches across
// nodes, so each iteration is one pass over the lattice: one kernel
// launch, which also writes the collision of f^(k) (the next state, in
// case k is the last iteration) and per-block max |l^(k) - l^(k-1)| and
// boundary fluxes.  A one-block check kernel reduces them in a fixed
// order and sets a device flag once max |l^(k) - l^(k-1)| <= tol; every
// later launch of the step sees the flag and returns, so the buffers keep
// the last iteration's results.  The host reads the flag after every few
// launches.  Tolerance and cap: the params' newton_tol and newton_max_it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "host_util.hpp"
#include "kernels.hpp"
#include "lbm_stefan.h"
#include "lbm_stefan_internal.hpp"

using namespace irebm;

namespace {

constexpr int kBlock = 256;      // threads per block of the inner kernel
constexpr int kBurst = 4;        // launches between two host checks

// device control block of one step's inner loop
struct IlfCtrl {
  int32_t done, kfinal;
  double dl, flux_in, flux_out;
};

struct IlfArgs {
  StepArgs A;            // lattice; A.src = Omega0, A.dst = next state
  const double *l;       // liquid fraction of the state
  const double *lprev;   // l^(k-1)
  double *lout;          // l^(k)
  double *pend;          // per block: max |dl|, flux in, flux out
  IlfCtrl *ctrl;
  double ste;
};

// Omega^(k)_i at node k: the collision with source of Algorithm 1
template <int Q, typename S>
__device__ __forceinline__ double omega_k(const IlfArgs &G, int i,
                                          int64_t node) {
  const S *src = (const S *)G.A.src;
  return (double)src[i * G.A.plane + node] +
         wt<Q>(i) * G.A.inv_ste * (G.l[node] - G.lprev[node]);
}

// lattice node of the pull source x - e_i (wrapped on periodic axes; the
// caller knows from the masks that it is one)
template <int Q>
__device__ __forceinline__ int64_t source_node(const StepArgs &A, int x, int y,
                                               int i) {
  int sx = x - cx<Q>(i), sy = y - cy<Q>(i);
  if (sx < 0) sx += A.nx;
  if (sx >= A.nx) sx -= A.nx;
  if (sy < 0) sy += A.ny;
  if (sy >= A.ny) sy -= A.ny;
  return (int64_t)sy * A.nx + sx;
}

// inner iteration at node k: writes l^(k) and the collision of f^(k), adds
// |l^(k) - l^(k-1)| (max), the closure inflow and the outflow
template <int Q, typename S>
__device__ __forceinline__ void ilfbm_node(const IlfArgs &G, int64_t k,
                                           double &dl, double &fin,
                                           double &fout) {
  const StepArgs &A = G.A;
  {
    const int x = (int)(k % A.nx), y = (int)(k / A.nx);
    uint32_t known, out;
    node_masks<Q>(A, x, y, known, out);
    double om[Q], q[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) om[j] = omega_k<Q, S>(G, j, k);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      q[i] = (known >> i & 1u) ? omega_k<Q, S>(G, i, source_node<Q>(A, x, y, i))
                               : 0.0;
    if (known != (1u << Q) - 1u) {
      double mirror = 0.0;
      int mx, my;
      if (neumann_mirror<Q>(A, x, y, mx, my)) {
        // M0 of the populations streamed into the mirror node; every
        // source is a lattice node (no bounce-back beside Neumann walls)
#pragma unroll
        for (int i = 0; i < Q; ++i)
          mirror += omega_k<Q, S>(G, i, source_node<Q>(A, mx, my, i));
      }
      fin += close_node<Q, SCHEME_ILFBM, true>(A, x, y, 0.0, om, q, known,
                                                mirror);
    }
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if (out >> i & 1u) fout += om[i];
    double m0 = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) m0 += q[i];
    const double H = m0 + G.lprev[k] * A.inv_ste;
    double ln = G.ste * (H - A.tm);
    ln = ln < 0.0 ? 0.0 : (ln > 1.0 ? 1.0 : ln);
    G.lout[k] = ln;
    dl = fmax(dl, fabs(ln - G.lprev[k]));
    // the collision of f^(k): the next state if k is the last iteration
    S *dst = (S *)A.dst;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      dst[i * A.plane + k] = (S)(A.a * q[i] + A.wtau[wclass<Q>(i)] * m0);
  }
}

template <int Q, typename S>
__global__ __launch_bounds__(kBlock) void ilfbm_iter_kernel(IlfArgs G) {
  if (G.ctrl->done) return;          // an earlier iteration converged
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double dl = 0.0, fin = 0.0, fout = 0.0;
  if (k < G.A.plane) ilfbm_node<Q, S>(G, k, dl, fin, fout);
  __shared__ double s_dl[kBlock / 64];
  dl = wave_max(dl);
  if ((threadIdx.x & 63) == 0) s_dl[threadIdx.x >> 6] = dl;
  const double bfin = block_sum_256(fin);
  const double bfout = block_sum_256(fout);
  if (threadIdx.x == 0) {
    double m = s_dl[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, s_dl[w]);
    G.pend[3 * blockIdx.x] = m;
    G.pend[3 * blockIdx.x + 1] = bfin;
    G.pend[3 * blockIdx.x + 2] = bfout;
  }
}

// iteration k's convergence test: max and sums over the blocks in a fixed
// order; sets done once max |dl| <= tol
__global__ __launch_bounds__(256) void ilfbm_check_kernel(const double *pend,
                                                          int64_t nblocks,
                                                          IlfCtrl *ctrl,
                                                          int32_t k,
                                                          double tol) {
  if (ctrl->done) return;
  double m = 0.0, fin = 0.0, fout = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += 256) {
    m = fmax(m, pend[3 * b]);
    fin += pend[3 * b + 1];
    fout += pend[3 * b + 2];
  }
  __shared__ double s_m[4];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  const double sfin = block_sum_256(fin);
  const double sfout = block_sum_256(fout);
  if (threadIdx.x == 0) {
    m = fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
    ctrl->dl = m;
    ctrl->flux_in = sfin;
    ctrl->flux_out = sfout;
    ctrl->kfinal = k;
    if (m <= tol) ctrl->done = 1;
  }
}

// Small lattices (at most kResidentNodes nodes): one workgroup runs
// `nsteps` whole steps in one launch, block barriers in place of launches
// and host reads.  Node updates and convergence decisions are those of
// the multi-launch path (same ilfbm_node, exact max), so the states are
// the same; only the flux sums are reduced in another order.  L[0] is the
// state's l plane, L[1] and L[2] the inner-loop planes; planes and buffers
// rotate in registers, and the final assignment and statistics are
// written to `res` for the host.
constexpr int kResident = 1024;         // threads of the resident block
constexpr int64_t kResidentNodes = 16384;

struct IlfResident {
  IlfArgs G;            // lattice, ste; l/lprev/lout/pend/ctrl unused
  void *buf[2];
  double *L[3];
  int32_t cur, nsteps, cap;
  double tol;
  double *res;          // out: cur, L roles (3), max_it, capped steps,
                        // max residual, flux in, flux out
};

// Block reductions with one barrier each: consecutive reductions use
// alternate halves of sh (`r` counts them), and the barrier of reduction
// r + 1 separates the reads of reduction r from the writes of r + 2.
// Every thread calls them in the same order.
__device__ __forceinline__ double block_max_1024(double v, double *sh,
                                                 int &r) {
  double *b = sh + (r++ & 1) * (kResident / 64);
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = b[0];
  for (int w = 1; w < kResident / 64; ++w) m = fmax(m, b[w]);
  return m;
}

__device__ __forceinline__ double block_sum_1024(double v, double *sh,
                                                 int &r) {
  double *b = sh + (r++ & 1) * (kResident / 64);
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = b[0];
  for (int w = 1; w < kResident / 64; ++w) m += b[w];
  return m;
}

template <int Q, typename S>
__global__ __launch_bounds__(kResident) void ilfbm_resident_kernel(
    IlfResident R) {
  __shared__ double sh[2 * (kResident / 64)];
  int red = 0;
  IlfArgs G = R.G;
  int cur = R.cur;
  int li = 0, la = 1, lb = 2;       // state, and the two inner planes
  int max_it = 0, capped = 0;
  double max_res = 0.0, fin_tot = 0.0, fout_tot = 0.0;
  const int64_t n = G.A.plane;
  for (int s = 0; s < R.nsteps; ++s) {
    G.A.src = R.buf[cur];
    G.A.dst = R.buf[cur ^ 1];
    G.l = R.L[li];
    int k = 0;
    bool done = false;
    double dl = 0.0, a = 0.0, b = 0.0;
    while (k < R.cap && !done) {
      ++k;
      G.lprev = k == 1 ? R.L[li] : R.L[(k - 1) & 1 ? la : lb];
      G.lout = R.L[k & 1 ? la : lb];
      double d = 0.0;
      a = 0.0;
      b = 0.0;
      for (int64_t j = threadIdx.x; j < n; j += kResident)
        ilfbm_node<Q, S>(G, j, d, a, b);
      // the barrier inside the reduction also orders this iteration's
      // writes before the next iteration's reads
      dl = block_max_1024(d, sh, red);
      done = dl <= R.tol;
    }
    // fluxes of the last iteration
    const double fin = block_sum_1024(a, sh, red);
    const double fout = block_sum_1024(b, sh, red);
    // l^(k) becomes the state's plane
    const int lk = k & 1 ? la : lb;
    if (lk == la) {
      la = li;
    } else {
      lb = li;
    }
    li = lk;
    cur ^= 1;
    max_it = max(max_it, k);
    if (!done) {
      capped++;
      max_res = fmax(max_res, dl);
    }
    fin_tot += fin;
    fout_tot += fout;
  }
  if (threadIdx.x == 0) {
    R.res[0] = cur;
    R.res[1] = li;
    R.res[2] = la;
    R.res[3] = lb;
    R.res[4] = max_it;
    R.res[5] = capped;
    R.res[6] = max_res;
    R.res[7] = fin_tot;
    R.res[8] = fout_tot;
  }
}

__global__ void ilfbm_reset_kernel(IlfCtrl *ctrl) {
  ctrl->done = 0;
  ctrl->kfinal = 0;
  ctrl->dl = 0.0;
  ctrl->flux_in = 0.0;
  ctrl->flux_out = 0.0;
}

int64_t iter_blocks(const lbm_stefan_params *p) {
  return (p->nx * p->ny + kBlock - 1) / kBlock;
}

}  // namespace

size_t irebm::ilfbm_bytes(const lbm_stefan_params *p) {
  if (p->scheme != LBM_SCHEME_ILFBM) return 0;
  const int64_t n = p->nx * p->ny;
  return 3 * align256((size_t)n * 8) + align256((size_t)iter_blocks(p) * 24) +
         256;
}

void irebm::ilfbm_attach(lbm_stefan_t *h, char *base) {
  const int64_t n = h->p.nx * h->p.ny;
  const size_t plane = align256((size_t)n * 8);
  h->lf = (double *)base;
  h->lscr[0] = (double *)(base + plane);
  h->lscr[1] = (double *)(base + 2 * plane);
  h->pend = (double *)(base + 3 * plane);
  h->ctrl = base + 3 * plane + align256((size_t)iter_blocks(&h->p) * 24);
  ilfbm_reset_stats(h);
}

void irebm::ilfbm_reset_stats(lbm_stefan_t *h) {
  h->ilf_max_it = 0;
  h->ilf_nonconv = 0;
  h->ilf_max_res = 0.0;
  h->ilf_fin = 0.0;
  h->ilf_fout = 0.0;
}

namespace {

// nsteps steps of a small lattice in launches of the resident kernel
hipError_t ilfbm_advance_resident(lbm_stefan_t *h, int64_t nsteps) {
  const lbm_stefan_params &p = h->p;
  constexpr int64_t kChunk = 2048;    // steps per launch
  IlfResident R;
  fill_step_args(h, &R.G.A);
  R.G.ste = p.ste;
  R.G.pend = nullptr;
  R.G.ctrl = nullptr;
  R.buf[0] = h->buf[0];
  R.buf[1] = h->buf[1];
  R.cap = p.newton_max_it;
  R.tol = p.newton_tol;
  R.res = h->pend;                    // >= 24 bytes: reuse the pending area
  for (int64_t left = nsteps; left > 0;) {
    const int32_t chunk = (int32_t)std::min(left, kChunk);
    double *Lp[3] = {h->lf, h->lscr[0], h->lscr[1]};
    for (int j = 0; j < 3; ++j) R.L[j] = Lp[j];
    R.cur = h->cur;
    R.nsteps = chunk;
    hipError_t e = dispatch_qs(p.q, p.storage, [&](auto qt, auto tt) {
      QS_TYPES(qt, tt);
      ilfbm_resident_kernel<Q, S><<<1, kResident, 0, h->stream>>>(R);
      return hipGetLastError();
    });
    double res[9];
    if (e == hipSuccess)
      e = hipMemcpyAsync(res, h->pend, sizeof(res), hipMemcpyDeviceToHost,
                         h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    h->cur = (int)res[0];
    h->lf = Lp[(int)res[1]];
    h->lscr[0] = Lp[(int)res[2]];
    h->lscr[1] = Lp[(int)res[3]];
    h->ilf_max_it = std::max(h->ilf_max_it, (int32_t)res[4]);
    h->ilf_nonconv += (int64_t)res[5];
    if (res[5] > 0) h->ilf_max_res = std::max(h->ilf_max_res, res[6]);
    h->ilf_fin += res[7];
    h->ilf_fout += res[8];
    h->steps += chunk;
    left -= chunk;
  }
  return hipSuccess;
}

}  // namespace

hipError_t irebm::ilfbm_advance(lbm_stefan_t *h, int64_t nsteps) {
  const lbm_stefan_params &p = h->p;
  if (p.nx * p.ny <= kResidentNodes) return ilfbm_advance_resident(h, nsteps);
  const int64_t nb = iter_blocks(&p);
  IlfCtrl *ctrl = (IlfCtrl *)h->ctrl;
  IlfArgs G;
  fill_step_args(h, &G.A);
  G.pend = h->pend;
  G.ctrl = ctrl;
  G.ste = p.ste;
  const int cap = p.newton_max_it;
  for (int64_t s = 0; s < nsteps; ++s) {
    G.A.src = h->buf[h->cur];
    G.A.dst = h->buf[h->cur ^ 1];
    G.l = h->lf;
    ilfbm_reset_kernel<<<1, 1, 0, h->stream>>>(ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    IlfCtrl hc{};
    int k = 0;
    while (k < cap) {
      const int burst = std::min(kBurst, cap - k);
      for (int b = 0; b < burst; ++b) {
        ++k;
        G.lprev = k == 1 ? h->lf : h->lscr[(k - 1) & 1];
        G.lout = h->lscr[k & 1];
        e = dispatch_qs(p.q, p.storage, [&](auto qt, auto tt) {
          QS_TYPES(qt, tt);
          ilfbm_iter_kernel<Q, S><<<(unsigned)nb, kBlock, 0, h->stream>>>(G);
          return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        ilfbm_check_kernel<<<1, 256, 0, h->stream>>>(h->pend, nb, ctrl, k,
                                                     p.newton_tol);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
      e = hipMemcpyAsync(&hc, ctrl, sizeof(hc), hipMemcpyDeviceToHost,
                         h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) return e;
      if (hc.done) break;
    }
    // the last iteration run: kfinal (converged) or the cap
    const int kf = hc.done ? hc.kfinal : k;
    std::swap(h->lf, h->lscr[kf & 1]);
    h->cur ^= 1;
    h->steps++;
    h->ilf_max_it = std::max(h->ilf_max_it, kf);
    if (!hc.done) {
      h->ilf_nonconv++;
      h->ilf_max_res = std::max(h->ilf_max_res, hc.dl);
    }
    h->ilf_fin += hc.flux_in;
    h->ilf_fout += hc.flux_out;
  }
  return hipSuccess;
}
