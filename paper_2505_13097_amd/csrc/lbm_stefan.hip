// lbm_stefan.hip -- gfx950 kernels and the C ABI of the IREBM step
// (Luddens, Lothode, Danaila, arXiv 2505.13097, Algorithm 3 with the
// boundary closures of Section 4.2).  See include/lbm_stefan.h.
//
// The kernels are in kernels.hpp; this unit holds the host side of the
// single-lattice handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>

#include "host_util.hpp"
#include "kernels.hpp"
#include "lbm_stefan.h"
#include "lbm_stefan_internal.hpp"

using namespace irebm;


// =====================================================================
// host side

namespace {

thread_local std::string g_err = "no error";


}  // namespace

std::string irebm::validate_params(const lbm_stefan_params *p) {
  if (!p) return "params is NULL";
  const bool lat = (p->dim == 1 && p->q == 3) ||
                   (p->dim == 2 && (p->q == 5 || p->q == 9)) ||
                   (p->dim == 3 && (p->q == 7 || p->q == 19));
  if (!lat) return "lattice must be D1Q3, D2Q5, D2Q9, D3Q7 or D3Q19";
  if (p->nx < 3) return "nx must be >= 3";
  if (p->dim == 1 && p->ny != 1) return "ny must be 1 for a 1D lattice";
  if (p->dim >= 2 && p->ny < 3) return "ny must be >= 3 for a 2D or 3D lattice";
  if (p->dim == 3 && p->nz < 3) return "nz must be >= 3 for a 3D lattice";
  if (p->nx > INT32_MAX || p->ny > INT32_MAX ||
      (p->dim == 3 && p->nz > INT32_MAX))
    return "nx, ny, nz too large";
  if (p->nx * p->ny * (p->dim == 3 ? p->nz : 1) > ((int64_t)1 << 31) - 1)
    return "the node count must be below 2^31";
  if (p->dim == 3) {
    if (p->scheme == LBM_SCHEME_ILFBM)
      return "3D lattices run the IREBM and EEBM schemes";
    if (p->flags & LBM_FLAG_ADJOINT)
      return "the reverse mode is for 1D and 2D lattices";
    for (int k = 0; k < 4; ++k)
      if (p->wall_profile[k])
        return "3D lattices take constant wall temperatures (no profiles)";
    for (int k = 0; k < 2; ++k) {
      if (p->bc_z[k] < LBM_BC_DIRICHLET || p->bc_z[k] > LBM_BC_NEUMANN)
        return "unknown boundary kind";
      if (!std::isfinite(p->wall_T_z[k])) return "wall_T must be finite";
    }
    if ((p->bc_z[0] == LBM_BC_PERIODIC) != (p->bc_z[1] == LBM_BC_PERIODIC))
      return "z walls: both or neither periodic";
  }
  if (p->storage != LBM_STORE_F64 && p->storage != LBM_STORE_F32)
    return "storage must be LBM_STORE_F64 or LBM_STORE_F32";
  if (p->newton_mode != LBM_NEWTON_SAFEGUARDED &&
      p->newton_mode != LBM_NEWTON_PLAIN)
    return "unknown newton_mode";
  if (p->scheme != LBM_SCHEME_IREBM && p->scheme != LBM_SCHEME_EEBM &&
      p->scheme != LBM_SCHEME_ILFBM)
    return "unknown scheme";
  if (p->scheme != LBM_SCHEME_IREBM && (p->flags & LBM_FLAG_ADJOINT))
    return "the reverse mode is for the IREBM scheme only";
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return "tau must be > 1/2";
  if (!(p->ste > 0.0) || !std::isfinite(p->ste)) return "ste must be > 0";
  if (!(p->delta > 0.0) || !std::isfinite(p->delta))
    return "delta must be > 0";
  if (!std::isfinite(p->t_m)) return "t_m must be finite";
  if (!(p->newton_tol > 0.0)) return "newton_tol must be > 0";
  if (p->newton_max_it < 1 || p->newton_max_it > 1000)
    return "newton_max_it must be in 1..1000";
  if (!(p->dx >= 0.0) || !std::isfinite(p->dx)) return "dx must be >= 0";
  bool neu = false, bb = false;
  for (int k = 0; k < 4; ++k) {
    if (p->dim == 1 && k >= 2) break;
    if (p->bc[k] < LBM_BC_DIRICHLET || p->bc[k] > LBM_BC_NEUMANN)
      return "unknown boundary kind";
    if (!std::isfinite(p->wall_T[k])) return "wall_T must be finite";
    neu |= p->bc[k] == LBM_BC_NEUMANN;
    bb |= p->bc[k] == LBM_BC_BOUNCEBACK;
  }
  for (int k = 0; p->dim == 3 && k < 2; ++k) {
    neu |= p->bc_z[k] == LBM_BC_NEUMANN;
    bb |= p->bc_z[k] == LBM_BC_BOUNCEBACK;
  }
  if (neu && bb) return "Neumann and bounce-back walls do not mix";
  if (neu && (p->flags & LBM_FLAG_ADJOINT))
    return "the reverse mode has no Neumann closure";
  if ((p->bc[0] == LBM_BC_PERIODIC) != (p->bc[1] == LBM_BC_PERIODIC))
    return "x walls: both or neither periodic";
  if (p->dim == 2 &&
      (p->bc[2] == LBM_BC_PERIODIC) != (p->bc[3] == LBM_BC_PERIODIC))
    return "y walls: both or neither periodic";
  int nv;
  if (p->dim == 3) variants3(&nv);
  else variants(p->q, &nv);
  if (p->variant < -1 || p->variant >= nv) return "unknown kernel variant";
  return "";
}

irebm::Layout irebm::layout_for(const lbm_stefan_params *p) {
  Layout L;
  const int64_t n = nodes_of(*p);
  const size_t s = p->storage == LBM_STORE_F64 ? 8 : 4;
  L.buf_bytes = align256((size_t)p->q * n * s);
  int nv;
  int64_t mt = 0;
  int64_t mf = 0;
  if (p->dim == 3) {
    const Variant3 *v3 = variants3(&nv);
    for (int i = 0; i < nv; ++i) {
      mt = std::max(mt, items3_for(v3[i], p->nx, p->ny, p->nz));
      if (v3[i].split && p->nx > 2 * kFront3Columns) {
        // quiet-pass items, then the front strip's
        const int64_t nq = items3_for(v3[i], p->nx - kFront3Columns, p->ny,
                                      p->nz);
        mf = std::max(mf, nq);
        mt = std::max(mt, nq + items3_for(v3[kFront3Variant], kFront3Columns,
                                          p->ny, p->nz));
      }
    }
  } else {
    const Variant *v = variants(p->q, &nv);
    for (int i = 0; i < nv; ++i)
      mt = std::max(mt, items_for(v[i], p->nx, p->ny));
  }
  L.max_items = mt;
  L.n_partials = (n + kEnergyChunk - 1) / kEnergyChunk;
  size_t off = 0;
  L.off_buf[0] = off;
  off += L.buf_bytes;
  L.off_buf[1] = off;
  off += L.buf_bytes;
  const int64_t plen = std::max(p->nx, p->ny);
  for (int k = 0; k < 4; ++k) {
    L.off_prof[k] = off;
    off += align256((size_t)plen * 8);
  }
  L.off_slots = off;
  off += align256((size_t)mt * sizeof(StatSlot));
  L.off_flags = off;
  off += align256((size_t)mf * sizeof(int32_t));
  L.off_partials = off;
  off += align256((size_t)L.n_partials * 8);
  L.off_small = off;
  off += align256((size_t)(std::max<int64_t>(rows_of(*p), 16) + 16) * 8);
  L.adjoint = (p->flags & LBM_FLAG_ADJOINT) != 0;
  L.off_adj = off;
  if (L.adjoint) off += adjoint_bytes(p, mt);
  L.off_lf = off;
  off += ilfbm_bytes(p);
  L.total = off;
  return L;
}

int irebm::fail(lbm_stefan_t *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  else g_err = msg;
  return code;
}

void irebm::set_global_error(const std::string &msg) { g_err = msg; }


void irebm::fill_args(const lbm_stefan_params &p, double *const prof[4],
                      StepArgs *A) {
  std::memset(A, 0, sizeof(*A));
  A->nx = (int32_t)p.nx;
  A->ny = (int32_t)p.ny;
  A->x_lim = A->x_cnt = (int32_t)p.nx;
  A->plane = p.nx * p.ny;
  A->periodic_x = p.bc[0] == LBM_BC_PERIODIC;
  A->periodic_y = p.dim == 2 && p.bc[2] == LBM_BC_PERIODIC;
  A->scheme = p.scheme;
  A->a = 1.0 - 1.0 / p.tau;
  A->inv_tau = 1.0 / p.tau;
  for (int i = 0; i < p.q; ++i) {
    const double w = p.q == 3 ? wt<3>(i) : (p.q == 5 ? wt<5>(i) : wt<9>(i));
    A->wtau[i] = w / p.tau;
    A->wste[i] = w / p.ste;
  }
  A->inv_ste = 1.0 / p.ste;
  A->tm = p.t_m;
  A->inv_delta = 1.0 / p.delta;
  A->tol = p.newton_tol;
  A->max_it = p.newton_max_it;
  A->neu = 0;
  for (int k = 0; k < 4; ++k) {
    A->bc[k] = (p.dim == 1 && k >= 2) ? BC_PERIODIC : p.bc[k];
    if (A->bc[k] == BC_NEUMANN) A->neu |= 1 << k;
    A->wall_T[k] = p.wall_T[k];
    A->prof[k] = prof ? prof[k] : nullptr;
  }
}

void irebm::fill_args3(const lbm_stefan_params &p, StepArgs3 *A) {
  std::memset(A, 0, sizeof(*A));
  A->nx = (int32_t)p.nx;
  A->ny = (int32_t)p.ny;
  A->nz = (int32_t)p.nz;
  A->plane = nodes_of(p);
  const int32_t bc[6] = {p.bc[0], p.bc[1], p.bc[2], p.bc[3], p.bc_z[0],
                         p.bc_z[1]};
  const double wT[6] = {p.wall_T[0], p.wall_T[1], p.wall_T[2],
                        p.wall_T[3], p.wall_T_z[0], p.wall_T_z[1]};
  for (int k = 0; k < 6; ++k) {
    A->bc[k] = bc[k];
    A->wall_T[k] = wT[k];
    if (bc[k] == BC_NEUMANN) A->neu |= 1 << k;
  }
  for (int a = 0; a < 3; ++a) A->periodic[a] = bc[2 * a] == BC_PERIODIC;
  A->a = 1.0 - 1.0 / p.tau;
  A->inv_tau = 1.0 / p.tau;
  const int rep[3] = {0, 1, 7};  // one direction of each weight class
  for (int c = 0; c < 3; ++c) {
    const double w = p.q == 7 ? wt3<7>(rep[c]) : wt3<19>(rep[c]);
    A->wtau[c] = w / p.tau;
    A->wste[c] = w / p.ste;
  }
  A->inv_ste = 1.0 / p.ste;
  A->tm = p.t_m;
  A->inv_delta = 1.0 / p.delta;
  A->tol = p.newton_tol;
  A->max_it = p.newton_max_it;
  A->x_off = 0;
  A->x_lim = (int32_t)p.nx;
  auto closes_in_rows = [](int32_t b) {
    return b == BC_DIRICHLET || b == BC_BOUNCEBACK;
  };
  A->xrow = p.nx >= 3 && closes_in_rows(bc[0]) && closes_in_rows(bc[1]) &&
            !(p.flags & LBM_FLAG_CHECKED_FACES);
}

void irebm::fill_step_args(const lbm_stefan_t *h, StepArgs *A) {
  double *prof[4];
  for (int k = 0; k < 4; ++k) prof[k] = h->has_prof[k] ? h->prof[k] : nullptr;
  fill_args(h->p, prof, A);
  A->slots = h->slots;
}

bool irebm::two_step_variant(const lbm_stefan_t *h) {
  if (h->p.dim == 3) return false;
  int nv;
  return variants(h->p.q, &nv)[h->variant].tb != 0 && !has_neumann(h->p);
}

hipError_t irebm::launch_step2(const lbm_stefan_t *h, const void *src,
                               void *dst, bool two) {
  StepArgs A;
  fill_step_args(h, &A);
  A.src = src;
  A.dst = dst;
  int nv;
  const Variant &v = variants(h->p.q, &nv)[h->variant];
  return step2_launch(mode_of(h->p), h->p.q, h->p.storage, A, v, two,
                      h->stream);
}

namespace {

// the 3D split step applies: a split variant, IREBM without Neumann faces,
// a Dirichlet x = 0 face off phi's lower plateau, and more columns than
// twice the front strip
bool split3_applies(const lbm_stefan_t *h, const Variant3 &v) {
  const lbm_stefan_params &p = h->p;
  return v.split && p.scheme == LBM_SCHEME_IREBM && !has_neumann(p) &&
         p.bc[0] == LBM_BC_DIRICHLET &&
         p.wall_T[0] >= p.t_m - 20.0 * p.delta &&
         p.nx > 2 * kFront3Columns;
}

// one split step (see step3_kernel): the front strip on the side stream
// beside the quiet pass, then the full pass over flagged items
hipError_t split3_step(lbm_stefan_t *h, const StepArgs3 &A,
                       const Variant3 &v, int mode) {
  hipError_t e = irebm::handle_side(h);
  if (e != hipSuccess) return e;
  int nv;
  const Variant3 &fv = variants3(&nv)[kFront3Variant];
  StepArgs3 Aq = A, Af = A;
  Aq.x_off = kFront3Columns;
  Aq.flags = h->flags;
  StepArgs3 T = Aq;
  set_tiling3(&T, v);
  if (h->flags_variant != h->variant) {
    e = zero_async(h->flags, (size_t)T.nitems * sizeof(int32_t), h->stream);
    if (e != hipSuccess) return e;
    h->flags_variant = h->variant;
  }
  Af.x_lim = kFront3Columns;
  Af.slots = A.slots + T.nitems;
  e = hipEventRecord(h->fork, h->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->fork, 0);
  if (e == hipSuccess)
    e = step3_launch(mode, h->p.q, h->p.storage, Af, fv, h->side, 0);
  if (e == hipSuccess) e = hipEventRecord(h->join, h->side);
  if (e == hipSuccess)
    e = step3_launch(mode, h->p.q, h->p.storage, Aq, v, h->stream, 1);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->join, 0);
  if (e == hipSuccess)
    e = step3_launch(mode, h->p.q, h->p.storage, Aq, v, h->stream, 2);
  return e;
}

}  // namespace

hipError_t irebm::handle_side(lbm_stefan_t *h) {
  hipError_t e = hipSuccess;
  if (!h->side) {
    e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(&h->join, hipEventDisableTiming);
  }
  return e;
}

hipError_t irebm::advance(lbm_stefan_t *h, int64_t nsteps) {
  if (h->p.scheme == LBM_SCHEME_ILFBM) return ilfbm_advance(h, nsteps);
  if (h->p.dim == 3) {
    StepArgs3 A;
    fill_args3(h->p, &A);
    A.slots = h->slots;
    int nv;
    const Variant3 &v = variants3(&nv)[h->variant];
    const int mode = mode_of(h->p);
    if (split3_applies(h, v)) {
      for (int64_t s = 0; s < nsteps; ++s) {
        A.src = h->buf[h->cur];
        A.dst = h->buf[h->cur ^ 1];
        const hipError_t e = split3_step(h, A, v, mode);
        if (e != hipSuccess) return e;
        h->cur ^= 1;
        h->steps++;
      }
      return hipSuccess;
    }
    // a Dirichlet x = 0 face is where the workloads heat: its tiles first
    A.front_first = h->p.bc[0] == LBM_BC_DIRICHLET;
    for (int64_t s = 0; s < nsteps; ++s) {
      A.src = h->buf[h->cur];
      A.dst = h->buf[h->cur ^ 1];
      const hipError_t e =
          step3_launch(mode, h->p.q, h->p.storage, A, v, h->stream);
      if (e != hipSuccess) return e;
      h->cur ^= 1;
      h->steps++;
    }
    return hipSuccess;
  }
  {
    int nv;
    if (variants(h->p.q, &nv)[h->variant].res && resident_ok(h->p)) {
      StepArgs A;
      fill_step_args(h, &A);
      const int mode = mode_of(h->p);
      while (nsteps > 0) {
        // bounded launches (a few ms each)
        const int32_t k = (int32_t)std::min<int64_t>(nsteps, 4096);
        A.src = h->buf[h->cur];
        A.dst = h->buf[h->cur ^ 1];
        const hipError_t e =
            resident_launch(mode, h->p.storage, A, k, h->stream);
        if (e != hipSuccess) return e;
        h->cur ^= k & 1;
        h->steps += k;
        nsteps -= k;
      }
      return hipSuccess;
    }
  }
  if (two_step_variant(h)) {
    for (; nsteps >= 2; nsteps -= 2) {
      const hipError_t e =
          launch_step2(h, h->buf[h->cur], h->buf[h->cur ^ 1], true);
      if (e != hipSuccess) return e;
      h->cur ^= 1;
      h->steps += 2;
    }
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    const hipError_t e = launch_step(h, h->buf[h->cur], h->buf[h->cur ^ 1]);
    if (e != hipSuccess) return e;
    h->cur ^= 1;
    h->steps++;
  }
  return hipSuccess;
}

hipError_t irebm::launch_step(const lbm_stefan_t *h, const void *src,
                              void *dst, hipStream_t stream) {
  StepArgs A;
  fill_step_args(h, &A);
  A.src = src;
  A.dst = dst;
  int nv;
  const Variant *vt = variants(h->p.q, &nv);
  // a single step under a two-step variant takes the default tiling, and
  // so does a step under the resident variant
  const Variant &v = vt[vt[h->variant].tb    ? kDefaultVariant2D
                        : vt[h->variant].res ? kDefaultVariant1D
                                             : h->variant];
  // a Dirichlet x = 0 wall is where the workloads heat: its tiles first
  A.front_first = h->p.bc[0] == LBM_BC_DIRICHLET;
  return step_launch(mode_of(h->p), h->p.q, h->p.storage, A, v,
                     v.rev && (h->steps & 1), stream ? stream : h->stream);
}

namespace {

// equilibrium initial state of a 3D lattice (A.dst)
hipError_t init3_async(int q, int storage, const StepArgs3 &A, bool eebm,
                       const double *T0, hipStream_t stream) {
  const unsigned blocks = blocks_for(A.plane, 256);
  const int e = eebm ? 1 : 0;
  if (q == 7) {
    if (storage == LBM_STORE_F32)
      init3_kernel<7, float><<<blocks, 256, 0, stream>>>(A, e, T0);
    else
      init3_kernel<7, double><<<blocks, 256, 0, stream>>>(A, e, T0);
  } else {
    if (storage == LBM_STORE_F32)
      init3_kernel<19, float><<<blocks, 256, 0, stream>>>(A, e, T0);
    else
      init3_kernel<19, double><<<blocks, 256, 0, stream>>>(A, e, T0);
  }
  return hipGetLastError();
}

// energy of the state `src` into h->small[kSmallEnergy] (device)
hipError_t handle_energy_async(const lbm_stefan_t *h, const void *src) {
  return irebm::energy_async(h->p, src, h->partials, h->small + kSmallEnergy,
                             h->stream, h->lf);
}

}  // namespace

hipError_t irebm::zero_stats_async(lbm_stefan_t *h) {
  ilfbm_reset_stats(h);
  return zero_async(h->slots, h->max_items * sizeof(StatSlot), h->stream);
}

int irebm::read_stats(lbm_stefan_t *h, lbm_stefan_stats *st) {
  stats_kernel<<<1, 256, 0, h->stream>>>(h->slots, h->max_items, h->small);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, handle_energy_async(h, h->buf[h->cur]));
  double hs[kSmallCount];
  HIPCHK(h, hipMemcpyAsync(hs, h->small, sizeof(hs), hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  st->steps = h->steps;
  st->max_newton_it = (int32_t)hs[0];
  st->reserved = 0;
  st->nonconverged = (int64_t)hs[1];
  st->max_residual = hs[2];
  st->flux_in = hs[3];
  st->flux_out = hs[4];
  if (h->p.scheme == LBM_SCHEME_ILFBM) {
    // the inner loop's statistics are kept on the host (per step)
    st->max_newton_it = h->ilf_max_it;
    st->nonconverged = h->ilf_nonconv;
    st->max_residual = h->ilf_max_res;
    st->flux_in = h->ilf_fin;
    st->flux_out = h->ilf_fout;
  }
  st->energy = hs[kSmallEnergy];
  if (!std::isfinite(st->energy))
    return fail(h, LBM_STEFAN_ENAN, "energy is not finite");
  return LBM_STEFAN_OK;
}

// ---------------------------------------------------------------------
// C ABI

extern "C" {

const char *lbm_stefan_version(void) {
  return "lbm_stefan 0.1 (gfx950, IREBM arXiv 2505.13097)";
}

const char *lbm_stefan_last_error(const lbm_stefan_t *h) {
  return h ? h->err.c_str() : g_err.c_str();
}

int lbm_stefan_workspace_bytes(const lbm_stefan_params *p, size_t *bytes) {
  const std::string e = validate_params(p);
  if (!e.empty()) return fail(nullptr, LBM_STEFAN_EINVAL, e);
  if (!bytes) return fail(nullptr, LBM_STEFAN_EINVAL, "bytes is NULL");
  *bytes = layout_for(p).total;
  return LBM_STEFAN_OK;
}

int lbm_stefan_init(const lbm_stefan_params *p, const double *T0,
                    void *workspace, size_t bytes, void *stream,
                    lbm_stefan_t **out) {
  const std::string e = validate_params(p);
  if (!e.empty()) return fail(nullptr, LBM_STEFAN_EINVAL, e);
  if (!out) return fail(nullptr, LBM_STEFAN_EINVAL, "out is NULL");
  *out = nullptr;
  const Layout L = layout_for(p);
  if (!workspace || bytes < L.total)
    return fail(nullptr, LBM_STEFAN_EINVAL, "workspace too small");
  if ((uintptr_t)workspace % 256)
    return fail(nullptr, LBM_STEFAN_EINVAL, "workspace not 256-byte aligned");
  lbm_stefan_t *h = new (std::nothrow) lbm_stefan_t();
  if (!h) return fail(nullptr, LBM_STEFAN_EDEVICE, "out of host memory");
  h->p = *p;
  if (h->p.dx == 0.0) h->p.dx = 1.0 / (double)(p->nx - 1);
  if (p->dim == 1) h->p.bc[2] = h->p.bc[3] = LBM_BC_PERIODIC;
  // default: the resident kernel for the small 1D lattices it takes
  h->variant = p->variant >= 0
                   ? p->variant
                   : (p->dim == 3 ? kDefaultVariant3D
                                  : (p->q == 3 ? (resident_ok(*p)
                                                      ? kResidentVariant1D
                                                      : kDefaultVariant1D)
                                               : kDefaultVariant2D));
  h->stream = (hipStream_t)stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, LBM_STEFAN_EDEVICE, "hipGetDevice failed");
  }
  char *ws = (char *)workspace;
  h->layout = L;
  h->ws = ws;
  h->buf[0] = ws + L.off_buf[0];
  h->buf[1] = ws + L.off_buf[1];
  h->cur = 0;
  h->slots = (StatSlot *)(ws + L.off_slots);
  h->max_items = L.max_items;
  h->flags = (int32_t *)(ws + L.off_flags);
  h->partials = (double *)(ws + L.off_partials);
  h->small = (double *)(ws + L.off_small);
  h->adj = ws + L.off_adj;
  const int64_t n = nodes_of(*p);
  for (int k = 0; k < 4; ++k) {
    h->prof[k] = (double *)(ws + L.off_prof[k]);
    h->has_prof[k] = p->wall_profile[k] != nullptr && !(p->dim == 1 && k >= 2);
  }
  auto bail = [&](int code) {
    g_err = h->err;
    delete h;
    return code;
  };
  for (int k = 0; k < 4; ++k)
    if (h->has_prof[k]) {
      const int64_t len = k < 2 ? p->ny : p->nx;
      for (int64_t j = 0; j < len; ++j)
        if (!std::isfinite(p->wall_profile[k][j]))
          return bail(fail(h, LBM_STEFAN_EINVAL, "wall profile not finite"));
      if (hipMemcpy(h->prof[k], p->wall_profile[k], len * 8,
                    hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(h, LBM_STEFAN_EDEVICE, "copy of a wall profile failed"));
    }
  // T0 is staged through the second population buffer (>= 12 n bytes)
  if (T0 && hipMemcpy(h->buf[1], T0, n * 8, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(h, LBM_STEFAN_EDEVICE, "copy of T0 failed"));
  const double *T0d = T0 ? (const double *)h->buf[1] : nullptr;
  hipError_t ie;
  if (p->dim == 3) {
    StepArgs3 A3;
    fill_args3(h->p, &A3);
    A3.dst = h->buf[0];
    ie = init3_async(p->q, p->storage, A3, p->scheme == LBM_SCHEME_EEBM, T0d,
                     h->stream);
  } else {
    StepArgs A;
    fill_step_args(h, &A);
    A.dst = h->buf[0];
    if (p->scheme == LBM_SCHEME_ILFBM) ilfbm_attach(h, ws + L.off_lf);
    ie = init_async(p->q, p->storage, A, T0d, h->stream, h->lf);
  }
  if (ie != hipSuccess || zero_stats_async(h) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return bail(fail(h, LBM_STEFAN_EDEVICE, "init kernels failed"));
  *out = h;
  return LBM_STEFAN_OK;
}

int lbm_stefan_step(lbm_stefan_t *h, int64_t nsteps, lbm_stefan_stats *stats) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(h, LBM_STEFAN_EINVAL, "nsteps < 0");
  DeviceGuard g(h->device);
  HIPCHK(h, advance(h, nsteps));
  if (stats || h->p.strict) {
    lbm_stefan_stats st;
    const int rc = read_stats(h, &st);
    if (stats) *stats = st;
    if (rc) return rc;
    if (h->p.strict && st.nonconverged > 0)
      return fail(h, LBM_STEFAN_ENOTCONV,
                  "a Newton solve reached newton_max_it");
  }
  return LBM_STEFAN_OK;
}

int lbm_stefan_reset_stats(lbm_stefan_t *h) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  DeviceGuard g(h->device);
  HIPCHK(h, zero_stats_async(h));
  return LBM_STEFAN_OK;
}

int lbm_stefan_query_front(lbm_stefan_t *h, int32_t mode, double *front,
                           double *energy) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  if (mode != LBM_FRONT_LIQUID_INTEGRAL && mode != LBM_FRONT_ZERO_CROSSING)
    return fail(h, LBM_STEFAN_EINVAL, "unknown front mode");
  DeviceGuard g(h->device);
  const lbm_stefan_params &p = h->p;
  double *fr = h->small + kSmallFront;
  if (front) {
    HIPCHK(h, front_async(p, h->buf[h->cur], mode, fr, h->stream, h->lf));
    HIPCHK(h, hipMemcpyAsync(front, fr, rows_of(p) * 8, hipMemcpyDeviceToHost,
                             h->stream));
  }
  double e = 0.0;
  if (energy) {
    HIPCHK(h, handle_energy_async(h, h->buf[h->cur]));
    HIPCHK(h, hipMemcpyAsync(&e, h->small + kSmallEnergy, 8,
                             hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (energy) {
    *energy = e;
    if (!std::isfinite(e)) return fail(h, LBM_STEFAN_ENAN, "energy is not finite");
  }
  return LBM_STEFAN_OK;
}

int lbm_stefan_get_field(lbm_stefan_t *h, int32_t what, void *host) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  if (!host) return fail(h, LBM_STEFAN_EINVAL, "host is NULL");
  DeviceGuard g(h->device);
  const lbm_stefan_params &p = h->p;
  const int64_t n = nodes_of(p);
  if (what == LBM_FIELD_STATE) {
    const size_t s = p.storage == LBM_STORE_F64 ? 8 : 4;
    HIPCHK(h, hipMemcpyAsync(host, h->buf[h->cur], p.q * n * s,
                             hipMemcpyDeviceToHost, h->stream));
  } else if (what == LBM_FIELD_T) {
    // the other population buffer is free between steps (>= 12 n bytes)
    double *T = (double *)h->buf[h->cur ^ 1];
    HIPCHK(h, temperature_async(p, h->buf[h->cur], T, h->stream));
    HIPCHK(h, hipMemcpyAsync(host, T, n * 8, hipMemcpyDeviceToHost, h->stream));
  } else if (what == LBM_FIELD_LIQUID) {
    double *l = (double *)h->buf[h->cur ^ 1];
    HIPCHK(h, liquid_async(p, h->buf[h->cur], h->lf, l, h->stream));
    HIPCHK(h, hipMemcpyAsync(host, l, n * 8, hipMemcpyDeviceToHost, h->stream));
  } else {
    return fail(h, LBM_STEFAN_EINVAL, "unknown field");
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return LBM_STEFAN_OK;
}

int lbm_stefan_set_state(lbm_stefan_t *h, const void *state, int32_t on_device) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  if (!state) return fail(h, LBM_STEFAN_EINVAL, "state is NULL");
  DeviceGuard g(h->device);
  const lbm_stefan_params &p = h->p;
  const size_t s = p.storage == LBM_STORE_F64 ? 8 : 4;
  const size_t bytes = (size_t)p.q * nodes_of(p) * s;
  HIPCHK(h, hipMemcpyAsync(h->buf[h->cur], state, bytes,
                           on_device ? hipMemcpyDeviceToDevice
                                     : hipMemcpyHostToDevice,
                           h->stream));
  if (!on_device) HIPCHK(h, hipStreamSynchronize(h->stream));
  return LBM_STEFAN_OK;
}

int lbm_stefan_state_ptr(lbm_stefan_t *h, void **dev_state) {
  if (!h || !dev_state) return fail(h, LBM_STEFAN_EINVAL, "NULL argument");
  *dev_state = h->buf[h->cur];
  return LBM_STEFAN_OK;
}

int lbm_stefan_variant_count(int32_t q, int32_t storage, int32_t *count) {
  if (!count || (q != 3 && q != 5 && q != 9 && q != 7 && q != 19) ||
      (storage != LBM_STORE_F64 && storage != LBM_STORE_F32))
    return fail(nullptr, LBM_STEFAN_EINVAL, "bad lattice, storage or count");
  int n;
  if (q == 7 || q == 19) variants3(&n);
  else variants(q, &n);
  *count = n;
  return LBM_STEFAN_OK;
}

const char *lbm_stefan_variant_name(int32_t q, int32_t storage,
                                    int32_t variant) {
  static thread_local char buf[64];
  int n;
  if (storage != LBM_STORE_F64 && storage != LBM_STORE_F32) return "";
  if (q == 7 || q == 19) {
    const Variant3 *v3 = variants3(&n);
    if (variant < 0 || variant >= n) return "";
    const Variant3 &w = v3[variant];
    std::snprintf(buf, sizeof(buf), "%dx%d/npt%d/z%d%s%s", w.bx * w.npt,
                  w.by, w.npt, w.cz, w.nt ? "/nt" : "", w.split ? "/s" : "");
    return buf;
  }
  if (q != 3 && q != 5 && q != 9) return "";
  const Variant *v = variants(q, &n);
  if (variant < 0 || variant >= n) return "";
  const Variant &w = v[variant];
  char rows[16] = "";
  if (w.rows > 1) std::snprintf(rows, sizeof(rows), "/r%d", w.rows);
  if (w.res)
    std::snprintf(buf, sizeof(buf), "resident%d", (int)kResident1D);
  else if (w.tb)
    std::snprintf(buf, sizeof(buf), "%dx%d/t2%s%s%s", w.bx, w.by,
                  w.tb == 2 ? "s" : "", rows, w.nt ? "/nt" : "");
  else
    std::snprintf(buf, sizeof(buf), "%dx%d/npt%d%s%s%s", w.bx * w.npt, w.by,
                  w.npt, rows, w.nt ? "/nt" : "", w.rev ? "/rev" : "");
  return buf;
}

int lbm_stefan_set_variant(lbm_stefan_t *h, int32_t variant) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  int n;
  if (h->p.dim == 3) variants3(&n);
  else variants(h->p.q, &n);
  if (variant < 0 || variant >= n)
    return fail(h, LBM_STEFAN_EINVAL, "unknown kernel variant");
  DeviceGuard g(h->device);
  h->variant = variant;
  // the tile -> slot mapping changes with the tile shape
  HIPCHK(h, zero_stats_async(h));
  return LBM_STEFAN_OK;
}

int lbm_stefan_autotune(lbm_stefan_t *h, void *scratch, size_t scratch_bytes,
                        int32_t steps, int32_t *best_variant,
                        double *best_ms_per_step) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  const lbm_stefan_params &p = h->p;
  const size_t sb = p.storage == LBM_STORE_F64 ? 8 : 4;
  const size_t bytes = (size_t)p.q * nodes_of(p) * sb;
  if (!scratch || scratch_bytes < bytes)
    return fail(h, LBM_STEFAN_EINVAL, "scratch smaller than the state");
  if (steps < 1 || steps > 10000)
    return fail(h, LBM_STEFAN_EINVAL, "steps must be in 1..10000");
  if (p.scheme == LBM_SCHEME_ILFBM) {
    // one kernel shape: nothing to choose
    if (best_variant) *best_variant = h->variant;
    if (best_ms_per_step) *best_ms_per_step = 0.0;
    return LBM_STEFAN_OK;
  }
  DeviceGuard g(h->device);
  int nv;
  const Variant *vt = nullptr;
  if (p.dim == 3) variants3(&nv);
  else vt = variants(p.q, &nv);
  const int cur0 = h->cur;
  HIPCHK(h, hipMemcpyAsync(scratch, h->buf[cur0], bytes,
                           hipMemcpyDeviceToDevice, h->stream));
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(h, LBM_STEFAN_EDEVICE, "hipEventCreate failed");
  }
  int best = h->variant;
  float best_ms = 0.0f;
  hipError_t err = hipSuccess;
  for (int v = 0; v < nv && err == hipSuccess; ++v) {
    // a Neumann lattice runs two-step variants as the default one, and a
    // lattice the resident kernel does not take runs that variant so too
    if (vt && vt[v].tb && has_neumann(p)) continue;
    if (vt && vt[v].res && !resident_ok(p)) continue;
    if (vt && vt[v].tb == 2) continue;  // single lattices: same as tb = 1
    h->variant = v;
    // two untimed steps, then the timed trial (an even count, so that a
    // two-step variant runs its own kernel only)
    const int64_t n = steps + (steps & 1);
    const int64_t steps0 = h->steps;
    err = advance(h, 2);
    if (err == hipSuccess) err = hipEventRecord(e0, h->stream);
    if (err == hipSuccess) err = advance(h, n);
    h->steps = steps0;
    if (err == hipSuccess) err = hipEventRecord(e1, h->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)n;
    if (err == hipSuccess && (v == 0 || ms < best_ms)) {
      best_ms = ms;
      best = v;
    }
    // restore the saved state for the next trial
    h->cur = cur0;
    if (err == hipSuccess)
      err = hipMemcpyAsync(h->buf[cur0], scratch, bytes,
                           hipMemcpyDeviceToDevice, h->stream);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->cur = cur0;
  h->variant = best;
  if (err != hipSuccess)
    return fail(h, LBM_STEFAN_EDEVICE,
                std::string("autotune: ") + hipGetErrorString(err));
  HIPCHK(h, zero_stats_async(h));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (best_variant) *best_variant = best;
  if (best_ms_per_step) *best_ms_per_step = best_ms;
  return LBM_STEFAN_OK;
}

int lbm_stefan_destroy(lbm_stefan_t *h) {
  if (!h) return LBM_STEFAN_OK;
  DeviceGuard g(h->device);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (h->side) {
    if (e == hipSuccess) e = hipStreamSynchronize(h->side);
    (void)hipEventDestroy(h->fork);
    (void)hipEventDestroy(h->join);
    (void)hipStreamDestroy(h->side);
  }
  delete h;
  if (e != hipSuccess)
    return fail(nullptr, LBM_STEFAN_EDEVICE, hipGetErrorString(e));
  return LBM_STEFAN_OK;
}

}  // extern "C"
