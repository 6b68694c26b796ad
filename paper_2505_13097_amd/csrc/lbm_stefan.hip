// lbm_stefan.hip -- gfx950 kernels and the C ABI of the IREBM step
// (Luddens, Lothode, Danaila, arXiv 2505.13097, Algorithm 3 with the
// boundary closures of Section 4.2).  See include/lbm_stefan.h.
//
// Kernels
//   step_kernel      one time step, one launch; each block owns one tile of
//                    the lattice (tile_x = bx * npt columns, tile_y = by
//                    rows).  Blocks are remapped so that each of the eight
//                    XCDs sweeps one contiguous band of tile rows: the rows
//                    a tile pulls from its neighbours then sit in that
//                    XCD's L2.  Interior tiles take a path with no bounds
//                    checks.  Per-tile Newton and flux statistics are
//                    accumulated by the owning block (no atomics).
//   init_kernel      equilibrium state from a temperature field.
//   temp_kernel      T = sum_i Omega_i.
//   energy_*         E = sum [T + phi(T)/Ste], two fixed-order passes.
//   front_*          per-row front position.
//   stats_kernel     fixed-order reduction of the per-tile slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>

#include "irebm_node.hpp"
#include "lbm_stefan.h"
#include "lbm_stefan_internal.hpp"

using namespace irebm;

namespace irebm {

constexpr int kEnergyChunk = 2048;  // nodes per energy partial

// ---------------------------------------------------------------------
// step

template <int Q, typename S, int NPT, bool PLAIN>
__global__ __launch_bounds__(256) void step_kernel(StepArgs A) {
  const int b = blockIdx.x;
  const int t = (b & 7) * A.per_xcd + (b >> 3);
  if (t >= A.ntiles) return;
  const int bx = blockDim.x, by = blockDim.y;
  const int TW = bx * NPT;
  const int tx = t % A.tiles_x, ty = t / A.tiles_x;
  const int x0 = tx * TW, y0 = ty * by;
  const bool fast = x0 >= 1 && x0 + TW <= A.nx - 1 &&
                    (Q == 3 || (y0 >= 1 && y0 + by <= A.ny - 1));
  const int y = y0 + (int)threadIdx.y;
  NodeStats st;
  if (fast) {
    NodeLoad<Q, S> L[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      load_node<Q, S, true>(A, x0 + (int)threadIdx.x + k * bx, y, L[k]);
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      update_node<Q, S, PLAIN, true>(A, x0 + (int)threadIdx.x + k * bx, y,
                                     L[k], st);
  } else {
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int x = x0 + (int)threadIdx.x + k * bx;
      if (x < A.nx && y < A.ny) {
        NodeLoad<Q, S> L;
        load_node<Q, S, false>(A, x, y, L);
        update_node<Q, S, PLAIN, false>(A, x, y, L, st);
      }
    }
  }
  // block reduction of the statistics, then one read-modify-write of the
  // tile's slot by thread 0
  __shared__ int s_it[4], s_nc[4];
  __shared__ double s_res[4], s_fin[4], s_fout[4];
  const int lin = (int)(threadIdx.x + threadIdx.y * blockDim.x);
  const int wid = lin >> 6, nw = (bx * by) >> 6;
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
    StatSlot *sl = A.slots + t;
    sl->max_it = max(sl->max_it, bit);
    sl->nonconv += bnc;
    sl->max_res = fmax(sl->max_res, bres);
    if (!fast) {
      sl->flux_in += bfin;
      sl->flux_out += bfout;
    }
  }
}

// ---------------------------------------------------------------------
// init, temperature, zero fill

template <int Q, typename S>
__global__ void init_kernel(StepArgs A, const double *T0) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.plane) return;
  const int x = (int)(k % A.nx), y = (int)(k / A.nx);
  const int wall = dirichlet_wall<Q>(A, x, y);
  const double T = wall >= 0 ? wall_value(A, wall, x, y) : (T0 ? T0[k] : 0.0);
  S *dst = (S *)A.dst;
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[i * A.plane + k] = (S)(wt<Q>(i) * T);
}

template <int Q, typename S>
__global__ void temp_kernel(const S *src, int64_t plane, double *T) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= plane) return;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) s += (double)src[j * plane + k];
  T[k] = s;
}

__global__ void zero_kernel(uint64_t *p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

// ---------------------------------------------------------------------
// fixed-order reductions

__device__ inline double block_sum_256(double v) {
  __shared__ double s[4];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s[w] = v;
  __syncthreads();
  double r = s[0] + s[1] + s[2] + s[3];
  __syncthreads();
  return r;
}

// partial[b] = sum over nodes [b*chunk, (b+1)*chunk) of T + phi(T)/Ste
template <int Q, typename S>
__global__ __launch_bounds__(256) void energy_partial_kernel(
    const S *src, int64_t plane, double tm, double inv_delta, double inv_ste,
    double *partial) {
  const int64_t base = (int64_t)blockIdx.x * kEnergyChunk;
  double acc = 0.0;
  for (int j = 0; j < kEnergyChunk / 256; ++j) {
    const int64_t k = base + j * 256 + threadIdx.x;
    if (k < plane) {
      double T = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) T += (double)src[i * plane + k];
      acc += T + phi_only(T, tm, inv_delta) * inv_ste;
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

// front of row blockIdx.x: dx * trapezoid sum of phi(T)
template <int Q, typename S>
__global__ __launch_bounds__(256) void front_integral_kernel(
    const S *src, int64_t plane, int nx, double tm, double inv_delta,
    double dx, double *out) {
  const int64_t row = (int64_t)blockIdx.x * nx;
  double acc = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) {
    double T = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) T += (double)src[i * plane + row + x];
    const double ph = phi_only(T, tm, inv_delta);
    acc += (x == 0 || x == nx - 1) ? 0.5 * ph : ph;
  }
  const double s = block_sum_256(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = dx * s;
}

template <int Q, typename S>
__device__ inline double temp_at(const S *src, int64_t plane, int64_t k) {
  double T = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) T += (double)src[i * plane + k];
  return T;
}

// first x (from x = 0) with T(x) - tm > 0 >= T(x+1) - tm, interpolated
template <int Q, typename S>
__global__ __launch_bounds__(256) void front_crossing_kernel(
    const S *src, int64_t plane, int nx, double tm, double dx, double *out) {
  const int64_t row = (int64_t)blockIdx.x * nx;
  const int chunk = (nx + 255) / 256;
  const int xa = threadIdx.x * chunk;
  int first = INT32_MAX;
  for (int x = xa; x < xa + chunk && x + 1 < nx; ++x) {
    const double t0 = temp_at<Q, S>(src, plane, row + x) - tm;
    const double t1 = temp_at<Q, S>(src, plane, row + x + 1) - tm;
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
    const double T0 = temp_at<Q, S>(src, plane, row) - tm;
    double pos;
    if (T0 <= 0.0) {
      pos = 0.0;
    } else if (m == INT32_MAX) {
      pos = (nx - 1) * dx;
    } else {
      const double t0 = temp_at<Q, S>(src, plane, row + m) - tm;
      const double t1 = temp_at<Q, S>(src, plane, row + m + 1) - tm;
      pos = dx * (m + t0 / (t0 - t1));
    }
    out[blockIdx.x] = pos;
  }
}

}  // namespace irebm

// =====================================================================
// host side

namespace {

thread_local std::string g_err = "no error";

struct Variant {
  int bx, by, npt;
};
const Variant kVariants1D[] = {{256, 1, 1}, {128, 1, 1}, {64, 1, 1},
                               {256, 1, 2}};
const Variant kVariants2D[] = {{64, 4, 1},  {256, 1, 1}, {128, 2, 1},
                               {64, 4, 2},  {128, 2, 2}, {256, 1, 2},
                               {64, 2, 2},  {64, 4, 4}};
constexpr int kNumV1 = sizeof(kVariants1D) / sizeof(Variant);
constexpr int kNumV2 = sizeof(kVariants2D) / sizeof(Variant);
constexpr int kDefaultV1 = 0;
constexpr int kDefaultV2 = 3;

const Variant *variants(int q, int *n) {
  if (q == 3) {
    *n = kNumV1;
    return kVariants1D;
  }
  *n = kNumV2;
  return kVariants2D;
}

int64_t tiles_for(const Variant &v, int64_t nx, int64_t ny) {
  const int64_t tw = (int64_t)v.bx * v.npt, th = v.by;
  return ((nx + tw - 1) / tw) * ((ny + th - 1) / th);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

std::string irebm::validate_params(const lbm_stefan_params *p) {
  if (!p) return "params is NULL";
  const bool lat = (p->dim == 1 && p->q == 3) ||
                   (p->dim == 2 && (p->q == 5 || p->q == 9));
  if (!lat) return "lattice must be D1Q3, D2Q5 or D2Q9";
  if (p->nx < 3) return "nx must be >= 3";
  if (p->dim == 1 && p->ny != 1) return "ny must be 1 for a 1D lattice";
  if (p->dim == 2 && p->ny < 3) return "ny must be >= 3 for a 2D lattice";
  if (p->nx * p->ny > ((int64_t)1 << 31) - 1)
    return "nx * ny must be below 2^31";
  if (p->nx > INT32_MAX || p->ny > INT32_MAX) return "nx, ny too large";
  if (p->storage != LBM_STORE_F64 && p->storage != LBM_STORE_F32)
    return "storage must be LBM_STORE_F64 or LBM_STORE_F32";
  if (p->newton_mode != LBM_NEWTON_SAFEGUARDED &&
      p->newton_mode != LBM_NEWTON_PLAIN)
    return "unknown newton_mode";
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return "tau must be > 1/2";
  if (!(p->ste > 0.0) || !std::isfinite(p->ste)) return "ste must be > 0";
  if (!(p->delta > 0.0) || !std::isfinite(p->delta))
    return "delta must be > 0";
  if (!std::isfinite(p->t_m)) return "t_m must be finite";
  if (!(p->newton_tol > 0.0)) return "newton_tol must be > 0";
  if (p->newton_max_it < 1 || p->newton_max_it > 1000)
    return "newton_max_it must be in 1..1000";
  if (!(p->dx >= 0.0) || !std::isfinite(p->dx)) return "dx must be >= 0";
  for (int k = 0; k < 4; ++k) {
    if (p->dim == 1 && k >= 2) break;
    if (p->bc[k] < LBM_BC_DIRICHLET || p->bc[k] > LBM_BC_PERIODIC)
      return "unknown boundary kind";
    if (!std::isfinite(p->wall_T[k])) return "wall_T must be finite";
  }
  if ((p->bc[0] == LBM_BC_PERIODIC) != (p->bc[1] == LBM_BC_PERIODIC))
    return "x walls: both or neither periodic";
  if (p->dim == 2 &&
      (p->bc[2] == LBM_BC_PERIODIC) != (p->bc[3] == LBM_BC_PERIODIC))
    return "y walls: both or neither periodic";
  int nv;
  variants(p->q, &nv);
  if (p->variant < -1 || p->variant >= nv) return "unknown kernel variant";
  return "";
}

irebm::Layout irebm::layout_for(const lbm_stefan_params *p) {
  Layout L;
  const int64_t n = p->nx * p->ny;
  const size_t s = p->storage == LBM_STORE_F64 ? 8 : 4;
  L.buf_bytes = align256((size_t)p->q * n * s);
  int nv;
  const Variant *v = variants(p->q, &nv);
  int64_t mt = 0;
  for (int i = 0; i < nv; ++i) mt = std::max(mt, tiles_for(v[i], p->nx, p->ny));
  L.max_tiles = mt;
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
  L.off_partials = off;
  off += align256((size_t)L.n_partials * 8);
  L.off_small = off;
  off += align256((size_t)(std::max<int64_t>(p->ny, 16) + 16) * 8);
  L.adjoint = (p->flags & LBM_FLAG_ADJOINT) != 0;
  L.off_adj = off;
  if (L.adjoint) off += adjoint_bytes(p, mt);
  L.total = off;
  return L;
}

int irebm::fail(lbm_stefan_t *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  else g_err = msg;
  return code;
}

#define HIPCHK(h, expr)                                                   \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return irebm::fail((h), LBM_STEFAN_EDEVICE,                         \
                         std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void irebm::fill_step_args(const lbm_stefan_t *h, StepArgs *A) {
  const lbm_stefan_params &p = h->p;
  std::memset(A, 0, sizeof(*A));
  A->nx = (int32_t)p.nx;
  A->ny = (int32_t)p.ny;
  A->plane = p.nx * p.ny;
  A->periodic_x = p.bc[0] == LBM_BC_PERIODIC;
  A->periodic_y = p.dim == 2 && p.bc[2] == LBM_BC_PERIODIC;
  A->a = 1.0 - 1.0 / p.tau;
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
  for (int k = 0; k < 4; ++k) {
    A->bc[k] = (p.dim == 1 && k >= 2) ? BC_PERIODIC : p.bc[k];
    A->wall_T[k] = p.wall_T[k];
    A->prof[k] = h->has_prof[k] ? h->prof[k] : nullptr;
  }
  A->slots = h->slots;
}

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess || prev == dev ||
        hipSetDevice(dev) != hipSuccess)
      prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <int Q, typename S>
hipError_t launch_step_t(const lbm_stefan_t *h, const StepArgs &A,
                         const Variant &v, bool plain) {
  const int64_t ntiles = tiles_for(v, h->p.nx, h->p.ny);
  const int per_xcd = (int)((ntiles + 7) / 8);
  StepArgs B = A;
  B.tiles_x = (int32_t)((h->p.nx + v.bx * v.npt - 1) / (v.bx * v.npt));
  B.ntiles = (int32_t)ntiles;
  B.per_xcd = per_xcd;
  dim3 grid(8 * per_xcd), block(v.bx, v.by);
#define LAUNCH(NPT, PL) \
  step_kernel<Q, S, NPT, PL><<<grid, block, 0, h->stream>>>(B)
  if (plain) {
    if (v.npt == 1) LAUNCH(1, true);
    else if (v.npt == 2) LAUNCH(2, true);
    else LAUNCH(4, true);
  } else {
    if (v.npt == 1) LAUNCH(1, false);
    else if (v.npt == 2) LAUNCH(2, false);
    else LAUNCH(4, false);
  }
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace

hipError_t irebm::launch_step(const lbm_stefan_t *h, const void *src,
                              void *dst) {
  StepArgs A;
  fill_step_args(h, &A);
  A.src = src;
  A.dst = dst;
  int nv;
  const Variant &v = variants(h->p.q, &nv)[h->variant];
  const bool plain = h->p.newton_mode == LBM_NEWTON_PLAIN;
  const bool f32 = h->p.storage == LBM_STORE_F32;
  switch (h->p.q) {
    case 3:
      return f32 ? launch_step_t<3, float>(h, A, v, plain)
                 : launch_step_t<3, double>(h, A, v, plain);
    case 5:
      return f32 ? launch_step_t<5, float>(h, A, v, plain)
                 : launch_step_t<5, double>(h, A, v, plain);
    default:
      return f32 ? launch_step_t<9, float>(h, A, v, plain)
                 : launch_step_t<9, double>(h, A, v, plain);
  }
}

namespace {

template <int Q>
using QT = std::integral_constant<int, Q>;
template <typename T>
struct TT {
  using type = T;
};

// calls f(QT<Q>{}, TT<S>{}) for the lattice and storage of a handle
template <typename F>
hipError_t dispatch_qs(int q, int storage, F &&f) {
  const bool f32 = storage == LBM_STORE_F32;
  switch (q) {
    case 3:
      return f32 ? f(QT<3>{}, TT<float>{}) : f(QT<3>{}, TT<double>{});
    case 5:
      return f32 ? f(QT<5>{}, TT<float>{}) : f(QT<5>{}, TT<double>{});
    default:
      return f32 ? f(QT<9>{}, TT<float>{}) : f(QT<9>{}, TT<double>{});
  }
}

#define QS_TYPES(qt, tt)                  \
  constexpr int Q = decltype(qt)::value; \
  using S = typename decltype(tt)::type

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t zero_async(uint64_t *p, int64_t n_words, hipStream_t s) {
  if (n_words <= 0) return hipSuccess;
  zero_kernel<<<blocks_for(n_words, 256), 256, 0, s>>>(p, n_words);
  return hipGetLastError();
}

// energy of the state `src` into h->small[kSmallEnergy] (device)
hipError_t energy_async(const lbm_stefan_t *h, const void *src) {
  return dispatch_qs(h->p.q, h->p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    const int64_t n = h->p.nx * h->p.ny;
    const int64_t parts = (n + kEnergyChunk - 1) / kEnergyChunk;
    energy_partial_kernel<Q, S><<<(unsigned)parts, 256, 0, h->stream>>>(
        (const S *)src, n, h->p.t_m, 1.0 / h->p.delta, 1.0 / h->p.ste,
        h->partials);
    sum_kernel<<<1, 256, 0, h->stream>>>(h->partials, parts,
                                         h->small + kSmallEnergy);
    return hipGetLastError();
  });
}

}  // namespace

hipError_t irebm::zero_stats_async(lbm_stefan_t *h) {
  return zero_async((uint64_t *)h->slots,
                    (int64_t)(h->max_tiles * sizeof(StatSlot) / 8), h->stream);
}

int irebm::read_stats(lbm_stefan_t *h, lbm_stefan_stats *st) {
  stats_kernel<<<1, 256, 0, h->stream>>>(h->slots, h->max_tiles, h->small);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, energy_async(h, h->buf[h->cur]));
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
  int nv;
  variants(p->q, &nv);
  h->variant = p->variant >= 0 ? p->variant : (p->q == 3 ? kDefaultV1 : kDefaultV2);
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
  h->max_tiles = L.max_tiles;
  h->partials = (double *)(ws + L.off_partials);
  h->small = (double *)(ws + L.off_small);
  h->adj = ws + L.off_adj;
  const int64_t n = p->nx * p->ny;
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
  StepArgs A;
  fill_step_args(h, &A);
  A.dst = h->buf[0];
  const double *T0d = T0 ? (const double *)h->buf[1] : nullptr;
  auto r = [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    init_kernel<Q, S><<<blocks_for(A.plane, 256), 256, 0, h->stream>>>(A, T0d);
    return hipGetLastError();
  };
  if (dispatch_qs(p->q, p->storage, r) != hipSuccess ||
      zero_stats_async(h) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return bail(fail(h, LBM_STEFAN_EDEVICE, "init kernels failed"));
  *out = h;
  return LBM_STEFAN_OK;
}

int lbm_stefan_step(lbm_stefan_t *h, int64_t nsteps, lbm_stefan_stats *stats) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(h, LBM_STEFAN_EINVAL, "nsteps < 0");
  DeviceGuard g(h->device);
  for (int64_t s = 0; s < nsteps; ++s) {
    HIPCHK(h, launch_step(h, h->buf[h->cur], h->buf[h->cur ^ 1]));
    h->cur ^= 1;
    h->steps++;
  }
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
    auto r = [&](auto qt, auto tt) {
      QS_TYPES(qt, tt);
      const S *src = (const S *)h->buf[h->cur];
      if (mode == LBM_FRONT_LIQUID_INTEGRAL)
        front_integral_kernel<Q, S><<<(unsigned)p.ny, 256, 0, h->stream>>>(
            src, p.nx * p.ny, (int)p.nx, p.t_m, 1.0 / p.delta, p.dx, fr);
      else
        front_crossing_kernel<Q, S><<<(unsigned)p.ny, 256, 0, h->stream>>>(
            src, p.nx * p.ny, (int)p.nx, p.t_m, p.dx, fr);
      return hipGetLastError();
    };
    HIPCHK(h, dispatch_qs(p.q, p.storage, r));
    HIPCHK(h, hipMemcpyAsync(front, fr, p.ny * 8, hipMemcpyDeviceToHost,
                             h->stream));
  }
  double e = 0.0;
  if (energy) {
    HIPCHK(h, energy_async(h, h->buf[h->cur]));
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
  const int64_t n = p.nx * p.ny;
  if (what == LBM_FIELD_STATE) {
    const size_t s = p.storage == LBM_STORE_F64 ? 8 : 4;
    HIPCHK(h, hipMemcpyAsync(host, h->buf[h->cur], p.q * n * s,
                             hipMemcpyDeviceToHost, h->stream));
  } else if (what == LBM_FIELD_T) {
    // the other population buffer is free between steps (>= 12 n bytes)
    double *T = (double *)h->buf[h->cur ^ 1];
    auto r = [&](auto qt, auto tt) {
      QS_TYPES(qt, tt);
      temp_kernel<Q, S><<<blocks_for(n, 256), 256, 0, h->stream>>>(
          (const S *)h->buf[h->cur], n, T);
      return hipGetLastError();
    };
    HIPCHK(h, dispatch_qs(p.q, p.storage, r));
    HIPCHK(h, hipMemcpyAsync(host, T, n * 8, hipMemcpyDeviceToHost, h->stream));
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
  const size_t bytes = (size_t)p.q * p.nx * p.ny * s;
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
  if (!count || (q != 3 && q != 5 && q != 9) ||
      (storage != LBM_STORE_F64 && storage != LBM_STORE_F32))
    return fail(nullptr, LBM_STEFAN_EINVAL, "bad lattice, storage or count");
  int n;
  variants(q, &n);
  *count = n;
  return LBM_STEFAN_OK;
}

const char *lbm_stefan_variant_name(int32_t q, int32_t storage,
                                    int32_t variant) {
  static thread_local char buf[64];
  int n;
  if ((q != 3 && q != 5 && q != 9) ||
      (storage != LBM_STORE_F64 && storage != LBM_STORE_F32))
    return "";
  const Variant *v = variants(q, &n);
  if (variant < 0 || variant >= n) return "";
  std::snprintf(buf, sizeof(buf), "%dx%d/npt%d", v[variant].bx * v[variant].npt,
                v[variant].by, v[variant].npt);
  return buf;
}

int lbm_stefan_set_variant(lbm_stefan_t *h, int32_t variant) {
  if (!h) return fail(nullptr, LBM_STEFAN_EINVAL, "handle is NULL");
  int n;
  variants(h->p.q, &n);
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
  const size_t bytes = (size_t)p.q * p.nx * p.ny * sb;
  if (!scratch || scratch_bytes < bytes)
    return fail(h, LBM_STEFAN_EINVAL, "scratch smaller than the state");
  if (steps < 1 || steps > 10000)
    return fail(h, LBM_STEFAN_EINVAL, "steps must be in 1..10000");
  DeviceGuard g(h->device);
  int nv;
  variants(p.q, &nv);
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
    h->variant = v;
    // two untimed steps, then the timed trial
    for (int s = 0; s < steps + 2 && err == hipSuccess; ++s) {
      if (s == 2) err = hipEventRecord(e0, h->stream);
      if (err == hipSuccess)
        err = launch_step(h, h->buf[h->cur], h->buf[h->cur ^ 1]);
      h->cur ^= 1;
    }
    if (err == hipSuccess) err = hipEventRecord(e1, h->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
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
  if (best_ms_per_step) *best_ms_per_step = best_ms / steps;
  return LBM_STEFAN_OK;
}

int lbm_stefan_destroy(lbm_stefan_t *h) {
  if (!h) return LBM_STEFAN_OK;
  DeviceGuard g(h->device);
  const hipError_t e = hipStreamSynchronize(h->stream);
  delete h;
  if (e != hipSuccess)
    return fail(nullptr, LBM_STEFAN_EDEVICE, hipGetErrorString(e));
  return LBM_STEFAN_OK;
}

}  // extern "C"
