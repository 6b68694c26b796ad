// host_util.hpp -- host-side helpers shared by the translation units of
// the library: kernel variant table, type dispatch, error macro, device
// guard and small launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "kernels.hpp"
#include "lbm_stefan.h"

namespace irebm {

// A kernel variant: block of bx x by threads, each thread updating npt
// nodes bx apart along x; the tile is (bx * npt) x by nodes, and one block
// sweeps `rows` tiles stacked along y.  nt: stores bypass the caches
// (non-temporal); rev: the item order is reversed on every other step, so
// that the rows written last (still in the memory-side cache) are read
// first.  tb: two steps per launch (step2_kernel): a window of bx columns
// (bx - 4 written), by rows per pass, `rows` rows per block, non-temporal
// stores.  res: D1Q3 lattices of at most kResident1D nodes run many steps
// per launch in one workgroup (resident1d_kernel); others take the default
// one-step tiling.  tb = 2: the same two-step kernel, run in the batched
// form with the front split (batch_step2_kernel: quiet pass, front strips,
// full pass over flagged items); single lattices run it as tb = 1.
struct Variant {
  int bx, by, npt, nt, rev, rows, tb, res;
};

inline const Variant *variants(int q, int *n) {
  static const Variant v1[] = {{256, 1, 1, 0, 0, 1, 0}, {128, 1, 1, 0, 0, 1, 0},
                               {64, 1, 1, 0, 0, 1, 0},  {256, 1, 2, 0, 0, 1, 0},
                               {1024, 1, 2, 0, 0, 1, 0, 1}};
  static const Variant v2[] = {
      {64, 4, 1, 0, 0, 1, 0}, {256, 1, 1, 0, 0, 1, 0}, {128, 2, 1, 0, 0, 1, 0},
      {64, 4, 2, 0, 0, 1, 0}, {128, 2, 2, 0, 0, 1, 0}, {256, 1, 2, 0, 0, 1, 0},
      {64, 2, 2, 0, 0, 1, 0}, {64, 4, 4, 0, 0, 1, 0},  {64, 4, 2, 1, 0, 1, 0},
      {64, 4, 2, 0, 1, 1, 0}, {64, 4, 2, 1, 1, 1, 0},  {128, 2, 2, 0, 1, 1, 0},
      {64, 4, 2, 1, 0, 2, 0}, {64, 4, 2, 1, 0, 4, 0},  {64, 4, 2, 1, 0, 8, 0},
      {64, 4, 2, 0, 0, 4, 0}, {64, 4, 1, 1, 0, 4, 0},  {64, 4, 2, 1, 1, 4, 0},
      {128, 2, 2, 1, 0, 4, 0}, {64, 4, 2, 1, 0, 16, 0}, {64, 1, 1, 0, 0, 1, 0},
      {64, 2, 1, 0, 0, 1, 0},
      {256, 2, 1, 1, 0, 32, 1},  {256, 2, 1, 1, 0, 64, 1},
      {128, 2, 1, 1, 0, 16, 1},  {128, 2, 1, 1, 0, 24, 1},
      {128, 2, 1, 1, 0, 32, 1},  {128, 2, 1, 1, 0, 64, 1},
      {128, 4, 1, 1, 0, 32, 1},  {128, 4, 1, 1, 0, 64, 1},
      {128, 2, 1, 1, 0, 16, 2},  {128, 2, 1, 1, 0, 24, 2},
      {128, 2, 1, 1, 0, 32, 2},  {128, 2, 1, 1, 0, 64, 2},
      {128, 4, 1, 1, 0, 32, 2},  {128, 2, 1, 1, 0, 96, 2},
      {128, 2, 1, 1, 0, 128, 2}};
  if (q == 3) {
    *n = (int)(sizeof(v1) / sizeof(Variant));
    return v1;
  }
  *n = (int)(sizeof(v2) / sizeof(Variant));
  return v2;
}
constexpr int kDefaultVariant1D = 0;
constexpr int kResidentVariant1D = 4;
constexpr int kDefaultVariant2D = 3;
// split two-step schedule: the front strip of an instance heated at x = 0
// is its first kFrontColumns columns (batch_front_kernel: at most 63)
constexpr int kFrontColumns = 60;

inline int64_t tiles_x_for(const Variant &v, int64_t nx) {
  const int64_t tw = (int64_t)v.bx * v.npt;
  return (nx + tw - 1) / tw;
}
inline int64_t tiles_y_for(const Variant &v, int64_t ny) {
  return (ny + v.by - 1) / v.by;
}
// work items (one block each) of an nx x ny lattice
inline int64_t items_for(const Variant &v, int64_t nx, int64_t ny) {
  if (v.tb)
    return ((nx + v.bx - 5) / (v.bx - 4)) * ((ny + v.rows - 1) / v.rows);
  return tiles_x_for(v, nx) * ((tiles_y_for(v, ny) + v.rows - 1) / v.rows);
}
// tile grid and work items of A for variant v
// (two-step variants: tiles_x strips of bx - 4 columns, tiles_y segments
// of `rows` rows, group = rows)
inline void set_tiling(StepArgs *A, const Variant &v) {
  if (v.tb) {
    A->tiles_x = (A->nx + v.bx - 5) / (v.bx - 4);
    A->tiles_y = (A->ny + v.rows - 1) / v.rows;
  } else {
    A->tiles_x = (int32_t)tiles_x_for(v, A->nx);
    A->tiles_y = (int32_t)tiles_y_for(v, A->ny);
  }
  A->group = v.rows;
  A->nitems = (int32_t)items_for(v, A->nx, A->ny);
  A->per_xcd = (A->nitems + 7) / 8;
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline unsigned blocks_for(int64_t n, int t) {
  return (unsigned)((n + t - 1) / t);
}

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

template <int Q>
using QT = std::integral_constant<int, Q>;
template <typename T>
struct TT {
  using type = T;
};

// calls f(QT<Q>{}, TT<S>{}) for a lattice and a storage type
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

// as dispatch_qs, also for the 3D lattices (q = 7, 19): for the kernels
// that only loop over the q planes (fields, energy, front)
template <typename F>
hipError_t dispatch_qs_all(int q, int storage, F &&f) {
  const bool f32 = storage == LBM_STORE_F32;
  if (q == 7) return f32 ? f(QT<7>{}, TT<float>{}) : f(QT<7>{}, TT<double>{});
  if (q == 19)
    return f32 ? f(QT<19>{}, TT<float>{}) : f(QT<19>{}, TT<double>{});
  return dispatch_qs(q, storage, f);
}

// nodes of a lattice, and its rows along x
inline int64_t lattice_nodes(const lbm_stefan_params &p) {
  return p.nx * p.ny * (p.dim == 3 ? p.nz : 1);
}
inline int64_t lattice_rows(const lbm_stefan_params &p) {
  return p.ny * (p.dim == 3 ? p.nz : 1);
}

#define QS_TYPES(qt, tt)                  \
  constexpr int Q = decltype(qt)::value; \
  using S = typename decltype(tt)::type

inline hipError_t zero_async(void *p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 8);
  if (n <= 0) return hipSuccess;
  zero_kernel<<<blocks_for(n, 256), 256, 0, s>>>((uint64_t *)p, n);
  return hipGetLastError();
}

// E = sum [T + phi(T)/Ste] (EEBM: sum H) of the state `src` of a lattice
// with params p into *out (device), using `partials` (>= ceil(nodes /
// kEnergyChunk) doubles) as scratch
inline hipError_t energy_async(const lbm_stefan_params &p, const void *src,
                               double *partials, double *out,
                               hipStream_t stream,
                               const double *lf = nullptr) {
  const int64_t n = lattice_nodes(p);
  return dispatch_qs_all(p.q, p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    const int64_t parts = (n + kEnergyChunk - 1) / kEnergyChunk;
    energy_partial_kernel<Q, S><<<(unsigned)parts, 256, 0, stream>>>(
        (const S *)src, n, p.scheme == LBM_SCHEME_EEBM, p.t_m, 1.0 / p.delta,
        1.0 / p.ste, lf, partials);
    sum_kernel<<<1, 256, 0, stream>>>(partials, parts, out);
    return hipGetLastError();
  });
}

// per-row front of the state `src` of a lattice with params p (p.dx > 0)
// into out[0..rows) (device; rows ny, or nz * ny in 3D); lf: the ILFBM
// liquid fraction plane
inline hipError_t front_async(const lbm_stefan_params &p, const void *src,
                              int mode, double *out, hipStream_t stream,
                              const double *lf = nullptr) {
  const int eebm = p.scheme == LBM_SCHEME_EEBM;
  const int64_t n = lattice_nodes(p);
  const unsigned rows = (unsigned)lattice_rows(p);
  return dispatch_qs_all(p.q, p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    if (mode == LBM_FRONT_LIQUID_INTEGRAL)
      front_integral_kernel<Q, S><<<rows, 256, 0, stream>>>(
          (const S *)src, n, (int)p.nx, eebm, p.t_m, 1.0 / p.delta, p.ste,
          lf, p.dx, out);
    else
      front_crossing_kernel<Q, S><<<rows, 256, 0, stream>>>(
          (const S *)src, n, (int)p.nx, eebm, p.t_m, 1.0 / p.ste, p.dx, out);
    return hipGetLastError();
  });
}

// temperature of every node of the state `src` into T (device doubles)
inline hipError_t temperature_async(const lbm_stefan_params &p,
                                    const void *src, double *T,
                                    hipStream_t stream) {
  const int64_t n = lattice_nodes(p);
  return dispatch_qs_all(p.q, p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    temp_kernel<Q, S><<<blocks_for(n, 256), 256, 0, stream>>>(
        (const S *)src, n, p.scheme == LBM_SCHEME_EEBM, p.t_m, 1.0 / p.ste,
        T);
    return hipGetLastError();
  });
}

// liquid fraction of every node of the state `src` into out (device)
inline hipError_t liquid_async(const lbm_stefan_params &p, const void *src,
                               const double *lf, double *out,
                               hipStream_t stream) {
  const int64_t n = lattice_nodes(p);
  return dispatch_qs_all(p.q, p.storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    liquid_kernel<Q, S><<<blocks_for(n, 256), 256, 0, stream>>>(
        (const S *)src, n, p.scheme == LBM_SCHEME_EEBM, p.t_m, 1.0 / p.delta,
        p.ste, lf, out);
    return hipGetLastError();
  });
}

// equilibrium initial state of the lattice described by A (A.dst), and
// the ILFBM liquid fraction into lf when given
inline hipError_t init_async(int q, int storage, const StepArgs &A,
                             const double *T0, hipStream_t stream,
                             double *lf = nullptr) {
  return dispatch_qs(q, storage, [&](auto qt, auto tt) {
    QS_TYPES(qt, tt);
    init_kernel<Q, S><<<blocks_for(A.plane, 256), 256, 0, stream>>>(A, T0,
                                                                     lf);
    return hipGetLastError();
  });
}

}  // namespace irebm

#define HIPCHK(h, expr)                                                   \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return irebm::fail((h), LBM_STEFAN_EDEVICE,                         \
                         std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
