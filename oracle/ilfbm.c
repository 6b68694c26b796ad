/*
 * ilfbm.c -- oracle for the implicit liquid fraction based method
 * (ILFBM, Section 3.3, Algorithm 1), the inner-loop scheme the paper
 * compares IREBM with.  TEST INFRASTRUCTURE ONLY: see oracle.h.
 *
 * The state is the distribution f (M0(f) = theta, f_i^eq = w_i theta) and
 * the liquid fraction field l, stored as plane q after the q population
 * planes.  One step (Algorithm 1):
 *   theta = M0(f), f^eq = w_i theta, l^(0) = l;
 *   for k = 1, 2, ...:
 *     collision with the source (w_i/Ste)(l - l^(k-1)),
 *     pull streaming to f^(k) (closures of Section 4.2 on the streamed
 *     populations, the Dirichlet target being T_D itself),
 *     H^(k) = M0(f^(k)) + l^(k-1)/Ste, l^(k) = l(H^(k)),
 *   until max |l^(k) - l^(k-1)| <= tol (at most max_it iterations);
 *   f~ = f^(k), l~ = l^(k).
 * l(H) = clamp(Ste (H - T_m), 0, 1) (Section 3.3 with T_m in place of 0).
 * The tolerance and the cap are the params' tol and max_it.  The line of
 * Algorithm 1 that sets H from phi(theta) before the loop has no use in
 * the step and is left out.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "explicit_common.h"

/* Dirichlet target of the closure: M0(f) = theta, so T_D itself */
static double wall_theta(const orc_params *p, double TD) {
  (void)p;
  return TD;
}

int orc_ilfbm_init(const orc_params *p, const double *T0, double *f) {
  lat L;
  if (check(p, &L)) return -1;
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++)
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      const int wall = dirichlet_wall(p, x, y);
      const double T = wall >= 0 ? wall_value(p, wall, x, y)
                                 : (T0 ? T0[k] : 0.0);
      for (int i = 0; i < p->q; i++) f[i * n + k] = L.w[i] * T;
      f[p->q * n + k] = lf_of_T(T, p->tm);
    }
  return 0;
}

/* BGK collision without source at every node: (1 - 1/tau) f + w theta/tau */
static void collide(const orc_params *p, const lat *L, const double *f,
                    double *omega) {
  const long n = p->nx * p->ny;
  for (long k = 0; k < n; k++) {
    double th = 0.0;
    for (int i = 0; i < p->q; i++) th += f[i * n + k];
    for (int i = 0; i < p->q; i++)
      omega[i * n + k] =
          f[i * n + k] - (f[i * n + k] - L->w[i] * th) / p->tau;
  }
}

int orc_ilfbm_collide(const orc_params *p, const double *f, double *omega) {
  lat L;
  if (check(p, &L)) return -1;
  collide(p, &L, f, omega);
  return 0;
}

typedef struct {
  double *om0, *om, *lprev;
} work;

/* one ILFBM step f -> fout (both with the l plane); returns the inner
   iteration count and the last max |l^(k) - l^(k-1)| in *dl */
static int step(const orc_params *p, const lat *L, const double *f,
                double *fout, const work *w, double *fin, double *fo,
                double *dl) {
  const long n = p->nx * p->ny;
  const double *l = f + p->q * n;
  double *lout = fout + p->q * n;
  collide(p, L, f, w->om0);
  memcpy(w->lprev, l, sizeof(double) * n);
  int k = 0;
  double d = 0.0;
  while (k < p->max_it) {
    k++;
    /* collision with the source (w_i/Ste)(l - l^(k-1)) */
    for (int i = 0; i < p->q; i++)
      for (long j = 0; j < n; j++)
        w->om[i * n + j] =
            w->om0[i * n + j] + L->w[i] / p->ste * (l[j] - w->lprev[j]);
    /* streaming and closures (fluxes of the last iteration only) */
    *fin = 0.0;
    *fo = 0.0;
    stream_close(p, L, w->om, wall_theta, fout, fin, fo);
    /* enthalpy and liquid fraction */
    d = 0.0;
    for (long j = 0; j < n; j++) {
      double th = 0.0;
      for (int i = 0; i < p->q; i++) th += fout[i * n + j];
      const double H = th + w->lprev[j] / p->ste;
      lout[j] = lf_of_H(H, p->ste, p->tm);
      const double e = fabs(lout[j] - w->lprev[j]);
      if (e > d) d = e;
    }
    if (d <= p->tol) break;
    memcpy(w->lprev, lout, sizeof(double) * n);
  }
  *dl = d;
  return k;
}

static int alloc_work(const orc_params *p, work *w) {
  const long n = p->nx * p->ny;
  w->om0 = malloc(sizeof(double) * p->q * n);
  w->om = malloc(sizeof(double) * p->q * n);
  w->lprev = malloc(sizeof(double) * n);
  if (w->om0 && w->om && w->lprev) return 0;
  free(w->om0);
  free(w->om);
  free(w->lprev);
  return -1;
}

static void free_work(work *w) {
  free(w->om0);
  free(w->om);
  free(w->lprev);
}

static void add_stats(const orc_params *p, orc_stats *st, int it, double dl,
                      double fin, double fo) {
  if (!st) return;
  if (it > st->max_it) st->max_it = it;
  if (dl > p->tol) {
    st->nonconverged++;
    if (dl > st->max_residual) st->max_residual = dl;
  }
  st->it_hist[it < 32 ? it : 32]++;
  st->flux_in += fin;
  st->flux_out += fo;
}

int orc_ilfbm_step(const orc_params *p, const double *f, double *fout,
                   orc_stats *st) {
  lat L;
  work w;
  if (check(p, &L) || p->max_it < 1 || alloc_work(p, &w)) return -1;
  double fin, fo, dl;
  const int it = step(p, &L, f, fout, &w, &fin, &fo, &dl);
  add_stats(p, st, it, dl, fin, fo);
  free_work(&w);
  return 0;
}

/* Compensated sum of E = sum_x [theta + l/Ste]. */
int orc_ilfbm_energy(const orc_params *p, const double *f, double *E) {
  lat L;
  if (check(p, &L)) return -1;
  const long n = p->nx * p->ny;
  double s = 0.0, c = 0.0;
  for (long k = 0; k < n; k++) {
    double th = 0.0;
    for (int i = 0; i < p->q; i++) th += f[i * n + k];
    const double h = th + f[p->q * n + k] / p->ste;
    double y = h - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  *E = s;
  return 0;
}

int orc_ilfbm_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
                  double *energy_trace, double *flux_trace) {
  lat L;
  work w;
  if (check(p, &L) || nsteps < 0 || p->max_it < 1) return -1;
  const long n = p->nx * p->ny;
  double *g = malloc(sizeof(double) * (p->q + 1) * n);
  if (!g || alloc_work(p, &w)) {
    free(g);
    return -1;
  }
  double *cur = f, *nxt = g;
  if (energy_trace) orc_ilfbm_energy(p, cur, &energy_trace[0]);
  for (long s = 0; s < nsteps; s++) {
    double fin, fo, dl;
    const int it = step(p, &L, cur, nxt, &w, &fin, &fo, &dl);
    add_stats(p, st, it, dl, fin, fo);
    if (flux_trace) {
      flux_trace[2 * s] = fin;
      flux_trace[2 * s + 1] = fo;
    }
    double *t = cur;
    cur = nxt;
    nxt = t;
    if (energy_trace) orc_ilfbm_energy(p, cur, &energy_trace[s + 1]);
  }
  if (cur != f) memcpy(f, cur, sizeof(double) * (p->q + 1) * n);
  free(g);
  free_work(&w);
  return 0;
}

int orc_ilfbm_temperature(const orc_params *p, const double *f, double *T) {
  lat L;
  if (check(p, &L)) return -1;
  const long n = p->nx * p->ny;
  for (long k = 0; k < n; k++) {
    double th = 0.0;
    for (int i = 0; i < p->q; i++) th += f[i * n + k];
    T[k] = th;
  }
  return 0;
}

/* Front per row: ORC_FRONT_INTEGRAL, dx * trapezoid sum of the liquid
   fraction l along x; ORC_FRONT_CROSSING, first place from x = 0 where
   theta - T_m goes from > 0 to <= 0, linearly interpolated. */
int orc_ilfbm_front(const orc_params *p, const double *f, int mode,
                    double *xf) {
  lat L;
  if (check(p, &L)) return -1;
  if (mode != ORC_FRONT_INTEGRAL && mode != ORC_FRONT_CROSSING) return -1;
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++) {
    double acc = 0.0, prev = 0.0, pos = (nx - 1) * p->dx;
    int found = 0;
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      if (mode == ORC_FRONT_INTEGRAL) {
        const double wx = (x == 0 || x == nx - 1) ? 0.5 : 1.0;
        acc += wx * f[p->q * n + k];
      } else if (!found) {
        double th = 0.0;
        for (int i = 0; i < p->q; i++) th += f[i * n + k];
        const double T = th - p->tm;
        if (x == 0 && T <= 0.0) {
          pos = 0.0;
          found = 1;
        } else if (x > 0 && prev > 0.0 && T <= 0.0) {
          pos = p->dx * (x - 1 + prev / (prev - T));
          found = 1;
        }
        prev = T;
      }
    }
    xf[y] = mode == ORC_FRONT_INTEGRAL ? p->dx * acc : pos;
  }
  return 0;
}
