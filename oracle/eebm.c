/*
 * eebm.c -- oracle for the explicit enthalpy based method (EEBM,
 * Section 3.4, Algorithm 2), the no-Newton scheme the paper compares
 * IREBM with.  TEST INFRASTRUCTURE ONLY: see oracle.h.
 *
 * The distribution f has the enthalpy as zeroth moment, H = M0(f); the
 * temperature is recovered explicitly, theta = Theta(H), with the sharp
 * liquid fraction (Section 3.4, with the melting temperature T_m in place
 * of 0):
 *   Theta(H) = H            for H < T_m,
 *            = T_m          for T_m <= H <= T_m + 1/Ste,
 *            = H - 1/Ste    for H > T_m + 1/Ste.
 * The equilibrium keeps the higher moments of w_i theta and moves the
 * difference to the rest population: f_i^eq = w_i theta (i != 0),
 * f_0^eq = H - (1 - w_0) theta, so M0(f^eq) = H.  One step is the BGK
 * collision towards f^eq followed by pull streaming, with the boundary
 * closures of the IREBM oracle applied to the streamed populations, the
 * Dirichlet target being the wall enthalpy T_D + l(T_D)/Ste (l = 1 above
 * T_m, 0 at or below it) and the Neumann target the enthalpy streamed
 * into the mirror node.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

double orc_eebm_theta(double H, double ste, double tm) {
  if (H < tm) return H;
  if (H <= tm + 1.0 / ste) return tm;
  return H - 1.0 / ste;
}

#include "explicit_common.h"

/* Dirichlet target of the closure: the wall enthalpy T_D + l(T_D)/Ste */
static double wall_enthalpy(const orc_params *p, double TD) {
  return TD + lf_of_T(TD, p->tm) / p->ste;
}

/* equilibrium populations of enthalpy H (temperature Theta(H)) */
static void equilibrium(const orc_params *p, const lat *L, double H,
                        double *feq) {
  const double th = orc_eebm_theta(H, p->ste, p->tm);
  for (int i = 1; i < p->q; i++) feq[i] = L->w[i] * th;
  feq[0] = H - (1.0 - L->w[0]) * th;
}

int orc_eebm_init(const orc_params *p, const double *T0, double *f) {
  lat L;
  if (check(p, &L)) return -1;
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++)
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      const int wall = dirichlet_wall(p, x, y);
      const double T = wall >= 0 ? wall_value(p, wall, x, y)
                                 : (T0 ? T0[k] : 0.0);
      double feq[9];
      equilibrium(p, &L, T + lf_of_T(T, p->tm) / p->ste, feq);
      for (int i = 0; i < p->q; i++) f[i * n + k] = feq[i];
    }
  return 0;
}

/* moments H = M0(f), equilibrium and BGK collision at every node */
static void collide(const orc_params *p, const lat *L, const double *f,
                    double *omega) {
  const long n = p->nx * p->ny;
  const double tau = p->tau;
  for (long k = 0; k < n; k++) {
    double H = 0.0, feq[9];
    for (int i = 0; i < p->q; i++) H += f[i * n + k];
    equilibrium(p, L, H, feq);
    for (int i = 0; i < p->q; i++)
      omega[i * n + k] = f[i * n + k] - (f[i * n + k] - feq[i]) / tau;
  }
}

int orc_eebm_collide(const orc_params *p, const double *f, double *omega) {
  lat L;
  if (check(p, &L)) return -1;
  collide(p, &L, f, omega);
  return 0;
}

/* one EEBM step f -> fout (Algorithm 2), closures as in the header */
static void step(const orc_params *p, const lat *L, const double *f,
                 double *fout, double *omega, double *fin, double *fo) {
  collide(p, L, f, omega);
  stream_close(p, L, omega, wall_enthalpy, fout, fin, fo);
}

int orc_eebm_step(const orc_params *p, const double *f, double *fout,
                  orc_stats *st) {
  lat L;
  if (check(p, &L)) return -1;
  double *om = malloc(sizeof(double) * p->q * p->nx * p->ny);
  if (!om) return -1;
  double fin = 0.0, fo = 0.0;
  step(p, &L, f, fout, om, &fin, &fo);
  if (st) {
    st->flux_in += fin;
    st->flux_out += fo;
  }
  free(om);
  return 0;
}

/* Compensated sum of E = sum_x H(x) = sum_x M0(f)(x). */
int orc_eebm_energy(const orc_params *p, const double *f, double *E) {
  lat L;
  if (check(p, &L)) return -1;
  const long n = p->nx * p->ny;
  double s = 0.0, c = 0.0;
  for (long k = 0; k < n; k++) {
    double H = 0.0;
    for (int i = 0; i < p->q; i++) H += f[i * n + k];
    double y = H - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  *E = s;
  return 0;
}

int orc_eebm_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
                 double *energy_trace, double *flux_trace) {
  lat L;
  if (check(p, &L) || nsteps < 0) return -1;
  const long n = p->nx * p->ny;
  double *g = malloc(sizeof(double) * p->q * n);
  double *om = malloc(sizeof(double) * p->q * n);
  if (!g || !om) {
    free(g);
    free(om);
    return -1;
  }
  double *cur = f, *nxt = g;
  if (energy_trace) orc_eebm_energy(p, cur, &energy_trace[0]);
  for (long s = 0; s < nsteps; s++) {
    double fin = 0.0, fo = 0.0;
    step(p, &L, cur, nxt, om, &fin, &fo);
    if (st) {
      st->flux_in += fin;
      st->flux_out += fo;
    }
    if (flux_trace) {
      flux_trace[2 * s] = fin;
      flux_trace[2 * s + 1] = fo;
    }
    double *t = cur;
    cur = nxt;
    nxt = t;
    if (energy_trace) orc_eebm_energy(p, cur, &energy_trace[s + 1]);
  }
  if (cur != f) memcpy(f, cur, sizeof(double) * p->q * n);
  free(g);
  free(om);
  return 0;
}

int orc_eebm_temperature(const orc_params *p, const double *f, double *T) {
  lat L;
  if (check(p, &L)) return -1;
  const long n = p->nx * p->ny;
  for (long k = 0; k < n; k++) {
    double H = 0.0;
    for (int i = 0; i < p->q; i++) H += f[i * n + k];
    T[k] = orc_eebm_theta(H, p->ste, p->tm);
  }
  return 0;
}

/* Front per row: ORC_FRONT_INTEGRAL, dx * trapezoid sum of the liquid
   fraction l(H) along x; ORC_FRONT_CROSSING, first place from x = 0 where
   Theta(H) - T_m goes from > 0 to <= 0, linearly interpolated. */
int orc_eebm_front(const orc_params *p, const double *f, int mode,
                   double *xf) {
  lat L;
  if (check(p, &L)) return -1;
  if (mode != ORC_FRONT_INTEGRAL && mode != ORC_FRONT_CROSSING) return -1;
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++) {
    double acc = 0.0, prev = 0.0, pos = (nx - 1) * p->dx;
    int found = 0;
    for (long x = 0; x < nx; x++) {
      double H = 0.0;
      for (int i = 0; i < p->q; i++) H += f[i * n + y * nx + x];
      if (mode == ORC_FRONT_INTEGRAL) {
        const double wx = (x == 0 || x == nx - 1) ? 0.5 : 1.0;
        acc += wx * lf_of_H(H, p->ste, p->tm);
      } else if (!found) {
        const double T = orc_eebm_theta(H, p->ste, p->tm) - p->tm;
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
