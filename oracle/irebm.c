/*
 * irebm.c -- the oracle proper (R = double).  TEST INFRASTRUCTURE ONLY:
 * see oracle.h.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define ORC_PI 3.14159265358979323846

#define R double
#define RN(name) r_##name
#ifdef ORC_PHI_LOGISTIC
/* A second rounding of the same function, tanh(z) = 2/(1 + exp(-2z)) - 1,
   built into a separate library (liboracle_alt.so) only to measure how far
   two correct FP64 evaluations of the scheme drift apart on an input. */
#define TANH(z) (2.0 / (1.0 + exp(-2.0 * (z))) - 1.0)
#else
#define TANH(z) tanh(z)
#endif
#define RE(z) (z)
#define CS 0
#include "irebm_body.h"

/* The reverse step below transposes the Dirichlet, bounce-back and
   periodic closures only. */
static int has_neumann(const orc_params *p) {
  for (int k = 0; k < (p->dim == 2 ? 4 : 2); k++)
    if (p->bc[k] == ORC_NEUMANN) return 1;
  return 0;
}

static void fill_vals(const orc_params *p, r_vals *v) {
  v->ste = p->ste;
  v->delta = p->delta;
  for (int k = 0; k < 4; k++) {
    v->wall_T[k] = p->wall_T[k];
    v->wall_profile[k] = p->wall_profile[k];
  }
}

int orc_lattice(int dim, int q, int *ex, int *ey, double *w, int *opp) {
  r_lat L;
  if (r_get_lat(dim, q, &L)) return -1;
  for (int i = 0; i < q; i++) {
    ex[i] = L.ex[i];
    ey[i] = L.ey[i];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  return 0;
}

double orc_phi(double theta, double tm, double delta) {
  return r_phi_(theta, tm, delta);
}

double orc_dphi(double theta, double tm, double delta) {
  return r_dphi_(theta, tm, delta);
}

int orc_newton(double m0, double theta, double ste, double tm, double delta,
               double tol, int max_it, int mode, double *theta_new,
               int *iters, int *converged) {
  if (!(ste > 0) || !(delta > 0) || !(tol > 0) || max_it < 1) return -1;
  *theta_new = r_newton_(m0, theta, ste, tm, delta, tol, max_it, mode, iters,
                         converged, 0);
  return 0;
}

int orc_init(const orc_params *p, const double *T0, double *f) {
  if (r_check(p)) return -1;
  r_vals v;
  fill_vals(p, &v);
  r_init_(p, &v, T0, f);
  return 0;
}

int orc_step(const orc_params *p, const double *f, double *fout,
             orc_stats *st) {
  if (r_check(p)) return -1;
  const long n = p->nx * p->ny;
  double *th = malloc(sizeof(double) * n);
  double *om = malloc(sizeof(double) * p->q * n);
  if (!th || !om) {
    free(th);
    free(om);
    return -1;
  }
  r_vals v;
  fill_vals(p, &v);
  double fin = 0.0, fo = 0.0;
  r_step_(p, &v, f, fout, th, om, st, &fin, &fo);
  if (st) {
    st->flux_in += fin;
    st->flux_out += fo;
  }
  free(th);
  free(om);
  return 0;
}

/* Compensated (Kahan) sum of E = sum_x [T + phi(T)/Ste] (eq. eq-H). */
int orc_energy(const orc_params *p, const double *f, double *E) {
  if (r_check(p)) return -1;
  const long n = p->nx * p->ny;
  double s = 0.0, c = 0.0;
  for (long k = 0; k < n; k++) {
    double T = 0.0;
    for (int i = 0; i < p->q; i++) T += f[i * n + k];
    double h = T + r_phi_(T, p->tm, p->delta) / p->ste;
    double y = h - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  *E = s;
  return 0;
}

int orc_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
            double *energy_trace, double *flux_trace) {
  if (r_check(p) || nsteps < 0) return -1;
  const long n = p->nx * p->ny;
  double *g = malloc(sizeof(double) * p->q * n);
  double *th = malloc(sizeof(double) * n);
  double *om = malloc(sizeof(double) * p->q * n);
  if (!g || !th || !om) {
    free(g);
    free(th);
    free(om);
    return -1;
  }
  r_vals v;
  fill_vals(p, &v);
  double *cur = f, *nxt = g;
  if (energy_trace) orc_energy(p, cur, &energy_trace[0]);
  for (long s = 0; s < nsteps; s++) {
    double fin = 0.0, fo = 0.0;
    r_step_(p, &v, cur, nxt, th, om, st, &fin, &fo);
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
    if (energy_trace) orc_energy(p, cur, &energy_trace[s + 1]);
  }
  if (cur != f) memcpy(f, cur, sizeof(double) * p->q * n);
  free(g);
  free(th);
  free(om);
  return 0;
}

int orc_temperature(const orc_params *p, const double *f, double *T) {
  if (r_check(p)) return -1;
  const long n = p->nx * p->ny;
  for (long k = 0; k < n; k++) {
    double s = 0.0;
    for (int i = 0; i < p->q; i++) s += f[i * n + k];
    T[k] = s;
  }
  return 0;
}

/*
 * Front position per row.  ORC_FRONT_INTEGRAL: dx * trapezoid sum of the
 * liquid fraction phi(T) along x.  ORC_FRONT_CROSSING: first place, from
 * x = 0, where T - tm changes from > 0 to <= 0, linearly interpolated;
 * 0 if T(0) <= tm, (nx-1) dx if T stays above tm.
 */
int orc_front(const orc_params *p, const double *f, int mode, double *xf) {
  if (r_check(p)) return -1;
  if (mode == ORC_FRONT_INTEGRAL) {
    r_vals v;
    fill_vals(p, &v);
    r_front_integral_(p, &v, f, xf);
    return 0;
  }
  if (mode != ORC_FRONT_CROSSING) return -1;
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  double *T = malloc(sizeof(double) * nx);
  if (!T) return -1;
  for (long y = 0; y < ny; y++) {
    for (long x = 0; x < nx; x++) {
      double s = 0.0;
      for (int i = 0; i < p->q; i++) s += f[i * n + y * nx + x];
      T[x] = s - p->tm;
    }
    double pos = (nx - 1) * p->dx;
    if (T[0] <= 0.0) {
      pos = 0.0;
    } else {
      for (long x = 0; x + 1 < nx; x++)
        if (T[x] > 0.0 && T[x + 1] <= 0.0) {
          pos = p->dx * (x + T[x] / (T[x] - T[x + 1]));
          break;
        }
    }
    xf[y] = pos;
  }
  free(T);
  return 0;
}

/*
 * Root lambda of the transcendental equation (eq. eq-Stefan-lambda) for
 * equal phase properties (rho = k = alpha = 1):
 *   exp(-l^2)/erf(l) + theta0 exp(-l^2)/erfc(l) = l sqrt(pi)/Ste.
 * The left side minus the right side decreases from +inf; bisection with
 * 200 halvings on a bracket grown from [1e-12, 1].
 */
static double stefan_g(double l, double ste, double theta0) {
  return exp(-l * l) / erf(l) + theta0 * exp(-l * l) / erfc(l) -
         l * sqrt(ORC_PI) / ste;
}

int orc_stefan_lambda(double ste, double theta0, double *lambda) {
  if (!(ste > 0) || !(theta0 <= 0)) return -1;
  double a = 1e-12, b = 1.0;
  while (stefan_g(b, ste, theta0) > 0.0) {
    b *= 2.0;
    if (b > 20.0) return -1;
  }
  for (int k = 0; k < 200; k++) {
    double m = 0.5 * (a + b);
    if (stefan_g(m, ste, theta0) > 0.0) a = m;
    else b = m;
  }
  *lambda = 0.5 * (a + b);
  return 0;
}

/* Neumann similarity solution (eq. eq-exact-sol), equal properties:
   liquid 1 - erf(x/2sqrt t)/erf(l) for x < 2 l sqrt t, solid
   theta0 - theta0 erfc(x/2sqrt t)/erfc(l) beyond. */
double orc_neumann_T(double x, double t, double lambda, double theta0) {
  double z = x / (2.0 * sqrt(t));
  if (z < lambda) return 1.0 - erf(z) / erf(lambda);
  return theta0 - theta0 * erfc(z) / erfc(lambda);
}

int orc_front_loss(const orc_params *p, const double *T0, long nsteps,
                   const double *target, double *loss) {
  if (r_check(p) || nsteps < 0 || !target || !loss) return -1;
  r_vals v;
  fill_vals(p, &v);
  return r_front_loss_(p, &v, T0, nsteps, target, loss);
}

/*
 * ---- Reverse mode ------------------------------------------------------
 * Adjoint of one step f -> f' at state f, given gbar = dL/df'.  The Newton
 * root is differentiated by the implicit-function theorem: with
 * R(t) = t + phi(t)/Ste - m0 - phi(theta)/Ste = 0 and J = 1 + phi'(t~)/Ste,
 *   dt~/dm0 = 1/J, dt~/dtheta = (phi'(theta)/Ste)/J,
 *   dt~/dSte = (phi(t~) - phi(theta))/(Ste^2 J),
 *   dt~/ddelta = -(dphi/ddelta(t~) - dphi/ddelta(theta))/(Ste J),
 * exact at converged nodes.  dphi/ddelta(t) = -((t - tm)/delta) phi'(t).
 * Writes fbar = dL/df and adds to g_wall (x- wall profile, per row),
 * *g_ste and *g_delta.
 */
static double dphi_ddelta(double t, double tm, double delta) {
  return -((t - tm) / delta) * r_dphi_(t, tm, delta);
}

static void adj_step(const orc_params *p, const r_vals *v, const double *f,
                     const double *gbar, double *fbar, double *th,
                     double *om, double *omb, double *thb, double *g_wall,
                     double *g_ste, double *g_delta) {
  r_lat L;
  r_get_lat(p->dim, p->q, &L);
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  const double tau = p->tau, S = v->ste, dl = v->delta, tm = p->tm;
  /* forward quantities of this step */
  for (long k = 0; k < n; k++) {
    double s = 0.0;
    for (int i = 0; i < p->q; i++) s += f[i * n + k];
    th[k] = s;
  }
  for (int i = 0; i < p->q; i++)
    for (long k = 0; k < n; k++)
      om[i * n + k] = (1.0 - 1.0 / tau) * f[i * n + k] + L.w[i] * th[k] / tau;
  memset(omb, 0, sizeof(double) * p->q * n);
  memset(thb, 0, sizeof(double) * n);
  double Sb = 0.0, db = 0.0;
  for (long y = 0; y < ny; y++)
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      double q[9], qb[9], fill;
      int known[9], it, conv;
      r_pull_close(p, v, &L, om, th, x, y, q, known, &fill);
      double m0 = 0.0;
      for (int i = 0; i < p->q; i++) m0 += q[i];
      double tn = r_newton_(m0, th[k], S, tm, dl, p->tol, p->max_it,
                            p->newton_mode, &it, &conv, 0);
      double P = r_phi_(th[k], tm, dl), Pt = r_phi_(tn, tm, dl);
      double d = r_dphi_(th[k], tm, dl), dt = r_dphi_(tn, tm, dl);
      double Pd = dphi_ddelta(th[k], tm, dl), Ptd = dphi_ddelta(tn, tm, dl);
      /* f'_i = q_i + w_i s,  s = (P - Pt)/S */
      double sb = 0.0;
      for (int i = 0; i < p->q; i++) {
        qb[i] = gbar[i * n + k];
        sb += L.w[i] * gbar[i * n + k];
      }
      double thl = sb / S * d;
      double tnb = -sb / S * dt;
      Sb += -sb * (P - Pt) / (S * S);
      db += sb / S * (Pd - Ptd);
      /* Newton root, implicit function theorem */
      double J = 1.0 + dt / S;
      double m0b = tnb / J;
      thl += tnb * (d / S) / J;
      Sb += tnb * (Pt - P) / (S * S * J);
      db += -tnb * (Ptd - Pd) / (S * J);
      for (int i = 0; i < p->q; i++) qb[i] += m0b;
      /* boundary closures, reversed: 3 (own Omega), 2 (Dirichlet deficit),
         1 (bounce-back from a known opposite) */
      int nunk = 0, bb[9], set[9];
      for (int i = 0; i < p->q; i++) {
        nunk += !known[i];
        bb[i] = !known[i] && known[L.opp[i]] &&
                r_leaves_by_bounceback(p, x, y, L.ex[i], L.ey[i]);
        set[i] = known[i] || bb[i];
      }
      if (nunk) {
        int wall = r_dirichlet_wall(p, x, y);
        if (wall >= 0) {
          double wu = 0.0, Db = 0.0;
          for (int i = 0; i < p->q; i++)
            if (!set[i]) wu += L.w[i];
          for (int i = 0; i < p->q; i++)
            if (!set[i]) Db += qb[i] * (L.w[i] / wu);
          for (int i = 0; i < p->q; i++)
            if (set[i]) qb[i] -= Db;
          double TD = r_wall_value(v, wall, x, y);
          if (wall == 0 && g_wall)
            g_wall[y] += Db * (1.0 + r_dphi_(TD, tm, dl) / S);
          thl += -Db * d / S;
          Sb += -Db * (r_phi_(TD, tm, dl) - P) / (S * S);
          db += Db * (dphi_ddelta(TD, tm, dl) - Pd) / S;
        } else {
          for (int i = 0; i < p->q; i++)
            if (!set[i]) omb[L.opp[i] * n + k] += qb[i];
        }
        for (int i = 0; i < p->q; i++)
          if (bb[i]) qb[L.opp[i]] += qb[i];
      }
      /* streaming: q_i(x) = Omega_i(x - e_i) */
      for (int i = 0; i < p->q; i++)
        if (known[i]) {
          long sx = 0, sy = 0;
          r_source(p, x, y, L.ex[i], L.ey[i], &sx, &sy);
          omb[(i * ny + sy) * nx + sx] += qb[i];
        }
      thb[k] += thl;
    }
  /* collision Omega_i = (1 - 1/tau) f_i + w_i theta/tau, theta = M0(f) */
  for (long k = 0; k < n; k++) {
    double s = 0.0;
    for (int i = 0; i < p->q; i++) s += L.w[i] / tau * omb[i * n + k];
    thb[k] += s;
  }
  for (int i = 0; i < p->q; i++)
    for (long k = 0; k < n; k++)
      fbar[i * n + k] = (1.0 - 1.0 / tau) * omb[i * n + k] + thb[k];
  *g_ste += Sb;
  *g_delta += db;
}

int orc_adjoint_step(const orc_params *p, const double *f,
                     const double *gbar, double *fbar, double *g_wall,
                     double *g_ste, double *g_delta) {
  if (r_check(p) || has_neumann(p)) return -1;
  const long n = p->nx * p->ny;
  double *th = malloc(sizeof(double) * n), *thb = malloc(sizeof(double) * n);
  double *om = malloc(sizeof(double) * p->q * n);
  double *omb = malloc(sizeof(double) * p->q * n);
  if (!th || !thb || !om || !omb) {
    free(th); free(thb); free(om); free(omb);
    return -1;
  }
  r_vals v;
  fill_vals(p, &v);
  adj_step(p, &v, f, gbar, fbar, th, om, omb, thb, g_wall, g_ste, g_delta);
  free(th); free(thb); free(om); free(omb);
  return 0;
}

/*
 * Gradient of the front misfit loss.  Stores every forward state (the
 * oracle is meant for small lattices), then runs the reverse steps.
 * Seeds: dL/df_j(x,y) = (xf(y) - target(y)) dx w_x phi'(T(x,y)) for every
 * j, plus the delta-dependence of the front itself.  The initial state
 * sets x- wall nodes to w_i T_w(y), which adds sum_i w_i fbar_i there.
 */
int orc_front_loss_grad(const orc_params *p, const double *T0, long nsteps,
                        const double *target, double *loss, double *g_wall,
                        double *g_ste, double *g_delta) {
  if (r_check(p) || has_neumann(p) || nsteps < 0 || !target) return -1;
  const long nx = p->nx, ny = p->ny, n = nx * ny, qn = p->q * n;
  double *F = malloc(sizeof(double) * qn * (nsteps + 1));
  double *gb = malloc(sizeof(double) * qn), *fb = malloc(sizeof(double) * qn);
  double *th = malloc(sizeof(double) * n), *thb = malloc(sizeof(double) * n);
  double *om = malloc(sizeof(double) * qn), *omb = malloc(sizeof(double) * qn);
  double *xf = malloc(sizeof(double) * ny);
  if (!F || !gb || !fb || !th || !thb || !om || !omb || !xf) {
    free(F); free(gb); free(fb); free(th); free(thb); free(om); free(omb);
    free(xf);
    return -1;
  }
  r_vals v;
  fill_vals(p, &v);
  r_init_(p, &v, T0, F);
  double fin = 0.0, fo = 0.0;
  for (long s = 0; s < nsteps; s++)
    r_step_(p, &v, F + s * qn, F + (s + 1) * qn, th, om, 0, &fin, &fo);
  const double *fN = F + nsteps * qn;
  r_front_integral_(p, &v, fN, xf);
  double Lsum = 0.0, gs = 0.0, gd = 0.0;
  for (long y = 0; y < ny; y++) Lsum += 0.5 * (xf[y] - target[y]) * (xf[y] - target[y]);
  if (g_wall) memset(g_wall, 0, sizeof(double) * ny);
  for (long y = 0; y < ny; y++) {
    double r = xf[y] - target[y];
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      double T = 0.0;
      for (int i = 0; i < p->q; i++) T += fN[i * n + k];
      double wx = (x == 0 || x == nx - 1) ? 0.5 : 1.0;
      double gT = r * p->dx * wx * r_dphi_(T, p->tm, p->delta);
      for (int i = 0; i < p->q; i++) gb[i * n + k] = gT;
      gd += r * p->dx * wx * dphi_ddelta(T, p->tm, p->delta);
    }
  }
  for (long s = nsteps - 1; s >= 0; s--) {
    adj_step(p, &v, F + s * qn, gb, fb, th, om, omb, thb, g_wall, &gs, &gd);
    double *t = gb; gb = fb; fb = t;
  }
  /* initial state: f_i = w_i T_w(y) at x- Dirichlet wall nodes */
  if (g_wall && p->bc[0] == ORC_DIRICHLET) {
    r_lat L;
    r_get_lat(p->dim, p->q, &L);
    for (long y = 0; y < ny; y++) {
      double s = 0.0;
      for (int i = 0; i < p->q; i++) s += L.w[i] * gb[i * n + y * nx];
      g_wall[y] += s;
    }
  }
  *loss = Lsum;
  *g_ste = gs;
  *g_delta = gd;
  free(F); free(gb); free(fb); free(th); free(thb); free(om); free(omb);
  free(xf);
  return 0;
}
