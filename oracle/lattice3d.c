/*
 * lattice3d.c -- the IREBM step (Algorithm 3) and the explicit enthalpy
 * step (Algorithm 2) on the 3D lattices D3Q7 and D3Q19.  TEST
 * INFRASTRUCTURE ONLY: see oracle.h.
 *
 * The enthalpy formulation (eq. eq-H) holds in any dimension (Section 2)
 * and the schemes are written for a DdQq lattice with its standard
 * weights, whose second moment must be T/3 times the identity for the
 * tau relation of Section 5 (eq. lambda2).  On D3Q19 these are 1/3 (rest),
 * 1/18 (the six faces) and 1/36 (the twelve edges); on D3Q7 the faces
 * must weigh 1/6 each, which leaves the rest population a weight of 0.
 *
 * The closures of Section 4.2 extend wall by wall as in 2D; the six walls
 * are taken in the order x-, x+, y-, y+, z-, z+:
 *   1. bounce-back q_i = q_opp(i) for an unknown whose source lies beyond
 *      bounce-back walls only, when the opposite is known;
 *   2. on a Dirichlet node (the first Dirichlet wall in the order above
 *      gives the temperature), M0(q) is fixed to the scheme's target
 *      (IREBM: T_D + (phi(T_D) - phi(T(x)))/Ste, eq. Dir_on_q; EEBM: the
 *      wall enthalpy T_D + l(T_D)/Ste), the deficit shared by weight
 *      among the remaining unknowns;
 *   3. on a Neumann node (eq. Neu_on_q), M0(q) is set to M0 of the pulled
 *      populations at the mirror node, one cell inward across every
 *      Neumann wall the node lies on, shared the same way;
 *   4. anything left takes the node's own Omega_opp(i).
 *
 * State: f[i][z][y][x] (x fastest).  Walls hold constant temperatures.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Velocities: rest; faces +x, +y, +z, -x, -y, -z; edges (1,1,0),
   (1,-1,0), (1,0,1), (1,0,-1), (0,1,1), (0,1,-1), then the negatives of
   these six in the same order.  D3Q7 is the first seven. */
static const int VEL[19][3] = {
    {0, 0, 0},   {1, 0, 0},   {0, 1, 0},  {0, 0, 1},   {-1, 0, 0},
    {0, -1, 0},  {0, 0, -1},  {1, 1, 0},  {1, -1, 0},  {1, 0, 1},
    {1, 0, -1},  {0, 1, 1},   {0, 1, -1}, {-1, -1, 0}, {-1, 1, 0},
    {-1, 0, -1}, {-1, 0, 1},  {0, -1, -1}, {0, -1, 1}};

typedef struct {
  int q;
  int e[19][3];
  double w[19];
  int opp[19];
} lat3;

/* geometry: node counts (x, y, z), wall kinds and temperatures in the
   order x-, x+, y-, y+, z-, z+ */
typedef struct {
  long n[3];
  int bc[6];
  double wT[6];
} geom;

static int get_lat3(int q, lat3 *L) {
  if (q != 7 && q != 19) return -1;
  L->q = q;
  for (int i = 0; i < q; i++) {
    for (int a = 0; a < 3; a++) L->e[i][a] = VEL[i][a];
    if (q == 7) L->w[i] = i == 0 ? 0.0 : 1.0 / 6.0;
    else L->w[i] = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  for (int i = 0; i < q; i++)
    for (int j = 0; j < q; j++)
      if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] &&
          L->e[j][2] == -L->e[i][2])
        L->opp[i] = j;
  return 0;
}

int orc_lattice3(int q, int *ex, int *ey, int *ez, double *w, int *opp) {
  lat3 L;
  if (get_lat3(q, &L)) return -1;
  for (int i = 0; i < q; i++) {
    ex[i] = L.e[i][0];
    ey[i] = L.e[i][1];
    ez[i] = L.e[i][2];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  return 0;
}

static int check3(const orc_params *p, lat3 *L, geom *g) {
  if (!p || p->dim != 3 || get_lat3(p->q, L)) return -1;
  g->n[0] = p->nx;
  g->n[1] = p->ny;
  g->n[2] = p->nz;
  for (int a = 0; a < 3; a++)
    if (g->n[a] < 3) return -1;
  if (!(p->tau > 0.5) || !(p->ste > 0.0) || !(p->delta > 0.0)) return -1;
  if (!(p->tol > 0.0) || p->max_it < 1) return -1;
  if (p->newton_mode != ORC_SAFEGUARDED && p->newton_mode != ORC_PLAIN)
    return -1;
  if (p->scheme != ORC_IREBM && p->scheme != ORC_EEBM) return -1;
  int neu = 0, bb = 0;
  for (int k = 0; k < 6; k++) {
    g->bc[k] = k < 4 ? p->bc[k] : p->bc_z[k - 4];
    g->wT[k] = k < 4 ? p->wall_T[k] : p->wall_T_z[k - 4];
    if (g->bc[k] < ORC_DIRICHLET || g->bc[k] > ORC_NEUMANN) return -1;
    neu |= g->bc[k] == ORC_NEUMANN;
    bb |= g->bc[k] == ORC_BOUNCEBACK;
    if (k < 4 && p->wall_profile[k]) return -1;
  }
  if (neu && bb) return -1;
  for (int a = 0; a < 3; a++)
    if ((g->bc[2 * a] == ORC_PERIODIC) != (g->bc[2 * a + 1] == ORC_PERIODIC))
      return -1;
  return 0;
}

static long nodes(const geom *g) { return g->n[0] * g->n[1] * g->n[2]; }

static long idx(const geom *g, const long c[3]) {
  return (c[2] * g->n[1] + c[1]) * g->n[0] + c[0];
}

/* the first Dirichlet wall (x-, x+, y-, y+, z-, z+) holding node c, or -1 */
static int dirichlet_wall(const geom *g, const long c[3]) {
  for (int k = 0; k < 6; k++) {
    const int a = k / 2;
    const long edge = (k & 1) ? g->n[a] - 1 : 0;
    if (c[a] == edge && g->bc[k] == ORC_DIRICHLET) return k;
  }
  return -1;
}

/* pull source c - e, wrapped on periodic axes; 0 when outside */
static int source(const geom *g, const long c[3], const int e[3], long s[3]) {
  for (int a = 0; a < 3; a++) {
    long v = c[a] - e[a];
    if (v < 0 || v >= g->n[a]) {
      if (g->bc[2 * a] != ORC_PERIODIC) return 0;
      v = (v + g->n[a]) % g->n[a];
    }
    s[a] = v;
  }
  return 1;
}

/* does the source c - e leave the lattice through bounce-back walls only?
   (a periodic axis wraps and is never left) */
static int leaves_by_bounceback(const geom *g, const long c[3],
                                const int e[3]) {
  for (int a = 0; a < 3; a++) {
    const long v = c[a] - e[a];
    const int k = v < 0 ? 2 * a : (v >= g->n[a] ? 2 * a + 1 : -1);
    if (k >= 0 && g->bc[k] != ORC_BOUNCEBACK && g->bc[k] != ORC_PERIODIC)
      return 0;
  }
  return 1;
}

/* mirror node of c: one cell inward across each Neumann wall it lies on;
   0 when it lies on none */
static int neumann_mirror(const geom *g, const long c[3], long m[3]) {
  int on = 0;
  for (int a = 0; a < 3; a++) {
    m[a] = c[a];
    if (c[a] == 0 && g->bc[2 * a] == ORC_NEUMANN) {
      m[a] = 1;
      on = 1;
    }
    if (c[a] == g->n[a] - 1 && g->bc[2 * a + 1] == ORC_NEUMANN) {
      m[a] = g->n[a] - 2;
      on = 1;
    }
  }
  return on;
}

static double phi(const orc_params *p, double T) {
  return orc_phi(T, p->tm, p->delta);
}

/* sharp liquid fraction of a temperature (EEBM wall enthalpy) and of an
   enthalpy (Section 3.4) */
static double lf_of_T(const orc_params *p, double T) {
  return T > p->tm ? 1.0 : 0.0;
}

static double lf_of_H(const orc_params *p, double H) {
  const double l = p->ste * (H - p->tm);
  return l < 0.0 ? 0.0 : (l > 1.0 ? 1.0 : l);
}

/* share the deficit D - sum(set q) by weight among the unset q */
static void share(const lat3 *L, double D, double *q, int *set,
                  double *fill) {
  double wu = 0.0;
  for (int i = 0; i < L->q; i++) {
    if (set[i]) D -= q[i];
    else wu += L->w[i];
  }
  for (int i = 0; i < L->q; i++)
    if (!set[i]) {
      q[i] = D * (L->w[i] / wu);
      set[i] = 1;
      *fill += q[i];
    }
}

/* pull streaming q_i = omega_i(c - e_i) at node c with the closures of
   the header; theta_c = M0 of the node before the step (IREBM target).
   Adds the closure-set populations to *fill. */
static void pull_close(const orc_params *p, const lat3 *L, const geom *g,
                       const double *omega, const long c[3], double theta_c,
                       double *q, double *fill) {
  const long n = nodes(g), k = idx(g, c);
  int known[19], set[19], nunk = 0;
  for (int i = 0; i < L->q; i++) {
    long s[3];
    known[i] = source(g, c, L->e[i], s);
    q[i] = known[i] ? omega[i * n + idx(g, s)] : 0.0;
    set[i] = known[i];
    nunk += !known[i];
  }
  if (!nunk) return;
  for (int i = 0; i < L->q; i++)
    if (!known[i] && known[L->opp[i]] &&
        leaves_by_bounceback(g, c, L->e[i])) {
      q[i] = q[L->opp[i]];
      set[i] = 1;
      *fill += q[i];
    }
  const int wall = dirichlet_wall(g, c);
  long m[3];
  if (wall >= 0) {
    const double TD = g->wT[wall];
    const double D = p->scheme == ORC_EEBM
                         ? TD + lf_of_T(p, TD) / p->ste
                         : TD + (phi(p, TD) - phi(p, theta_c)) / p->ste;
    share(L, D, q, set, fill);
  } else if (neumann_mirror(g, c, m)) {
    /* every pull source of the mirror is a lattice node: it lies inside
       each Neumann wall of c, c lies on no Dirichlet wall, bounce-back
       walls do not occur beside Neumann ones and periodic axes wrap */
    double D = 0.0;
    for (int i = 0; i < L->q; i++) {
      long s[3] = {m[0], m[1], m[2]};
      source(g, m, L->e[i], s);
      D += omega[i * n + idx(g, s)];
    }
    share(L, D, q, set, fill);
  }
  for (int i = 0; i < L->q; i++)
    if (!set[i]) {
      q[i] = omega[L->opp[i] * n + k];
      *fill += q[i];
    }
}

/* post-collision populations of node c whose destination c + e_i lies
   outside the lattice */
static double outgoing(const lat3 *L, const geom *g, const double *omega,
                       const long c[3]) {
  const long n = nodes(g), k = idx(g, c);
  double s = 0.0;
  for (int i = 1; i < L->q; i++) {
    const int me[3] = {-L->e[i][0], -L->e[i][1], -L->e[i][2]};
    long d[3];
    if (!source(g, c, me, d)) s += omega[i * n + k];
  }
  return s;
}

/* EEBM equilibrium of enthalpy H: w_i Theta(H), rest H - (1 - w_0) Theta */
static void eebm_equilibrium(const orc_params *p, const lat3 *L, double H,
                             double *feq) {
  const double th = orc_eebm_theta(H, p->ste, p->tm);
  for (int i = 1; i < L->q; i++) feq[i] = L->w[i] * th;
  feq[0] = H - (1.0 - L->w[0]) * th;
}

/* collision at every node: IREBM (1 - 1/tau) f + (w/tau) M0(f) (eq.
   def_qi_omegai); EEBM f - (f - f^eq(M0(f)))/tau (Algorithm 2) */
static void collide(const orc_params *p, const lat3 *L, const geom *g,
                    const double *f, double *theta, double *omega) {
  const long n = nodes(g);
  for (long k = 0; k < n; k++) {
    double s = 0.0, feq[19];
    for (int i = 0; i < L->q; i++) s += f[i * n + k];
    theta[k] = s;
    if (p->scheme == ORC_EEBM) eebm_equilibrium(p, L, s, feq);
    else
      for (int i = 0; i < L->q; i++) feq[i] = L->w[i] * s;
    for (int i = 0; i < L->q; i++)
      omega[i * n + k] = f[i * n + k] - (f[i * n + k] - feq[i]) / p->tau;
  }
}

/* one step f -> fout; theta (n) and omega (q n) are work arrays */
static void step3(const orc_params *p, const lat3 *L, const geom *g,
                  const double *f, double *fout, double *theta,
                  double *omega, orc_stats *st, double *fin, double *fo) {
  const long n = nodes(g);
  collide(p, L, g, f, theta, omega);
  long c[3];
  for (c[2] = 0; c[2] < g->n[2]; c[2]++)
    for (c[1] = 0; c[1] < g->n[1]; c[1]++)
      for (c[0] = 0; c[0] < g->n[0]; c[0]++) {
        const long k = idx(g, c);
        double q[19], fill = 0.0;
        pull_close(p, L, g, omega, c, theta[k], q, &fill);
        *fin += fill;
        *fo += outgoing(L, g, omega, c);
        if (p->scheme == ORC_EEBM) {
          for (int i = 0; i < L->q; i++) fout[i * n + k] = q[i];
          continue;
        }
        /* Newton on the local equation, source and update (Algorithm 3) */
        double m0 = 0.0;
        for (int i = 0; i < L->q; i++) m0 += q[i];
        double tn;
        int it, conv;
        orc_newton(m0, theta[k], p->ste, p->tm, p->delta, p->tol, p->max_it,
                   p->newton_mode, &tn, &it, &conv);
        const double pth = phi(p, theta[k]), pnew = phi(p, tn);
        for (int i = 0; i < L->q; i++)
          fout[i * n + k] = q[i] + L->w[i] / p->ste * (pth - pnew);
        if (st) {
          const double r = fabs(tn + pnew / p->ste - (m0 + pth / p->ste));
          if (r > st->max_residual) st->max_residual = r;
          if (it > st->max_it) st->max_it = it;
          if (!conv) st->nonconverged++;
          st->it_hist[it < 32 ? it : 32]++;
        }
      }
}

int orc3_init(const orc_params *p, const double *T0, double *f) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g)) return -1;
  const long n = nodes(&g);
  long c[3];
  for (c[2] = 0; c[2] < g.n[2]; c[2]++)
    for (c[1] = 0; c[1] < g.n[1]; c[1]++)
      for (c[0] = 0; c[0] < g.n[0]; c[0]++) {
        const long k = idx(&g, c);
        const int wall = dirichlet_wall(&g, c);
        const double T = wall >= 0 ? g.wT[wall] : (T0 ? T0[k] : 0.0);
        double feq[19];
        if (p->scheme == ORC_EEBM)
          eebm_equilibrium(p, &L, T + lf_of_T(p, T) / p->ste, feq);
        else
          for (int i = 0; i < L.q; i++) feq[i] = L.w[i] * T;
        for (int i = 0; i < L.q; i++) f[i * n + k] = feq[i];
      }
  return 0;
}

int orc3_step(const orc_params *p, const double *f, double *fout,
              orc_stats *st) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g)) return -1;
  const long n = nodes(&g);
  double *th = malloc(sizeof(double) * n);
  double *om = malloc(sizeof(double) * L.q * n);
  if (!th || !om) {
    free(th);
    free(om);
    return -1;
  }
  double fin = 0.0, fo = 0.0;
  step3(p, &L, &g, f, fout, th, om, st, &fin, &fo);
  if (st) {
    st->flux_in += fin;
    st->flux_out += fo;
  }
  free(th);
  free(om);
  return 0;
}

/* the enthalpy of a node's M0: IREBM T + phi(T)/Ste (eq. eq-H), EEBM H */
static double node_enthalpy(const orc_params *p, double m) {
  return p->scheme == ORC_EEBM ? m : m + phi(p, m) / p->ste;
}

/* compensated (Kahan) sum of the enthalpy over the nodes */
int orc3_energy(const orc_params *p, const double *f, double *E) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g)) return -1;
  const long n = nodes(&g);
  double s = 0.0, c = 0.0;
  for (long k = 0; k < n; k++) {
    double m = 0.0;
    for (int i = 0; i < L.q; i++) m += f[i * n + k];
    const double y = node_enthalpy(p, m) - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  *E = s;
  return 0;
}

int orc3_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
             double *energy_trace, double *flux_trace) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g) || nsteps < 0) return -1;
  const long n = nodes(&g);
  double *h = malloc(sizeof(double) * L.q * n);
  double *th = malloc(sizeof(double) * n);
  double *om = malloc(sizeof(double) * L.q * n);
  if (!h || !th || !om) {
    free(h);
    free(th);
    free(om);
    return -1;
  }
  double *cur = f, *nxt = h;
  if (energy_trace) orc3_energy(p, cur, &energy_trace[0]);
  for (long s = 0; s < nsteps; s++) {
    double fin = 0.0, fo = 0.0;
    step3(p, &L, &g, cur, nxt, th, om, st, &fin, &fo);
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
    if (energy_trace) orc3_energy(p, cur, &energy_trace[s + 1]);
  }
  if (cur != f) memcpy(f, cur, sizeof(double) * L.q * n);
  free(h);
  free(th);
  free(om);
  return 0;
}

int orc3_temperature(const orc_params *p, const double *f, double *T) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g)) return -1;
  const long n = nodes(&g);
  for (long k = 0; k < n; k++) {
    double m = 0.0;
    for (int i = 0; i < L.q; i++) m += f[i * n + k];
    T[k] = p->scheme == ORC_EEBM ? orc_eebm_theta(m, p->ste, p->tm) : m;
  }
  return 0;
}

/* Front of each row along x (rows ordered z-major, then y):
   ORC_FRONT_INTEGRAL, dx * trapezoid sum of the liquid fraction (phi(T),
   EEBM l(H)); ORC_FRONT_CROSSING, the first place from x = 0 where T - T_m
   goes from > 0 to <= 0, linearly interpolated (0 if T(0) <= T_m,
   (nx - 1) dx if T stays above T_m). */
int orc3_front(const orc_params *p, const double *f, int mode, double *xf) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g)) return -1;
  if (mode != ORC_FRONT_INTEGRAL && mode != ORC_FRONT_CROSSING) return -1;
  const long nx = g.n[0], rows = g.n[1] * g.n[2], n = nodes(&g);
  for (long r = 0; r < rows; r++) {
    double acc = 0.0, prev = 0.0, pos = (nx - 1) * p->dx;
    int found = 0;
    for (long x = 0; x < nx; x++) {
      double m = 0.0;
      for (int i = 0; i < L.q; i++) m += f[i * n + r * nx + x];
      if (mode == ORC_FRONT_INTEGRAL) {
        const double wx = (x == 0 || x == nx - 1) ? 0.5 : 1.0;
        acc += wx * (p->scheme == ORC_EEBM ? lf_of_H(p, m) : phi(p, m));
      } else if (!found) {
        const double T =
            (p->scheme == ORC_EEBM ? orc_eebm_theta(m, p->ste, p->tm) : m) -
            p->tm;
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
    xf[r] = mode == ORC_FRONT_INTEGRAL ? p->dx * acc : pos;
  }
  return 0;
}

/* post-collision populations of every node (the GPU state) */
int orc3_collide(const orc_params *p, const double *f, double *omega) {
  lat3 L;
  geom g;
  if (check3(p, &L, &g)) return -1;
  double *th = malloc(sizeof(double) * nodes(&g));
  if (!th) return -1;
  collide(p, &L, &g, f, th, omega);
  free(th);
  return 0;
}
