/*
 * irebm_body.h -- the IREBM time step of the oracle, written once over a
 * scalar type R.  irebm.c includes it with R = double (the oracle proper);
 * irebm_cs.c includes it with R = double complex so that a complex-step
 * derivative runs exactly the same arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Required macros: R, RN(name) (name mangling), TANH(z), RE(z) (real
 * part), CS (1 in the complex-step build).
 *
 * The step follows the paper's Algorithm 3 (Section 4.1) in its order:
 *   moments, equilibrium, collision (def. of Omega_i), streaming
 *   q_i = Omega_i(x - e_i), Newton on the local scalar equation for the
 *   new temperature, source term g_i, update f~_i = q_i + g_i,
 * with the boundary closures on q of Section 4.2.
 */

/* Parameters that a complex-step run perturbs. */
typedef struct {
  R ste, delta;
  R wall_T[4];
  const R *wall_profile[4];
} RN(vals);

/* Regularized liquid fraction, Section 4.1: 1/2 (1 + tanh(theta/delta)),
   centred on the melting temperature tm. */
static R RN(phi_)(R th, R tm, R delta) {
  return 0.5 * (1.0 + TANH((th - tm) / delta));
}

/* Its derivative: (1 - tanh^2)/(2 delta). */
static R RN(dphi_)(R th, R tm, R delta) {
  R t = TANH((th - tm) / delta);
  return (1.0 - t * t) / (2.0 * delta);
}

/*
 * Newton solve of the local equation (eq. rhs_fl_2):
 *   theta~ = M0(q) + (phi(theta) - phi(theta~)) / Ste,
 * i.e. F(t) = t + phi(t)/Ste - c = 0 with c = m0 + phi(theta)/Ste,
 * started from theta^(0) = theta as in Algorithm 3.
 *
 * ORC_PLAIN uses the paper's update formula as printed.  It can cycle
 * between the solid and liquid plateaus when 1/Ste is large against delta.
 *
 * ORC_SAFEGUARDED (the default) takes the same Newton step inside the
 * safeguard of "rtsafe" (Press et al., Numerical Recipes, sec. 9.4): keep
 * a bracket [a, b] of the root and bisect it whenever the Newton step
 * leaves the bracket or is not less than half the step before the last.
 * F is strictly increasing (F' >= 1) and 0 <= phi <= 1, so
 * F(c - 1/Ste) <= 0 <= F(c): the root is unique and [c - 1/Ste, c]
 * brackets it.  In the quadratic phase every Newton step is kept, so the
 * iterates are those of the plain method.
 *
 * Stops when |theta^(k+1) - theta^(k)| <= tol, then takes one more
 * Newton step (below); *iters counts the candidates before it.
 */
static R RN(newton_)(R m0, R th, R ste, R tm, R delta, double tol,
                     int max_it, int mode, int *iters, int *conv,
                     long *bis) {
  R phth = RN(phi_)(th, tm, delta);
  R c = m0 + phth / ste;
  R a = c - 1.0 / ste, b = c;
  double dx = RE(b - a), dxold = dx;
  R cur = th, cand = th;
  int k = 0;
  *conv = 0;
  while (k < max_it) {
    R ph = RN(phi_)(cur, tm, delta);
    R dph = RN(dphi_)(cur, tm, delta);
    if (mode == ORC_PLAIN) {
      cand = (m0 + phth / ste + dph * cur / ste - ph / ste) /
             (1.0 + dph / ste);
    } else {
      R F = cur + ph / ste - c;
      if (RE(F) < 0.0) a = cur;
      else if (RE(F) > 0.0) b = cur;
      R stp = F / (1.0 + dph / ste);
      cand = cur - stp;
      if (RE(cand) < RE(a) || RE(cand) > RE(b) ||
          2.0 * fabs(RE(stp)) > fabs(dxold)) {
        cand = 0.5 * (a + b);
        dxold = dx;
        dx = 0.5 * RE(b - a);
        if (bis) (*bis)++;
      } else {
        dxold = dx;
        dx = RE(stp);
      }
    }
    k++;
    if (fabs(RE(cand) - RE(cur)) <= tol) {
      *conv = 1;
      break;
    }
    cur = cand;
  }
  *iters = k;
  /* A solve that stops on a bisection step is only within tol of the
     root.  One more Newton step from the converged iterate returns the
     root itself to rounding (error ~ tol^2 F''/F'), so the result does
     not depend on the path the safeguard took; in the complex-step build
     it also makes the imaginary part the implicit-function derivative. */
  if (*conv) {
    R ph = RN(phi_)(cand, tm, delta);
    R dph = RN(dphi_)(cand, tm, delta);
    cand = cand - (cand + ph / ste - c) / (1.0 + dph / ste);
  }
  return cand;
}

/* Lattice tables (Section 3.2, "standard weights"): rest velocity first,
   then +x, +y, -x, -y, then the diagonals.  Weights give the second
   moment (1/3) theta I required by the Chapman-Enskog analysis. */
static const int RN(EX3)[3] = {0, 1, -1};
static const double RN(W3)[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
static const int RN(O3)[3] = {0, 2, 1};
static const int RN(EX5)[5] = {0, 1, 0, -1, 0};
static const int RN(EY5)[5] = {0, 0, 1, 0, -1};
static const double RN(W5)[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0,
                                 1.0 / 6.0, 1.0 / 6.0};
static const int RN(O5)[5] = {0, 3, 4, 1, 2};
static const int RN(EX9)[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int RN(EY9)[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double RN(W9)[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                 1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int RN(O9)[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const int RN(ZERO9)[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

typedef struct {
  const int *ex, *ey, *opp;
  const double *w;
} RN(lat);

static int RN(get_lat)(int dim, int q, RN(lat) *L) {
  if (dim == 1 && q == 3) {
    L->ex = RN(EX3); L->ey = RN(ZERO9); L->w = RN(W3); L->opp = RN(O3);
  } else if (dim == 2 && q == 5) {
    L->ex = RN(EX5); L->ey = RN(EY5); L->w = RN(W5); L->opp = RN(O5);
  } else if (dim == 2 && q == 9) {
    L->ex = RN(EX9); L->ey = RN(EY9); L->w = RN(W9); L->opp = RN(O9);
  } else {
    return -1;
  }
  return 0;
}

static int RN(check)(const orc_params *p) {
  RN(lat) L;
  if (!p || RN(get_lat)(p->dim, p->q, &L)) return -1;
  if (p->nx < 3 || p->ny < 1 || (p->dim == 1 && p->ny != 1)) return -1;
  if (p->dim == 2 && p->ny < 3) return -1;
  if (!(p->tau > 0.5) || !(p->ste > 0.0) || !(p->delta > 0.0)) return -1;
  if (!(p->tol > 0.0) || p->max_it < 1) return -1;
  if (p->newton_mode != ORC_SAFEGUARDED && p->newton_mode != ORC_PLAIN)
    return -1;
  int neu = 0, bb = 0;
  for (int k = 0; k < 4; k++) {
    if (p->bc[k] < ORC_DIRICHLET || p->bc[k] > ORC_NEUMANN) return -1;
    if (p->dim == 2 || k < 2) {
      neu |= p->bc[k] == ORC_NEUMANN;
      bb |= p->bc[k] == ORC_BOUNCEBACK;
    }
  }
  if (neu && bb) return -1;
  if ((p->bc[0] == ORC_PERIODIC) != (p->bc[1] == ORC_PERIODIC)) return -1;
  if (p->dim == 2 && (p->bc[2] == ORC_PERIODIC) != (p->bc[3] == ORC_PERIODIC))
    return -1;
  return 0;
}

/* Dirichlet wall holding node (x, y), or -1.  Where two Dirichlet walls
   meet, the first in the order x-, x+, y-, y+ gives the temperature. */
static int RN(dirichlet_wall)(const orc_params *p, long x, long y) {
  if (x == 0 && p->bc[0] == ORC_DIRICHLET) return 0;
  if (x == p->nx - 1 && p->bc[1] == ORC_DIRICHLET) return 1;
  if (p->dim == 2 && y == 0 && p->bc[2] == ORC_DIRICHLET) return 2;
  if (p->dim == 2 && y == p->ny - 1 && p->bc[3] == ORC_DIRICHLET) return 3;
  return -1;
}

static R RN(wall_value)(const RN(vals) *v, int wall, long x, long y) {
  if (v->wall_profile[wall]) return v->wall_profile[wall][wall < 2 ? y : x];
  return v->wall_T[wall];
}

/* Mirror node of a node on Neumann walls (Section 4.2, eq. Neu_on_q):
   the node moved one cell inward across each Neumann wall it lies on
   (at the corner of two, the diagonal neighbour).  Returns 0 when the
   node lies on no Neumann wall. */
static int RN(neumann_mirror)(const orc_params *p, long x, long y, long *mx,
                              long *my) {
  long dx = 0, dy = 0;
  if (x == 0 && p->bc[0] == ORC_NEUMANN) dx = 1;
  if (x == p->nx - 1 && p->bc[1] == ORC_NEUMANN) dx = -1;
  if (p->dim == 2 && y == 0 && p->bc[2] == ORC_NEUMANN) dy = 1;
  if (p->dim == 2 && y == p->ny - 1 && p->bc[3] == ORC_NEUMANN) dy = -1;
  if (dx == 0 && dy == 0) return 0;
  *mx = x + dx;
  *my = y + dy;
  return 1;
}

/* Source node of the pull x - e_i, wrapped on periodic axes.  Returns 0
   when it lies outside the lattice. */
static int RN(source)(const orc_params *p, long x, long y, int ex, int ey,
                      long *sx, long *sy) {
  long a = x - ex, b = y - ey;
  if (a < 0 || a >= p->nx) {
    if (p->bc[0] != ORC_PERIODIC) return 0;
    a = (a + p->nx) % p->nx;
  }
  if (b < 0 || b >= p->ny) {
    if (p->bc[2] != ORC_PERIODIC) return 0;
    b = (b + p->ny) % p->ny;
  }
  *sx = a;
  *sy = b;
  return 1;
}

/* Does the pull source x - e_i of node (x, y) leave the lattice only
   through bounce-back walls?  (Periodic axes wrap and are never left.) */
static int RN(leaves_by_bounceback)(const orc_params *p, long x, long y,
                                    int ex, int ey) {
  long a = x - ex, b = y - ey;
  /* a periodic axis wraps: crossing its seam leaves nothing */
  if (a < 0 && p->bc[0] != ORC_BOUNCEBACK && p->bc[0] != ORC_PERIODIC)
    return 0;
  if (a >= p->nx && p->bc[1] != ORC_BOUNCEBACK && p->bc[1] != ORC_PERIODIC)
    return 0;
  if (b < 0 && p->bc[2] != ORC_BOUNCEBACK && p->bc[2] != ORC_PERIODIC)
    return 0;
  if (b >= p->ny && p->bc[3] != ORC_BOUNCEBACK && p->bc[3] != ORC_PERIODIC)
    return 0;
  return 1;
}

/*
 * Streaming and boundary closure at one node: fills q[i] = Omega_i(x-e_i)
 * where the source is a lattice node, then closes the unknown q_i.
 *   1. Bounce-back (Section 4.2): an unknown whose source lies beyond
 *      bounce-back walls only takes q_i = q_opp(i) when that opposite
 *      population is known.
 *   2. Dirichlet node (Section 4.2, eq. Dir_on_q): the zeroth moment must
 *      be M0(q) = T_D + (phi(T_D) - phi(theta(x)))/Ste, which makes the new
 *      temperature equal T_D.  The deficit D = (M0 target) - (sum of the
 *      q_i known so far) is shared among the remaining unknowns in
 *      proportion to w_i (for D1Q3 and flat D2Q5 walls there is one such
 *      unknown and it takes all of D).
 *   3. Neumann node (Section 4.2, eq. Neu_on_q): M0(q) must equal M0(q)
 *      at the mirror node (the interior neighbour across the Neumann
 *      walls, neumann_mirror), whose pulled populations are all known;
 *      the deficit is shared among the unknowns in proportion to w_i
 *      (one unknown on flat D2Q5 and D1Q3 walls: eq. Neu_on_q itself).
 *   4. Any unknown still left (corner of two bounce-back walls, where the
 *      opposite is unknown too) takes the node's own post-collision
 *      population Omega_opp(i)(x).
 * Reports the closure-filled sum to *fill.
 */
static void RN(pull_close)(const orc_params *p, const RN(vals) *v,
                           const RN(lat) *L, const R *omega, const R *theta,
                           long x, long y, R *q, int *known, R *fill) {
  const long nx = p->nx, ny = p->ny, n = y * nx + x;
  int nunk = 0, set[9];
  for (int i = 0; i < p->q; i++) {
    long sx, sy;
    known[i] = RN(source)(p, x, y, L->ex[i], L->ey[i], &sx, &sy);
    q[i] = known[i] ? omega[(i * ny + sy) * nx + sx] : 0.0;
    set[i] = known[i];
    if (!known[i]) nunk++;
  }
  *fill = 0.0;
  if (nunk == 0) return;
  for (int i = 0; i < p->q; i++)
    if (!known[i] && known[L->opp[i]] &&
        RN(leaves_by_bounceback)(p, x, y, L->ex[i], L->ey[i])) {
      q[i] = q[L->opp[i]];
      set[i] = 1;
      *fill += q[i];
    }
  int wall = RN(dirichlet_wall)(p, x, y);
  if (wall >= 0) {
    R TD = RN(wall_value)(v, wall, x, y);
    R target = TD + (RN(phi_)(TD, p->tm, v->delta) -
                     RN(phi_)(theta[n], p->tm, v->delta)) / v->ste;
    R D = target;
    double wu = 0.0;
    for (int i = 0; i < p->q; i++) {
      if (set[i]) D -= q[i];
      else wu += L->w[i];
    }
    for (int i = 0; i < p->q; i++)
      if (!set[i]) {
        q[i] = D * (L->w[i] / wu);
        set[i] = 1;
        *fill += q[i];
      }
  }
  long mx, my;
  if (wall < 0 && RN(neumann_mirror)(p, x, y, &mx, &my)) {
    /* every pull of the mirror is a lattice node: the mirror is one cell
       inside each Neumann wall of the node, and check() admits no
       bounce-back wall beside a Neumann one (periodic axes wrap) */
    R D = 0.0;
    for (int i = 0; i < p->q; i++) {
      long sx = mx, sy = my;
      RN(source)(p, mx, my, L->ex[i], L->ey[i], &sx, &sy);
      D += omega[(i * ny + sy) * nx + sx];
    }
    double wu = 0.0;
    for (int i = 0; i < p->q; i++) {
      if (set[i]) D -= q[i];
      else wu += L->w[i];
    }
    for (int i = 0; i < p->q; i++)
      if (!set[i]) {
        q[i] = D * (L->w[i] / wu);
        set[i] = 1;
        *fill += q[i];
      }
  }
  for (int i = 0; i < p->q; i++)
    if (!set[i]) {
      int o = L->opp[i];
      q[i] = omega[(o * ny + y) * nx + x];
      *fill += q[i];
    }
}

/* Sum of post-collision populations at node (x, y) whose destination
   x + e_i lies outside the lattice. */
static R RN(outgoing)(const orc_params *p, const RN(lat) *L, const R *omega,
                      long x, long y) {
  R s = 0.0;
  for (int i = 1; i < p->q; i++) {
    long dx_, dy_;
    if (!RN(source)(p, x, y, -L->ex[i], -L->ey[i], &dx_, &dy_))
      s += omega[(i * p->ny + y) * p->nx + x];
  }
  return s;
}

/*
 * One IREBM step f -> fout (Algorithm 3).  theta and omega are work
 * arrays of n and q*n values.  Accumulates statistics into st and the
 * boundary fluxes into *fin, *fout_flux.
 */
static void RN(step_)(const orc_params *p, const RN(vals) *v, const R *f,
                      R *fout, R *theta, R *omega, orc_stats *st, R *fin,
                      R *fo) {
  RN(lat) L;
  RN(get_lat)(p->dim, p->q, &L);
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  const double tau = p->tau;
  /* moments: theta = M0(f) */
  for (long k = 0; k < n; k++) {
    R s = 0.0;
    for (int i = 0; i < p->q; i++) s += f[i * n + k];
    theta[k] = s;
  }
  /* equilibrium w_i theta and BGK collision */
  for (int i = 0; i < p->q; i++)
    for (long k = 0; k < n; k++) {
      R feq = L.w[i] * theta[k];
      omega[i * n + k] = (1.0 - 1.0 / tau) * f[i * n + k] + feq / tau;
    }
  for (long y = 0; y < ny; y++)
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      R q[9], fill;
      int known[9];
      /* streaming q_i = Omega_i(x - e_i) and boundary closure */
      RN(pull_close)(p, v, &L, omega, theta, x, y, q, known, &fill);
      *fin += fill;
      *fo += RN(outgoing)(p, &L, omega, x, y);
      /* Newton initialization m0 = M0(q), theta^(0) = theta */
      R m0 = 0.0;
      for (int i = 0; i < p->q; i++) m0 += q[i];
      int it, conv;
      R tn = RN(newton_)(m0, theta[k], v->ste, p->tm, v->delta, p->tol,
                         p->max_it, p->newton_mode, &it, &conv,
                         st ? &st->bisections : 0);
      /* source term g_i = w_i/Ste (phi(theta) - phi(theta~)) and update */
      R pth = RN(phi_)(theta[k], p->tm, v->delta);
      R pnew = RN(phi_)(tn, p->tm, v->delta);
      for (int i = 0; i < p->q; i++) {
        R g = L.w[i] / v->ste * (pth - pnew);
        fout[i * n + k] = q[i] + g;
      }
      if (st) {
        double r = fabs(RE(tn + pnew / v->ste - (m0 + pth / v->ste)));
        if (r > st->max_residual) st->max_residual = r;
        if (it > st->max_it) st->max_it = it;
        if (!conv) st->nonconverged++;
        st->it_hist[it < 32 ? it : 32]++;
      }
    }
}

/* Initial state (equilibrium): f_i = w_i T0, with Dirichlet wall nodes
   set to their wall temperature.  T0 == NULL means uniform 0. */
static void RN(init_)(const orc_params *p, const RN(vals) *v, const double *T0,
                      R *f) {
  RN(lat) L;
  RN(get_lat)(p->dim, p->q, &L);
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++)
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      int wall = RN(dirichlet_wall)(p, x, y);
      R T = wall >= 0 ? RN(wall_value)(v, wall, x, y)
                      : (R)(T0 ? T0[k] : 0.0);
      for (int i = 0; i < p->q; i++) f[i * n + k] = L.w[i] * T;
    }
}

/* Liquid-fraction front of each row: dx * trapezoid sum of phi(T). */
static void RN(front_integral_)(const orc_params *p, const RN(vals) *v,
                                const R *f, R *xf) {
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++) {
    R s = 0.0;
    for (long x = 0; x < nx; x++) {
      R T = 0.0;
      for (int i = 0; i < p->q; i++) T += f[i * n + y * nx + x];
      R ph = RN(phi_)(T, p->tm, v->delta);
      s += (x == 0 || x == nx - 1) ? 0.5 * ph : ph;
    }
    xf[y] = p->dx * s;
  }
}

/* Forward run from equilibrium of T0 and front misfit loss. */
static int RN(front_loss_)(const orc_params *p, const RN(vals) *v,
                           const double *T0, long nsteps,
                           const double *target, R *loss) {
  const long n = p->nx * p->ny;
  R *f = malloc(sizeof(R) * p->q * n), *g = malloc(sizeof(R) * p->q * n);
  R *th = malloc(sizeof(R) * n), *om = malloc(sizeof(R) * p->q * n);
  R *xf = malloc(sizeof(R) * p->ny);
  if (!f || !g || !th || !om || !xf) {
    free(f); free(g); free(th); free(om); free(xf);
    return -1;
  }
  RN(init_)(p, v, T0, f);
  R fin = 0.0, fo = 0.0;
  for (long s = 0; s < nsteps; s++) {
    RN(step_)(p, v, f, g, th, om, 0, &fin, &fo);
    R *t = f; f = g; g = t;
  }
  RN(front_integral_)(p, v, f, xf);
  R L = 0.0;
  for (long y = 0; y < p->ny; y++) {
    R d = xf[y] - target[y];
    L += 0.5 * d * d;
  }
  *loss = L;
  free(f); free(g); free(th); free(om); free(xf);
  return 0;
}
