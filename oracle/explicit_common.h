/*
 * explicit_common.h -- pieces shared by the oracles of the two schemes
 * the paper compares IREBM with (eebm.c: Algorithm 2; ilfbm.c: Algorithm
 * 1): lattice tables, wall lookups, the sharp liquid fraction, and pull
 * streaming of post-collision populations with the boundary closures of
 * Section 4.2 applied to the streamed populations.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#ifndef ORACLE_EXPLICIT_COMMON_H
#define ORACLE_EXPLICIT_COMMON_H

#include "oracle.h"

/* sharp liquid fraction of a temperature, and of an enthalpy */
static double lf_of_T(double T, double tm) { return T > tm ? 1.0 : 0.0; }

static double lf_of_H(double H, double ste, double tm) {
  const double l = ste * (H - tm);
  return l < 0.0 ? 0.0 : (l > 1.0 ? 1.0 : l);
}

typedef struct {
  int ex[9], ey[9], opp[9];
  double w[9];
} lat;

static int check(const orc_params *p, lat *L) {
  if (!p || !(p->tau > 0.5) || !(p->ste > 0)) return -1;
  if (p->nx < 3 || p->ny < 1 || (p->dim == 2 && p->ny < 3)) return -1;
  if (p->dim == 1 && p->ny != 1) return -1;
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
  return orc_lattice(p->dim, p->q, L->ex, L->ey, L->w, L->opp);
}

static int dirichlet_wall(const orc_params *p, long x, long y) {
  if (x == 0 && p->bc[0] == ORC_DIRICHLET) return 0;
  if (x == p->nx - 1 && p->bc[1] == ORC_DIRICHLET) return 1;
  if (p->dim == 2 && y == 0 && p->bc[2] == ORC_DIRICHLET) return 2;
  if (p->dim == 2 && y == p->ny - 1 && p->bc[3] == ORC_DIRICHLET) return 3;
  return -1;
}

static double wall_value(const orc_params *p, int wall, long x, long y) {
  if (p->wall_profile[wall]) return p->wall_profile[wall][wall < 2 ? y : x];
  return p->wall_T[wall];
}

/* the interior neighbour across the Neumann walls of node (x, y) (the
   diagonal one at the corner of two); 0 when on no Neumann wall */
static int neumann_mirror(const orc_params *p, long x, long y, long *mx,
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

/* pull source x - e of node (x, y), wrapped on periodic axes; 0 outside */
static int source(const orc_params *p, long x, long y, int ex, int ey,
                  long *sx, long *sy) {
  long a = x - ex, b = y - ey;
  if (a < 0 || a >= p->nx) {
    if (p->bc[0] != ORC_PERIODIC) return 0;
    a = (a + p->nx) % p->nx;
  }
  if (b < 0 || b >= p->ny) {
    if (p->dim == 1 || p->bc[2] != ORC_PERIODIC) return 0;
    b = (b + p->ny) % p->ny;
  }
  *sx = a;
  *sy = b;
  return 1;
}

/* does the pull source x - e of node (x, y) leave the lattice through
   bounce-back walls only?  (Periodic axes wrap and are never left.) */
static int leaves_by_bounceback(const orc_params *p, long x, long y, int ex,
                                int ey) {
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
 * Pull streaming g_i(x) = omega_i(x - e_i) of post-collision populations
 * at every node into fout, closing the populations whose source lies
 * outside the lattice (Section 4.2), in this order:
 *   1. bounce-back g_i = g_opp(i) beyond bounce-back walls only, when the
 *      opposite is known;
 *   2. Dirichlet node: M0(g) is set to dirichlet_m0(T_D) (the deficit
 *      shared by weight among the remaining unknowns);
 *   3. Neumann node (eq. Neu_on_q): M0(g) is set to M0 of the streamed
 *      populations at the mirror node, shared the same way;
 *   4. what is left (corner of two bounce-back walls): omega_opp(i)(x).
 * Adds the closure-set populations to *fin and the post-collision
 * populations leaving the lattice to *fo.
 */
static void stream_close(const orc_params *p, const lat *L,
                         const double *omega,
                         double (*dirichlet_m0)(const orc_params *, double),
                         double *fout, double *fin, double *fo) {
  const long nx = p->nx, ny = p->ny, n = nx * ny;
  for (long y = 0; y < ny; y++)
    for (long x = 0; x < nx; x++) {
      const long k = y * nx + x;
      double g[9];
      int known[9], set[9], nunk = 0;
      for (int i = 0; i < p->q; i++) {
        long sx, sy;
        known[i] = source(p, x, y, L->ex[i], L->ey[i], &sx, &sy);
        g[i] = known[i] ? omega[i * n + sy * nx + sx] : 0.0;
        set[i] = known[i];
        nunk += !known[i];
      }
      if (nunk) {
        for (int i = 0; i < p->q; i++)
          if (!known[i] && known[L->opp[i]] &&
              leaves_by_bounceback(p, x, y, L->ex[i], L->ey[i])) {
            g[i] = g[L->opp[i]];
            set[i] = 1;
            *fin += g[i];
          }
        const int wall = dirichlet_wall(p, x, y);
        if (wall >= 0) {
          const double TD = wall_value(p, wall, x, y);
          double D = dirichlet_m0(p, TD), wu = 0.0;
          for (int i = 0; i < p->q; i++) {
            if (set[i]) D -= g[i];
            else wu += L->w[i];
          }
          for (int i = 0; i < p->q; i++)
            if (!set[i]) {
              g[i] = D * (L->w[i] / wu);
              set[i] = 1;
              *fin += g[i];
            }
        }
        long mx, my;
        if (wall < 0 && neumann_mirror(p, x, y, &mx, &my)) {
          /* M0 of the populations streamed into the mirror node */
          double D = 0.0, wu = 0.0;
          for (int i = 0; i < p->q; i++) {
            long sx = mx, sy = my;   /* always a lattice node (check) */
            source(p, mx, my, L->ex[i], L->ey[i], &sx, &sy);
            D += omega[i * n + sy * nx + sx];
          }
          for (int i = 0; i < p->q; i++) {
            if (set[i]) D -= g[i];
            else wu += L->w[i];
          }
          for (int i = 0; i < p->q; i++)
            if (!set[i]) {
              g[i] = D * (L->w[i] / wu);
              set[i] = 1;
              *fin += g[i];
            }
        }
        for (int i = 0; i < p->q; i++)
          if (!set[i]) {
            g[i] = omega[L->opp[i] * n + k];
            *fin += g[i];
          }
      }
      /* populations leaving the lattice */
      for (int i = 1; i < p->q; i++) {
        long dx_, dy_;
        if (!source(p, x, y, -L->ex[i], -L->ey[i], &dx_, &dy_))
          *fo += omega[i * n + k];
      }
      for (int i = 0; i < p->q; i++) fout[i * n + k] = g[i];
    }
}

#endif
