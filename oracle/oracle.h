/*
 * oracle.h -- CPU FP64 oracle for the implicit regularized enthalpy
 * lattice Boltzmann method (IREBM) of Luddens, Lothode and Danaila,
 * "An implicit regularized enthalpy Lattice Boltzmann Method for the
 * Stefan problem" (arXiv 2505.13097).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct statement of what the GPU path computes.  It shares no code,
 * header, table or helper with the GPU library, and it is only called by
 * the tests, by the smoke check and by the CPU-baseline leg of the bench.
 *
 * State layout: distribution functions f[i][y][x] (plane i of q planes,
 * row-major, nx fastest), double precision.  1D lattices use ny = 1; the
 * 3D lattices (lattice3d.c) use f[i][z][y][x].
 *
 * Every function returns 0 on success and -1 on an invalid argument.
 */
#ifndef IREBM_ORACLE_H
#define IREBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* wall kinds; Neumann (eq. Neu_on_q) and bounce-back walls do not mix in
   one lattice */
enum { ORC_DIRICHLET = 0, ORC_BOUNCEBACK = 1, ORC_PERIODIC = 2,
       ORC_NEUMANN = 3 };
enum { ORC_SAFEGUARDED = 0, ORC_PLAIN = 1 };
enum { ORC_IREBM = 0, ORC_EEBM = 1 };   /* scheme of the 3D functions */
enum { ORC_FRONT_INTEGRAL = 0, ORC_FRONT_CROSSING = 1 };

typedef struct {
  int dim;              /* 1, 2 or 3 */
  int q;                /* 3 (D1Q3), 5 (D2Q5), 9 (D2Q9), 7 (D3Q7), 19 (D3Q19) */
  long nx, ny;          /* node counts; ny = 1 in 1D */
  double tau;           /* BGK relaxation time */
  double ste;           /* Stefan number */
  double tm;            /* melting temperature (0 in the scaled problem) */
  double delta;         /* regularization width, temperature units */
  int bc[4];            /* walls x-, x+, y-, y+ */
  double wall_T[4];     /* Dirichlet temperature per wall */
  const double *wall_profile[4]; /* optional per-node wall temperatures
                                    (length ny for x walls, nx for y walls) */
  double tol;           /* Newton stopping tolerance on |theta_{k+1}-theta_k| */
  int max_it;           /* Newton iteration cap */
  int newton_mode;      /* ORC_SAFEGUARDED or ORC_PLAIN */
  double dx;            /* lattice spacing, used by the front position */
  /* 3D lattices only (orc3_*): */
  long nz;              /* node count along z */
  int bc_z[2];          /* walls z-, z+ */
  double wall_T_z[2];   /* their Dirichlet temperatures */
  int scheme;           /* ORC_IREBM or ORC_EEBM */
} orc_params;

typedef struct {
  int max_it;           /* largest Newton iteration count seen */
  long nonconverged;    /* node-steps that reached the cap */
  long bisections;      /* safeguard bisections taken */
  double max_residual;  /* largest |F(theta_new)| */
  double flux_in;       /* sum of populations set by boundary closures */
  double flux_out;      /* sum of post-collision populations leaving */
  long it_hist[33];     /* iteration histogram, last bin counts >= 32 */
} orc_stats;

/* lattice tables: velocities, weights, opposite directions */
int orc_lattice(int dim, int q, int *ex, int *ey, double *w, int *opp);

/* regularized liquid fraction and its derivative */
double orc_phi(double theta, double tm, double delta);
double orc_dphi(double theta, double tm, double delta);

/* the local scalar problem of one node: returns the new temperature */
int orc_newton(double m0, double theta, double ste, double tm, double delta,
               double tol, int max_it, int mode, double *theta_new,
               int *iters, int *converged);

int orc_init(const orc_params *p, const double *T0, double *f);
int orc_step(const orc_params *p, const double *f, double *fout,
             orc_stats *st);
int orc_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
            double *energy_trace, double *flux_trace);
int orc_temperature(const orc_params *p, const double *f, double *T);
int orc_energy(const orc_params *p, const double *f, double *E);
int orc_front(const orc_params *p, const double *f, int mode, double *xf);

/* Neumann similarity solution of the two-phase Stefan problem */
int orc_stefan_lambda(double ste, double theta0, double *lambda);
double orc_neumann_T(double x, double t, double lambda, double theta0);

/* front misfit loss L = 1/2 sum_y (xf(y) - target(y))^2 after nsteps,
   starting from the equilibrium state of T0 */
int orc_front_loss(const orc_params *p, const double *T0, long nsteps,
                   const double *target, double *loss);

/* reverse mode of orc_front_loss: gradients with respect to the x- wall
   temperature profile (length ny), Ste and delta */
int orc_front_loss_grad(const orc_params *p, const double *T0, long nsteps,
                        const double *target, double *loss,
                        double *g_wall, double *g_ste, double *g_delta);

/* reverse mode of one step at state f: fbar = (df'/df)^T gbar, and the
   matching additions to the parameter gradients */
int orc_adjoint_step(const orc_params *p, const double *f,
                     const double *gbar, double *fbar, double *g_wall,
                     double *g_ste, double *g_delta);

/* complex-step evaluation of one step at f + i f_im with perturbed
   parameters (tangent of the step: Im(out)/h) */
int orc_cs_step(const orc_params *p, const double *f_re, const double *f_im,
                double ste_im, double delta_im, const double *wall_im,
                double *out_re, double *out_im);

/* complex-step evaluation of orc_front_loss: perturbs Ste, delta and the
   x- wall profile by i*(imaginary parts) and returns Re and Im of L */
int orc_cs_front_loss(const orc_params *p, const double *T0, long nsteps,
                      const double *target, double ste_im, double delta_im,
                      const double *wall_im, double *loss_re,
                      double *loss_im);

/* The explicit enthalpy based method (Algorithm 2): state f with
   M0(f) = H; same parameters (delta, tol, max_it, newton_mode unused),
   same boundary conditions (eebm.c states the closures). */
double orc_eebm_theta(double H, double ste, double tm);
int orc_eebm_init(const orc_params *p, const double *T0, double *f);
int orc_eebm_step(const orc_params *p, const double *f, double *fout,
                  orc_stats *st);
int orc_eebm_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
                 double *energy_trace, double *flux_trace);
int orc_eebm_temperature(const orc_params *p, const double *f, double *T);
int orc_eebm_energy(const orc_params *p, const double *f, double *E);
int orc_eebm_front(const orc_params *p, const double *f, int mode,
                   double *xf);
/* the collision half of a step (moments, equilibrium, BGK) at every node:
   the post-collision populations, whose pull streaming gives the next f */
int orc_eebm_collide(const orc_params *p, const double *f, double *omega);

/* The implicit liquid fraction based method (Algorithm 1): state f (q
   planes, M0(f) = theta) followed by the liquid fraction plane l, so
   (q + 1) planes; the inner loop stops when max |l^(k) - l^(k-1)| <= tol
   or after max_it iterations (orc_stats: max_it = largest inner
   iteration count, nonconverged = steps that hit the cap, max_residual =
   their largest last change of l; delta and newton_mode unused).
   ilfbm.c states the closures. */
int orc_ilfbm_init(const orc_params *p, const double *T0, double *f);
int orc_ilfbm_step(const orc_params *p, const double *f, double *fout,
                   orc_stats *st);
int orc_ilfbm_run(const orc_params *p, double *f, long nsteps,
                  orc_stats *st, double *energy_trace, double *flux_trace);
int orc_ilfbm_temperature(const orc_params *p, const double *f, double *T);
int orc_ilfbm_energy(const orc_params *p, const double *f, double *E);
int orc_ilfbm_front(const orc_params *p, const double *f, int mode,
                    double *xf);
/* collision without source of the q population planes of f */
int orc_ilfbm_collide(const orc_params *p, const double *f, double *omega);

/* The 3D lattices D3Q7 and D3Q19 (lattice3d.c): one step of IREBM
   (Algorithm 3) or EEBM (Algorithm 2), selected by p->scheme, with
   constant wall temperatures (wall_profile must be NULL).  State
   f[i][z][y][x]; fields [z][y][x]; the front has one value per row along
   x, rows ordered [z][y].  Statistics as for 2D (bisections not counted).
   Velocities: rest, +x, +y, +z, -x, -y, -z, then (1,1,0), (1,-1,0),
   (1,0,1), (1,0,-1), (0,1,1), (0,1,-1) and their negatives. */
int orc_lattice3(int q, int *ex, int *ey, int *ez, double *w, int *opp);
int orc3_init(const orc_params *p, const double *T0, double *f);
int orc3_step(const orc_params *p, const double *f, double *fout,
              orc_stats *st);
int orc3_run(const orc_params *p, double *f, long nsteps, orc_stats *st,
             double *energy_trace, double *flux_trace);
int orc3_temperature(const orc_params *p, const double *f, double *T);
int orc3_energy(const orc_params *p, const double *f, double *E);
int orc3_front(const orc_params *p, const double *f, int mode, double *xf);
/* the post-collision populations of every node */
int orc3_collide(const orc_params *p, const double *f, double *omega);

#ifdef __cplusplus
}
#endif
#endif
