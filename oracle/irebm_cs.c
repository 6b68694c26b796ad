/*
 * irebm_cs.c -- the oracle's step over complex doubles, for complex-step
 * derivatives: with Ste, delta and the wall temperatures given imaginary
 * parts h*v (h ~ 1e-30), Im(L)/h is the directional derivative of the
 * loss along v to rounding, with no subtractive cancellation.
 * TEST INFRASTRUCTURE ONLY: see oracle.h.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define R double complex
#define RN(name) c_##name
#define TANH(z) ctanh(z)
#define RE(z) creal(z)
#define CS 1
#include "irebm_body.h"

int orc_cs_front_loss(const orc_params *p, const double *T0, long nsteps,
                      const double *target, double ste_im, double delta_im,
                      const double *wall_im, double *loss_re,
                      double *loss_im) {
  if (c_check(p) || nsteps < 0 || !target) return -1;
  c_vals v;
  double complex *prof = malloc(sizeof(double complex) * p->ny);
  if (!prof) return -1;
  v.ste = p->ste + I * ste_im;
  v.delta = p->delta + I * delta_im;
  for (int k = 0; k < 4; k++) {
    v.wall_T[k] = p->wall_T[k];
    v.wall_profile[k] = 0;
  }
  /* the x- wall always gets a complex profile (real part from the
     parameters, imaginary part from wall_im) */
  for (long y = 0; y < p->ny; y++) {
    double re = p->wall_profile[0] ? p->wall_profile[0][y] : p->wall_T[0];
    prof[y] = re + I * (wall_im ? wall_im[y] : 0.0);
  }
  v.wall_profile[0] = prof;
  double complex L;
  int rc = c_front_loss_(p, &v, T0, nsteps, target, &L);
  free(prof);
  if (rc) return rc;
  *loss_re = creal(L);
  *loss_im = cimag(L);
  return 0;
}

/*
 * Complex-step tangent of one step: f' = step(f + i v, Ste + i s_im,
 * delta + i d_im, x- wall profile + i wall_im); returns Re and Im of f'.
 */
int orc_cs_step(const orc_params *p, const double *f_re, const double *f_im,
                double ste_im, double delta_im, const double *wall_im,
                double *out_re, double *out_im) {
  if (c_check(p)) return -1;
  const long n = p->nx * p->ny, qn = p->q * n;
  double complex *f = malloc(sizeof(double complex) * qn);
  double complex *g = malloc(sizeof(double complex) * qn);
  double complex *th = malloc(sizeof(double complex) * n);
  double complex *om = malloc(sizeof(double complex) * qn);
  double complex *prof = malloc(sizeof(double complex) * p->ny);
  if (!f || !g || !th || !om || !prof) {
    free(f); free(g); free(th); free(om); free(prof);
    return -1;
  }
  for (long k = 0; k < qn; k++) f[k] = f_re[k] + I * (f_im ? f_im[k] : 0.0);
  c_vals v;
  v.ste = p->ste + I * ste_im;
  v.delta = p->delta + I * delta_im;
  for (int k = 0; k < 4; k++) {
    v.wall_T[k] = p->wall_T[k];
    v.wall_profile[k] = 0;
  }
  for (long y = 0; y < p->ny; y++) {
    double re = p->wall_profile[0] ? p->wall_profile[0][y] : p->wall_T[0];
    prof[y] = re + I * (wall_im ? wall_im[y] : 0.0);
  }
  v.wall_profile[0] = prof;
  double complex fin = 0.0, fo = 0.0;
  c_step_(p, &v, f, g, th, om, 0, &fin, &fo);
  for (long k = 0; k < qn; k++) {
    out_re[k] = creal(g[k]);
    out_im[k] = cimag(g[k]);
  }
  free(f); free(g); free(th); free(om); free(prof);
  return 0;
}
