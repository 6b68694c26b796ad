/*
 * lbm_stefan.h -- C ABI of the MI355X (gfx950) implementation of the
 * implicit regularized enthalpy lattice Boltzmann method (IREBM) for the
 * two-phase Stefan problem (Luddens, Lothode, Danaila, arXiv 2505.13097).
 *
 * One time step is Algorithm 3 of Section 4.1: BGK collision of the
 * thermal populations with equilibrium w_i T, pull streaming, the zeroth
 * moment, a local Newton solve of
 *     T~ = M0(q) + (phi(T) - phi(T~)) / Ste,
 *     phi(T) = (1 + tanh((T - T_m)/delta)) / 2        (Section 4.1)
 * for the new temperature, the source term (w_i/Ste)(phi(T) - phi(T~))
 * and the update, with the boundary closures on the pulled populations of
 * Section 4.2 (Dirichlet, bounce-back) or periodic axes.
 *
 * The same handles also run the explicit enthalpy based method the paper
 * compares with (EEBM, Section 3.4, Algorithm 2; params.scheme =
 * LBM_SCHEME_EEBM): H = M0(f), theta = Theta(H) in closed form (H below
 * T_m, T_m for T_m <= H <= T_m + 1/Ste, H - 1/Ste above), equilibrium
 * w_i theta (i != 0) and H - (1 - w_0) theta (rest), BGK collision and
 * pull streaming, with the same closures (Dirichlet target: the wall
 * enthalpy T_D + l(T_D)/Ste, l = 1 above T_m and 0 otherwise).
 *
 * Conventions
 *   - All entry points return LBM_STEFAN_OK (0) or a negative error code;
 *     the text of the last error of a handle is lbm_stefan_last_error(h)
 *     (lbm_stefan_last_error(NULL) for errors raised before a handle
 *     exists).  No entry point aborts the process.
 *   - "host" pointers are ordinary CPU memory and are only read or written
 *     during the call.  "device" pointers are GPU memory of the device that
 *     was current when the handle was created.
 *   - Lattices: D1Q3 (dim 1), D2Q5 and D2Q9 (dim 2).  Velocity order: rest,
 *     +x, +y, -x, -y, then (+1,+1), (-1,+1), (-1,-1), (+1,-1); weights
 *     D1Q3 (2/3, 1/6, 1/6), D2Q5 (1/3, 1/6 x4), D2Q9 (4/9, 1/9 x4,
 *     1/36 x4): the "standard weights" of Section 3.2, whose second moment
 *     is T/3 times the identity as the Chapman-Enskog analysis requires.
 *   - 3D lattices (dim 3; the enthalpy model of Section 2 holds in 3D):
 *     D3Q7 and D3Q19.  Velocity order: rest, +x, +y, +z, -x, -y, -z, then
 *     (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1), (0,1,-1) and their
 *     negatives in that order (D3Q7: the first seven).  The same second
 *     moment fixes D3Q19 (1/3, 1/18 x6, 1/36 x12) and D3Q7 (faces 1/6,
 *     rest 0).  Planes and fields are [nz][ny][nx]; fronts have one value
 *     per row along x, rows ordered [nz][ny].  The six faces x-, x+, y-,
 *     y+, z-, z+ take the closures of the 2D walls (the first Dirichlet
 *     face in that order gives a node's temperature) with constant
 *     temperatures (no wall profiles).  Schemes IREBM and EEBM; no reverse
 *     mode, no batched form; kernel variants of their own.
 *   - The state is the set of post-collision populations
 *     Omega_i = (1 - 1/tau) f_i + (w_i/tau) T  (eq. def_qi_omegai) at the
 *     current time, stored as q planes [q][ny][nx] (3D: [q][nz][ny][nx];
 *     x fastest) in the
 *     storage type (double or float).  T = sum_i Omega_i = sum_i f_i.
 *     EEBM: Omega_i = f_i - (f_i - f_i^eq)/tau, the populations after the
 *     collision of Algorithm 2 and before its streaming; sum_i Omega_i =
 *     sum_i f_i = H and T = Theta(H).  Per-node arithmetic is always
 *     double precision.
 *   - nx nodes span x in [0, 1] unless dx says otherwise; wall nodes are
 *     lattice nodes ("wet" walls).
 *   - A handle enqueues all GPU work on the stream it was created with and
 *     is not thread-safe; use one handle per stream.  Calls that overlap on
 *     one handle race.
 */
#ifndef LBM_STEFAN_H
#define LBM_STEFAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define LBM_STEFAN_OK 0
#define LBM_STEFAN_EINVAL (-1)   /* invalid argument (see each call) */
#define LBM_STEFAN_EDEVICE (-2)  /* a HIP runtime error; text in last_error */
#define LBM_STEFAN_ENOTCONV (-3) /* strict mode: a Newton solve hit the cap */
#define LBM_STEFAN_ENAN (-4)     /* a reduction found NaN or Inf */

/* boundary kind of a wall (Section 4.2) */
#define LBM_BC_DIRICHLET 0   /* eq. Dir_on_q: fixes the wall temperature */
#define LBM_BC_BOUNCEBACK 1  /* q_i = q_opp(i): homogeneous Neumann */
#define LBM_BC_PERIODIC 2    /* both walls of the axis must be periodic */
#define LBM_BC_NEUMANN 3     /* eq. Neu_on_q: homogeneous Neumann by copying
                                the zeroth moment of the pulled populations
                                of the interior neighbour across the wall
                                (the diagonal one at the corner of two
                                Neumann walls; several unknowns share by
                                weight).  Not beside a bounce-back wall in
                                one lattice; such lattices take one step
                                per launch (two-step variants run as the
                                default one) and have no reverse mode. */

/* population storage */
#define LBM_STORE_F64 0
#define LBM_STORE_F32 1

/* Newton variant */
#define LBM_NEWTON_SAFEGUARDED 0 /* Newton step kept inside a bisection
                                    safeguard (rtsafe rule), default */
#define LBM_NEWTON_PLAIN 1       /* the update of Algorithm 3 as printed */

/* front position of each row y (Section 6: "position of the interface") */
#define LBM_FRONT_LIQUID_INTEGRAL 0 /* dx * trapezoid sum_x phi(T(x, y));
                                       EEBM: of l(H) = clamp(Ste (H - T_m),
                                       0, 1); ILFBM: of its l plane */
#define LBM_FRONT_ZERO_CROSSING 1   /* first x where T - T_m goes from > 0
                                       to <= 0, linearly interpolated */

/* time-step scheme */
#define LBM_SCHEME_IREBM 0 /* Algorithm 3 (Section 4.1), default */
#define LBM_SCHEME_EEBM 1  /* Algorithm 2 (Section 3.4): no Newton solve;
                              delta, newton_* and newton_mode are unused
                              but still validated; no reverse mode */
#define LBM_SCHEME_ILFBM 2 /* Algorithm 1 (Section 3.3): the state adds the
                              liquid fraction l (workspace); each step runs
                              the inner loop of collision with the source
                              (w_i/Ste)(l - l^(k-1)), pull streaming and
                              l^(k) = clamp(Ste (M0(f^(k)) + l^(k-1)/Ste -
                              T_m), 0, 1) until max |l^(k) - l^(k-1)| <=
                              newton_tol or newton_max_it iterations, one
                              launch per iteration (the host reads a device
                              flag every few); Dirichlet closures target
                              T_D.  Kernel variants do not apply; no reverse
                              mode, not in the batched form.  Statistics:
                              max_newton_it = most inner iterations of a
                              step, nonconverged = steps that hit the cap,
                              max_residual = their largest last change of
                              l.  E = sum [T + l/Ste]. */

/* fields for lbm_stefan_get_field */
#define LBM_FIELD_T 0     /* temperature, double [ny][nx] */
#define LBM_FIELD_STATE 1 /* the state planes, storage type [q][ny][nx] */
#define LBM_FIELD_LIQUID 2 /* liquid fraction, double [ny][nx]: phi(T)
                              (IREBM), l(H) (EEBM), the l plane (ILFBM) */

typedef struct lbm_stefan_params {
  int32_t dim;           /* 1, 2 or 3 */
  int32_t q;             /* 3 (dim 1), 5 or 9 (dim 2), 7 or 19 (dim 3) */
  int64_t nx, ny;        /* node counts; ny = 1 when dim = 1 */
  int32_t storage;       /* LBM_STORE_F64 or LBM_STORE_F32 */
  int32_t newton_mode;   /* LBM_NEWTON_* */
  double tau;            /* BGK relaxation time (eq. std_lbm_collide_stream),
                            > 1/2; diffusivity (tau - 1/2)/3 in lattice
                            units (Section 5) */
  double ste;            /* Stefan number (Section 2), > 0 */
  double t_m;            /* melting temperature (0 in scaled units) */
  double delta;          /* width of the regularized liquid fraction, in
                            temperature units, > 0 (Section 4.1) */
  int32_t bc[4];         /* walls x-, x+, y-, y+: LBM_BC_*; y walls are
                            ignored when dim = 1 */
  double wall_T[4];      /* Dirichlet temperature of each wall */
  const double *wall_profile[4]; /* host, nullable: per-node Dirichlet
                            temperatures (length ny for x walls, nx for y
                            walls); copied during init */
  double dx;             /* lattice spacing used by the front position;
                            0 means 1/(nx - 1) */
  double newton_tol;     /* stop when |T^(k+1) - T^(k)| <= tol, > 0 */
  int32_t newton_max_it; /* iteration cap, 1..1000 */
  int32_t strict;        /* nonzero: lbm_stefan_step returns
                            LBM_STEFAN_ENOTCONV if a solve hit the cap */
  int32_t variant;       /* kernel variant (lbm_stefan_variant_name); -1
                            picks the library default for the lattice
                            (D1Q3 lattices the resident variant takes:
                            that one) */
  int32_t flags;         /* LBM_FLAG_* */
  int32_t scheme;        /* LBM_SCHEME_*; 0 (zeroed params) is IREBM */
  int64_t nz;            /* dim 3: nodes along z, >= 3; ignored otherwise */
  int32_t bc_z[2];       /* dim 3: faces z-, z+ (LBM_BC_*) */
  double wall_T_z[2];    /* dim 3: their Dirichlet temperatures */
} lbm_stefan_params;

#define LBM_FLAG_ADJOINT 1 /* reserve workspace for the reverse mode */
/* 3D lattices: every node of a tile that holds an x face takes the
 * bounds-checked path, a node at a time, instead of the interior loads
 * with the x-face closure in registers (both give the same states bit for
 * bit; the flag exists to check that, and costs speed) */
#define LBM_FLAG_CHECKED_FACES 2

typedef struct lbm_stefan_stats {
  int64_t steps;         /* steps taken since init */
  int32_t max_newton_it; /* largest Newton iteration count since the last
                            lbm_stefan_reset_stats (or init); EEBM: 0, as
                            are nonconverged and max_residual */
  int32_t reserved;
  int64_t nonconverged;  /* node-steps that reached the cap, same window */
  double max_residual;   /* largest |T~ + phi(T~)/Ste - M0(q) - phi(T)/Ste| */
  double energy;         /* E = sum_x [T + phi(T)/Ste] of the current state
                            (eq. eq-H; EEBM: sum_x H), FP64 in a fixed
                            summation order */
  double flux_in;        /* sum of populations set by boundary closures */
  double flux_out;       /* sum of post-collision populations leaving the
                            lattice; E(n) - E(0) = flux_in - flux_out up to
                            Newton residuals (same window) */
} lbm_stefan_stats;

typedef struct lbm_stefan lbm_stefan_t;

/* Library version string (static storage). */
const char *lbm_stefan_version(void);

/* Text of the last error of h, or of the calling thread's last failed
   lbm_stefan_init / *_workspace_bytes when h is NULL.  Static or
   handle-owned storage; never NULL. */
const char *lbm_stefan_last_error(const lbm_stefan_t *h);

/*
 * Device workspace needed by a handle for params p (the two population
 * buffers, wall profiles, per-tile statistics and reduction scratch).
 * Errors: EINVAL for invalid params (same checks as init).
 */
int lbm_stefan_workspace_bytes(const lbm_stefan_params *p, size_t *bytes);

/*
 * Create a handle and its initial state: Omega_i = w_i T0 (the
 * equilibrium state, f_i = w_i T0), with nodes on Dirichlet walls at their
 * wall temperature (where two Dirichlet walls meet, the first of x-, x+,
 * y-, y+ gives it).
 *   T0         host, nullable: initial temperature [ny][nx] (3D:
 *              [nz][ny][nx]) (NULL: 0).
 *   workspace  device, >= lbm_stefan_workspace_bytes(p), 256-byte
 *              aligned; owned by the caller, must outlive the handle.
 *   stream     hipStream_t to enqueue on (NULL: the null stream).
 *   out        receives the handle (host memory owned by the library).
 * Blocks until the state is built.  Errors: EINVAL (invalid params:
 * tau <= 1/2, Ste <= 0, delta <= 0, tol <= 0, max_it outside 1..1000,
 * nx < 3, ny < 3 in 2D or != 1 in 1D, nz < 3 in 3D, more than 2^31 - 1
 * nodes, lattice/dim mismatch, a periodic axis with one non-periodic
 * wall, workspace too small or misaligned, unknown variant or scheme,
 * LBM_FLAG_ADJOINT with LBM_SCHEME_EEBM, a Neumann wall or a 3D lattice,
 * Neumann and bounce-back walls in one lattice, a 3D lattice with a wall
 * profile or LBM_SCHEME_ILFBM), EDEVICE.
 */
int lbm_stefan_init(const lbm_stefan_params *p, const double *T0,
                    void *workspace, size_t bytes, void *stream,
                    lbm_stefan_t **out);

/*
 * Advance nsteps >= 0 time steps (one kernel launch per step on the
 * handle's stream).  Asynchronous when stats is NULL and strict is off;
 * otherwise waits for the stream and fills *stats (the energy is
 * recomputed from the final state).  Errors: EINVAL (nsteps < 0),
 * ENOTCONV (strict), ENAN (the energy is not finite), EDEVICE.
 */
int lbm_stefan_step(lbm_stefan_t *h, int64_t nsteps, lbm_stefan_stats *stats);

/* Zero the Newton and flux accumulators (asynchronous). */
int lbm_stefan_reset_stats(lbm_stefan_t *h);

/*
 * Front position of every row of the current state (mode LBM_FRONT_*),
 * written to front (host, ny doubles, 3D: nz*ny, may be NULL), and the
 * energy E
 * (host, may be NULL).  Both reductions are FP64 in a fixed order.
 * Waits for the stream.  Errors: EINVAL (bad mode), ENAN, EDEVICE.
 */
int lbm_stefan_query_front(lbm_stefan_t *h, int32_t mode, double *front,
                           double *energy);

/*
 * Copy a field of the current state to host memory: LBM_FIELD_T or
 * LBM_FIELD_LIQUID (ny*nx doubles, 3D: nz*ny*nx) or LBM_FIELD_STATE
 * (q times as many values of the storage type).
 * Waits for the stream.  Errors: EINVAL, EDEVICE.
 */
int lbm_stefan_get_field(lbm_stefan_t *h, int32_t what, void *host);

/*
 * Replace the current state by q planes of the storage type (layout as
 * above), read from device memory (on_device != 0) or host memory.
 * Enqueued on the stream; a host source is copied before return.  ILFBM:
 * the liquid fraction plane is left as it is.
 */
int lbm_stefan_set_state(lbm_stefan_t *h, const void *state,
                         int32_t on_device);

/* Device pointer of the current state planes (valid until the next
   step, set_state or destroy). */
int lbm_stefan_state_ptr(lbm_stefan_t *h, void **dev_state);

/* Number of compiled kernel variants for a lattice/storage pair, and the
   name of one ("<tile_x>x<tile_y>/npt<k>[/r<m>][/nt][/rev]": tile size,
   nodes per thread, m tiles stacked along y per thread block,
   non-temporal stores, block order reversed every other step; or
   "<w>x<b>/t2/r<m>[/nt]": two time steps per launch, a w-column window
   sweeping m rows, b rows per pass; a single trailing step then uses the
   default variant, and a lattice with a Neumann wall runs the default
   variant; q = 3 also "resident2048": D1Q3 lattices of at most 2048 nodes
   with no Neumann wall run many steps per launch in one workgroup, both
   states in LDS (others run the default variant; the batched form rejects
   it); 3D lattices, q = 7 or 19: "<tile_x>x<tile_y>/npt<k>/z<c>[/nt]", c z
   slices swept by one block); used by autotuners. */
int lbm_stefan_variant_count(int32_t q, int32_t storage, int32_t *count);
const char *lbm_stefan_variant_name(int32_t q, int32_t storage,
                                    int32_t variant);

/* Select the kernel variant of an existing handle (resets statistics). */
int lbm_stefan_set_variant(lbm_stefan_t *h, int32_t variant);

/*
 * Autotuner: time every compiled variant for `steps` steps (1..10000) with
 * HIP events on the handle's stream, keep the fastest.  The state is saved
 * to `scratch` (device, >= q*nodes*sizeof(storage) bytes, caller-owned)
 * before the trials and restored after each one, so the handle's state
 * and step count are unchanged; statistics are reset.  Writes the chosen
 * variant and its time per step (ms); either output may be NULL.  Waits
 * for the stream.  ILFBM (one kernel shape): returns the current variant
 * and 0 ms without running.  Errors: EINVAL, EDEVICE.
 */
int lbm_stefan_autotune(lbm_stefan_t *h, void *scratch, size_t scratch_bytes,
                        int32_t steps, int32_t *best_variant,
                        double *best_ms_per_step);

/* Free the handle (host memory only; the workspace stays the caller's).
   Waits for the stream. */
int lbm_stefan_destroy(lbm_stefan_t *h);

/* ---------------------------------------------------------------------
 * A step that allocates nothing, for callers that cannot allocate device
 * memory or own a workspace: code under HIP graph capture, tight serving
 * loops and harnesses that forbid hipMalloc.
 *
 * lbm_stefan_step_noalloc: one time step of the lattice described by p
 * from the state src to dst, the same step lbm_stefan_step takes on a
 * handle made from p whose state is src (bit for bit, in the one-step
 * tiling of p->variant: a two-step variant's single step and the resident
 * variant's step take the library defaults, as on a handle).
 *   src, dst  device, distinct, q planes of the storage type each (the
 *             layout of lbm_stefan_state_ptr), on the current device.
 *   stats     host, nullable: the statistics of this one step (steps = 1;
 *             energy of dst).  With stats (or p->strict) the call waits
 *             for the stream; without, it only enqueues a fill kernel and
 *             the step kernel on `stream`.
 *   stream    hipStream_t (NULL: the null stream).
 * The per-item statistics, energy partials and the result block live in
 * a fixed device array of LBM_STEFAN_NOALLOC_SCRATCH_BYTES per device,
 * held until the process ends; nothing is allocated.  Every call on a
 * device shares that array (the call clears what it needs first), so
 * calls that overlap on one device (several streams or threads) race;
 * calls on one stream are ordered.
 * Errors (text in lbm_stefan_last_error(NULL)): EINVAL (invalid params as
 * for lbm_stefan_init, NULL or equal buffers, wall profiles, the ILFBM
 * scheme, LBM_FLAG_ADJOINT, or a lattice whose statistics slots and
 * energy partials exceed the fixed array), ENOTCONV (strict), ENAN (the
 * energy of dst is not finite), EDEVICE.
 */
#define LBM_STEFAN_NOALLOC_SCRATCH_BYTES (16u << 20)
int lbm_stefan_step_noalloc(const lbm_stefan_params *p, const void *src,
                            void *dst, lbm_stefan_stats *stats, void *stream);

/* ---------------------------------------------------------------------
 * Reverse mode (handle created with LBM_FLAG_ADJOINT).  The reverse step
 * is the exact adjoint of the forward step of this library (Algorithm 3,
 * Section 4.1, with the closures of Section 4.2): the transposes of the
 * collision, pull, source and closures, and the implicit-function theorem
 * at the Newton root (dT~/dm0 = 1/J, dT~/dT = (phi'(T)/Ste)/J,
 * J = 1 + phi'(T~)/Ste), exact where the solve converged.  Adjoint arrays
 * ("abar": the adjoint of the state, q planes [q][ny][nx]) are FP64 device
 * memory in every storage mode.  Gradients with respect to Ste, delta and
 * every Dirichlet wall node's temperature accumulate in the handle until
 * lbm_stefan_adjoint_reset.
 * --------------------------------------------------------------------- */

/* Zero the gradient accumulators (asynchronous). */
int lbm_stefan_adjoint_reset(lbm_stefan_t *h);

/*
 * Seed from the front position (LBM_FRONT_LIQUID_INTEGRAL) of `state`
 * (device, state layout): abar = d(sum_y g(y) xf(y))/dOmega with g =
 * dL_dfront (host, ny doubles), i.e. g(y) dx w_x phi'(T(x, y)) in every
 * plane; adds the delta-dependence of the front to the delta gradient.
 * abar: device, q*nx*ny doubles, overwritten.  Waits for the stream.
 */
int lbm_stefan_front_vjp(lbm_stefan_t *h, const void *state,
                         const double *dL_dfront, double *abar);

/*
 * One reverse step at forward state state_n (device): abar_n = (dOmega^{n+1}
 * /dOmega^n)^T abar_np1, and the step's Ste, delta and wall-temperature
 * terms are added to the accumulators.  abar_np1 and abar_n: device FP64,
 * distinct.  Asynchronous.
 */
int lbm_stefan_adjoint_step(lbm_stefan_t *h, const void *state_n,
                            const double *abar_np1, double *abar_n);

/* Add the dependence of the equilibrium initial state (Dirichlet nodes at
   w_i T_D) on the wall temperatures, given abar_0 (device).  Asynchronous. */
int lbm_stefan_adjoint_initial_state(lbm_stefan_t *h, const double *abar_0);

/*
 * Read the accumulated gradients: g_wall (host, nullable) receives the
 * wall-temperature gradients of the x-, x+ walls (ny values each) then
 * the y-, y+ walls (nx values each), one per Dirichlet wall node (zero
 * elsewhere); g_ste and g_delta (host, nullable).  Fixed-order FP64 sums.
 * Waits for the stream.  Errors: ENAN, EDEVICE.
 */
int lbm_stefan_adjoint_gradients(lbm_stefan_t *h, double *g_wall,
                                 double *g_ste, double *g_delta);

/* Device pointers of the handle's two adjoint work arrays (q*nx*ny FP64
   each), usable as abar arguments; valid for the handle's lifetime. */
int lbm_stefan_adjoint_buffers(lbm_stefan_t *h, double **abar0,
                               double **abar1);

/*
 * Checkpointed gradient of a front functional ("tape").  Checkpoints are
 * taken every `interval` steps (sqrt(nsteps) balances memory and
 * recomputation); the reverse sweep recomputes each segment from its
 * checkpoint, then runs its reverse steps.
 *   lbm_stefan_tape_bytes: device bytes of a tape for (p, nsteps,
 *     interval): (ceil(nsteps/interval) + 1 + 2 interval) states (the
 *     checkpoints, then two segments: the reverse sweep of one segment
 *     overlaps the recomputation of the next on a second stream).
 *   lbm_stefan_forward_tape: advance the handle nsteps from its current
 *     state (the state the gradient is taken at: normally the initial state
 *     built by lbm_stefan_init), storing checkpoints in `tape` (device,
 *     256-byte aligned, caller-owned).  Asynchronous.
 *   lbm_stefan_backward_tape: with g = dL_dfront (host, ny doubles) the
 *     derivative of a loss with respect to the final integral front,
 *     compute dL/d(wall temperatures) (g_wall, layout as in
 *     lbm_stefan_adjoint_gradients), dL/dSte and dL/ddelta, including the
 *     initial state's dependence on the wall temperatures.  Resets the
 *     accumulators first; the handle's state stays the final state; the
 *     statistics also count the recomputed steps.  Waits for the stream.
 * Errors: EINVAL (no LBM_FLAG_ADJOINT, bad sizes, a tape that is not the
 * one of the last forward_tape), ENAN, EDEVICE.
 */
int lbm_stefan_tape_bytes(const lbm_stefan_params *p, int64_t nsteps,
                          int64_t interval, size_t *bytes);
int lbm_stefan_forward_tape(lbm_stefan_t *h, int64_t nsteps, int64_t interval,
                            void *tape, size_t bytes);
int lbm_stefan_backward_tape(lbm_stefan_t *h, const double *dL_dfront,
                             void *tape, size_t bytes, double *g_wall,
                             double *g_ste, double *g_delta);

/* ---------------------------------------------------------------------
 * Batched form: many independent lattices with their own sizes and
 * parameters, advanced together by one persistent kernel launch per time
 * step (optionally replayed from a captured hipGraph).  Every instance is
 * stepped by exactly the arithmetic of the single-lattice step (Algorithm
 * 3, Section 4.1; closures of Section 4.2): a batch member evolves
 * bit-identically to the same lattice run alone.  Instances must share
 * q, storage and newton_mode; everything else may differ.  The variant
 * field of the params is ignored (the batch has one schedule).
 * --------------------------------------------------------------------- */
typedef struct lbm_stefan_batch lbm_stefan_batch_t;

/* Workspace for `count` instances (params array of length count).
   Errors: EINVAL (an invalid instance, mixed q/storage/newton_mode/
   scheme, an instance with a Neumann wall). */
int lbm_stefan_batch_workspace_bytes(const lbm_stefan_params *params,
                                     int32_t count, size_t *bytes);

/*
 * Create a batch: equilibrium initial state of every instance, as in
 * lbm_stefan_init.  T0: host, nullable array of `count` nullable host
 * arrays [ny_k][nx_k].  workspace: device, 256-byte aligned, >= the size
 * above, owned by the caller.  Default schedule: the library's default
 * variant, one block per work item (a stack of tiles), no graph.  Blocks
 * until built.
 */
int lbm_stefan_batch_init(const lbm_stefan_params *params, int32_t count,
                          const double *const *T0, void *workspace,
                          size_t bytes, void *stream,
                          lbm_stefan_batch_t **out);

/*
 * Schedule: kernel variant (-1: default); blocks_per_cu 0 launches one
 * block per work item (in XCD-contiguous chunks of the item table), 1..32 a
 * persistent grid of blocks_per_cu x compute units walking the table; and
 * graph_steps (even, 0..1e5):
 * when > 0, lbm_stefan_batch_step replays a captured hipGraph of that many
 * launches (captured on first use) and launches any remainder directly.
 * Changing the variant resets statistics.
 */
int lbm_stefan_batch_set_schedule(lbm_stefan_batch_t *b, int32_t variant,
                                  int32_t blocks_per_cu, int32_t graph_steps);

/* Advance every instance nsteps (asynchronous on the batch's stream). */
int lbm_stefan_batch_step(lbm_stefan_batch_t *b, int64_t nsteps);

/* Per-instance statistics (out: host, count entries), as for a single
   lattice.  Waits for the stream.  Errors: ENAN, EDEVICE. */
int lbm_stefan_batch_stats(lbm_stefan_batch_t *b, lbm_stefan_stats *out);

/* Zero every instance's Newton and flux accumulators. */
int lbm_stefan_batch_reset_stats(lbm_stefan_batch_t *b);

/* Front (host, ny_k doubles, nullable) and energy (host, nullable) of one
   instance; as lbm_stefan_query_front. */
int lbm_stefan_batch_query_front(lbm_stefan_batch_t *b, int32_t inst,
                                 int32_t mode, double *front, double *energy);

/* One instance's field, as lbm_stefan_get_field. */
int lbm_stefan_batch_get_field(lbm_stefan_batch_t *b, int32_t inst,
                               int32_t what, void *host);

/* Bytes of all instances' current states together (autotune scratch). */
int lbm_stefan_batch_state_bytes(const lbm_stefan_batch_t *b, size_t *bytes);

/*
 * Autotuner of the batched kernel: times every (variant, blocks per CU in
 * {0 (one block per tile), 2, 4, 8}) pair for `steps` steps with HIP events, saving the states
 * to `scratch` (device, >= lbm_stefan_batch_state_bytes) and restoring
 * them after each trial; keeps the fastest pair (the graph length is
 * kept).  Outputs are nullable.  Resets statistics.  Waits for the stream.
 */
int lbm_stefan_batch_autotune(lbm_stefan_batch_t *b, void *scratch,
                              size_t scratch_bytes, int32_t steps,
                              int32_t *best_variant,
                              int32_t *best_blocks_per_cu,
                              double *best_ms_per_step);

/* Text of the batch's last error (NULL: as lbm_stefan_last_error(NULL)). */
const char *lbm_stefan_batch_last_error(const lbm_stefan_batch_t *b);

/* Free the batch (host memory and its graphs).  Waits for the stream. */
int lbm_stefan_batch_destroy(lbm_stefan_batch_t *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_STEFAN_H */
