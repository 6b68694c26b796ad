"""Seeded synthetic workloads for the IREBM Stefan-problem step.

This module only describes problems and draws their seeded inputs (initial
temperature fields, wall profiles, per-instance parameter tables).  It
holds none of the method's arithmetic, and it is the one module that both
the GPU path's callers and the CPU oracle's callers use.

Conventions (the problem statement of Section 2 in scaled form):
  * temperatures are the scaled theta = (T - T_f)/(T_h - T_f): hot wall 1,
    melting temperature 0;
  * ``nx`` counts nodes on x in [0, 1], so dx = 1/(nx - 1); wall nodes are
    lattice nodes; a periodic y (or z) axis of ny nodes has period ny*dx;
  * 3D lattices (dim 3, D3Q7 or D3Q19) add ``nz`` and the z walls; fields
    are [z][y][x];
  * ``delta`` (the width of the regularized liquid fraction) is in
    temperature units; workloads quoted in cells use delta = cells * dx.

Random draws:
  * node noise: splitmix64 (Steele, Lea, Flood 2014) of (seed XOR node
    index), top 53 bits as a uniform in [0, 1), mapped to [-a, a];
  * parameter tables: numpy PCG64(seed), drawing per instance in the
    order (size, Ste, delta in cells, tau).
"""
from dataclasses import dataclass, field, replace
import math

import numpy as np

DEFAULT_SEED = 20250519

BC_NAMES = ("dirichlet", "bounceback", "periodic", "neumann")


@dataclass
class Problem:
    """One Stefan-problem instance on a DdQq lattice."""
    dim: int
    q: int
    nx: int
    ny: int
    tau: float
    ste: float
    delta: float
    bc: tuple            # x-, x+, y-, y+ in BC_NAMES
    wall_T: tuple        # Dirichlet temperature per wall
    tm: float = 0.0
    wall_profile: tuple = (None, None, None, None)
    tol: float = 1e-12
    max_it: int = 20
    newton_mode: str = "safeguarded"
    storage: str = "f64"  # population storage: "f64" or "f32"
    T0: object = None     # initial temperature: (ny, nx) array or scalar
    nsteps: int = 0
    name: str = ""
    dx: float = field(default=None)
    scheme: str = "irebm"  # "irebm" (Algorithm 3) or "eebm" (Algorithm 2)
    nz: int = 1            # 3D lattices: nodes along z
    bc_z: tuple = ("periodic", "periodic")   # z-, z+ (3D)
    wall_T_z: tuple = (0.0, 0.0)

    def __post_init__(self):
        if self.dx is None:
            self.dx = 1.0 / (self.nx - 1)

    @property
    def nodes(self):
        return self.nx * self.ny * (self.nz if self.dim == 3 else 1)

    @property
    def field_shape(self):
        """shape of a node field: (ny, nx), or (nz, ny, nx) in 3D"""
        if self.dim == 3:
            return (self.nz, self.ny, self.nx)
        return (self.ny, self.nx)

    def with_(self, **kw):
        return replace(self, **kw)


def splitmix64(x):
    """splitmix64 output for each uint64 in x (wrapping arithmetic)."""
    z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def node_noise(seed, n, amplitude):
    """n uniforms in [-amplitude, amplitude] from splitmix64(seed ^ k)."""
    with np.errstate(over="ignore"):
        k = np.arange(n, dtype=np.uint64)
        u = splitmix64(np.uint64(seed) ^ k) >> np.uint64(11)
    return amplitude * (2.0 * (u.astype(np.float64) * 2.0 ** -53) - 1.0)


def stefan_1d(nx=256, nsteps=20000):
    """1D two-phase melting, D1Q3, FP64: tau 0.8, Ste 0.1, delta 0.02,
    solid at -0.5, hot wall +1 at x = 0, -0.5 at x = 1, Newton tol 1e-12
    with at most 20 iterations."""
    return Problem(dim=1, q=3, nx=nx, ny=1, tau=0.8, ste=0.1, delta=0.02,
                   bc=("dirichlet", "dirichlet", "periodic", "periodic"),
                   wall_T=(1.0, -0.5, 0.0, 0.0), tol=1e-12, max_it=20,
                   storage="f64", T0=np.full((1, nx), -0.5), nsteps=nsteps,
                   name=f"stefan1d_d1q3_f64_n{nx}")


def planar_2d(n=2048, ny=None, nsteps=10000, seed=DEFAULT_SEED,
              storage="f32"):
    """2D planar-front melting, D2Q5: y periodic, x = 0 at +1, x = 1 at
    -0.5, initial -0.5 plus seeded noise of +-1e-3, Ste 0.05, delta one
    cell, tau 0.7."""
    ny = n if ny is None else ny
    T0 = -0.5 + node_noise(seed, n * ny, 1e-3).reshape(ny, n)
    return Problem(dim=2, q=5, nx=n, ny=ny, tau=0.7, ste=0.05,
                   delta=1.0 / (n - 1),
                   bc=("dirichlet", "dirichlet", "periodic", "periodic"),
                   wall_T=(1.0, -0.5, 0.0, 0.0), tol=1e-12, max_it=32,
                   storage=storage, T0=T0, nsteps=nsteps,
                   name=f"planar2d_d2q5_{storage}_{n}x{ny}")


def cavity_ste(seed=DEFAULT_SEED):
    """Stefan number of the cavity workload: log-uniform in [0.01, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return float(math.exp(rng.uniform(math.log(0.01), math.log(1.0))))


def cavity_2d(n=8192, ny=None, nsteps=2000, seed=DEFAULT_SEED,
              storage="f32"):
    """2D melting in a square cavity heated at one wall, D2Q9: x = 0 at +1,
    x = 1 at -0.5, adiabatic (bounce-back) y walls, initial -0.5,
    Ste log-uniform from the seed, delta 1.5 cells, tau 0.6."""
    ny = n if ny is None else ny
    return Problem(dim=2, q=9, nx=n, ny=ny, tau=0.6, ste=cavity_ste(seed),
                   delta=1.5 / (n - 1),
                   bc=("dirichlet", "dirichlet", "bounceback", "bounceback"),
                   wall_T=(1.0, -0.5, 0.0, 0.0), tol=1e-12, max_it=32,
                   storage=storage, T0=-0.5, nsteps=nsteps,
                   name=f"cavity2d_d2q9_{storage}_{n}x{ny}")


# the 2D case of Section 6.2 in scaled units: lengths in L = 1 m,
# temperatures in T_i - T_f = 10 K from T_f = 0, time in L^2/alpha
FREEZE_STE = 1.762 * 10.0 / 338.0          # c (T_i - T_f) / h_sl = 0.0521
FREEZE_T_END = 20.0 * 3600.0 * 1.26e-6     # 20 h, alpha = 1.26e-6 m^2/s
FREEZE_SIDE = 4.0                          # quarter of the 8 m cavity


def freezing_cavity_2d(n=201, q=5, storage="f64", scheme="irebm",
                       delta=0.02, tau=0.84, t_end=FREEZE_T_END):
    """The paper's 2D case (Section 6.2): the lower-left quarter of a
    square cavity of water at 10 C cooled to -20 C on all sides.  A 4 x 4
    square of n x n nodes (dx = 4/(n - 1)), Dirichlet -2 on the x- and y-
    walls, homogeneous Neumann (symmetry, eq. Neu_on_q) on x+ and y+,
    liquid at +1 initially, Ste 0.0521, delta 0.02, tau 0.84; the step
    count reaches t_end (20 h by default) with dt = (tau - 1/2) dx^2 / 3."""
    dx = FREEZE_SIDE / (n - 1)
    dt = (tau - 0.5) * dx * dx / 3.0
    return Problem(dim=2, q=q, nx=n, ny=n, tau=tau, ste=FREEZE_STE,
                   delta=delta,
                   bc=("dirichlet", "neumann", "dirichlet", "neumann"),
                   wall_T=(-2.0, 0.0, -2.0, 0.0), tol=1e-12, max_it=32,
                   storage=storage, T0=np.ones((n, n)),
                   nsteps=int(round(t_end / dt)), dx=dx, scheme=scheme,
                   name=f"freeze2d_d2q{q}_{scheme}_{storage}_{n}")


def batch_table(count=512, seed=DEFAULT_SEED, sizes=None, nsteps=5000,
                storage="f32", noise=True):
    """``count`` independent D2Q5 instances: square sizes uniform in
    {64, 128, ..., 1024}, Ste log-uniform in [0.01, 1], delta uniform in
    [0.5, 2] cells, tau uniform in [0.55, 1.0]; boundaries as planar_2d.
    ``sizes`` restricts the size choices (for small test batches)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    choices = np.arange(64, 1025, 64) if sizes is None else np.asarray(sizes)
    probs = []
    for k in range(count):
        n = int(rng.choice(choices))
        ste = float(math.exp(rng.uniform(math.log(0.01), math.log(1.0))))
        cells = float(rng.uniform(0.5, 2.0))
        tau = float(rng.uniform(0.55, 1.0))
        T0 = None
        if noise:
            T0 = -0.5 + node_noise(seed ^ (k + 1), n * n, 1e-3).reshape(n, n)
        probs.append(Problem(
            dim=2, q=5, nx=n, ny=n, tau=tau, ste=ste, delta=cells / (n - 1),
            bc=("dirichlet", "dirichlet", "periodic", "periodic"),
            wall_T=(1.0, -0.5, 0.0, 0.0), tol=1e-12, max_it=32,
            storage=storage, T0=T0 if noise else np.full((n, n), -0.5),
            nsteps=nsteps, name=f"batch{k}_d2q5_{storage}_{n}"))
    return probs


def wall_target_profile(ny, seed=DEFAULT_SEED, amplitude=0.1, modes=4):
    """Seeded hot-wall profile 1 + a * sum_k a_k sin(2 pi k y/ny + p_k),
    a_k ~ U[-1, 1], p_k ~ U[0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    a = rng.uniform(-1.0, 1.0, modes)
    ph = rng.uniform(0.0, 2.0 * math.pi, modes)
    y = np.arange(ny)
    s = sum(a[k] * np.sin(2.0 * math.pi * (k + 1) * y / ny + ph[k])
            for k in range(modes))
    return 1.0 + amplitude * s


def adjoint_2d(n=512, ny=None, nsteps=4096, storage="f32"):
    """Inverse problem workload: D2Q5, periodic y, hot-wall profile T_w(y)
    (initial guess 1), x = 1 at -0.5, initial -0.5, tau 0.8, Ste 0.2,
    delta 1.5 cells."""
    ny = n if ny is None else ny
    return Problem(dim=2, q=5, nx=n, ny=ny, tau=0.8, ste=0.2,
                   delta=1.5 / (n - 1),
                   bc=("dirichlet", "dirichlet", "periodic", "periodic"),
                   wall_T=(1.0, -0.5, 0.0, 0.0),
                   wall_profile=(np.ones(ny), None, None, None),
                   tol=1e-12, max_it=32, storage=storage,
                   T0=np.full((ny, n), -0.5), nsteps=nsteps,
                   name=f"adjoint2d_d2q5_{storage}_{n}x{ny}")


def cavity_3d(n=512, ny=None, nz=None, q=19, nsteps=200, seed=DEFAULT_SEED,
              storage="f32", scheme="irebm"):
    """3D melting in a cube heated at one face, D3Q19 (or D3Q7): x = 0 at
    +1, x = 1 at -0.5, adiabatic (bounce-back) y and z walls, initial -0.5
    plus seeded noise of +-1e-3, Ste log-uniform from the seed (as the 2D
    cavity), delta 1.5 cells, tau 0.6."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    T0 = -0.5 + node_noise(seed, n * ny * nz, 1e-3).reshape(nz, ny, n)
    return Problem(dim=3, q=q, nx=n, ny=ny, nz=nz, tau=0.6,
                   ste=cavity_ste(seed), delta=1.5 / (n - 1),
                   bc=("dirichlet", "dirichlet", "bounceback", "bounceback"),
                   bc_z=("bounceback", "bounceback"),
                   wall_T=(1.0, -0.5, 0.0, 0.0), tol=1e-12, max_it=32,
                   storage=storage, T0=T0, nsteps=nsteps, scheme=scheme,
                   name=f"cavity3d_d3q{q}_{scheme}_{storage}_{n}x{ny}x{nz}")


def freezing_cube_3d(n=61, q=7, storage="f64", scheme="irebm", delta=0.02,
                     tau=0.84, t_end=FREEZE_T_END):
    """The freezing case of Section 6.2 taken to 3D: one octant of a cube
    of water at 10 C cooled to -20 C on every face, so Dirichlet -2 on the
    x-, y- and z- faces and symmetry (Neumann, eq. Neu_on_q) on x+, y+ and
    z+; 4 x 4 x 4 in units of 1 m, n nodes per edge, other parameters as
    freezing_cavity_2d."""
    dx = FREEZE_SIDE / (n - 1)
    dt = (tau - 0.5) * dx * dx / 3.0
    return Problem(dim=3, q=q, nx=n, ny=n, nz=n, tau=tau, ste=FREEZE_STE,
                   delta=delta,
                   bc=("dirichlet", "neumann", "dirichlet", "neumann"),
                   bc_z=("dirichlet", "neumann"),
                   wall_T=(-2.0, 0.0, -2.0, 0.0), wall_T_z=(-2.0, 0.0),
                   tol=1e-12, max_it=32, storage=storage,
                   T0=np.ones((n, n, n)), nsteps=int(round(t_end / dt)),
                   dx=dx, scheme=scheme,
                   name=f"freeze3d_d3q{q}_{scheme}_{storage}_{n}")
