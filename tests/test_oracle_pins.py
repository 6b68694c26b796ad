"""Pins of the CPU oracle to facts outside itself.

Each test checks the oracle against something the paper or the
mathematics fixes: printed numbers of the paper's 1D case, closed-form
solutions, invariants, algebraic reductions and brute force.  A plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import erfc

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DIR2 = ("dirichlet", "dirichlet", "periodic", "periodic")


def _prob1d(nx, tau, ste, delta, T0, walls=(1.0, -0.5), **kw):
    return synth.Problem(dim=1, q=3, nx=nx, ny=1, tau=tau, ste=ste,
                         delta=delta, bc=DIR2,
                         wall_T=(walls[0], walls[1], 0.0, 0.0),
                         T0=np.asarray(T0, dtype=float).reshape(1, nx), **kw)


# --------------------------------------------------------------------------
# lattice tables: the moments the Chapman-Enskog analysis needs (Section 5)

@pytest.mark.parametrize("dim,q", [(1, 3), (2, 5), (2, 9)])
def test_lattice_moments(dim, q):
    ex, ey, w, opp = O.lattice(dim, q)
    assert ex[0] == 0 and ey[0] == 0
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs((w * ex).sum()) < 1e-15 and abs((w * ey).sum()) < 1e-15
    # second moment (1/3) I: Lambda_2 = theta/3 I for f_eq = w theta
    assert abs((w * ex * ex).sum() - 1.0 / 3.0) < 1e-15
    if dim == 2:
        assert abs((w * ey * ey).sum() - 1.0 / 3.0) < 1e-15
        assert abs((w * ex * ey).sum()) < 1e-15
    for i in range(q):
        assert ex[opp[i]] == -ex[i] and ey[opp[i]] == -ey[i]
        assert w[opp[i]] == w[i]
    # all velocities distinct
    assert len({(a, b) for a, b in zip(ex, ey)}) == q


# --------------------------------------------------------------------------
# regularized liquid fraction (Section 4.1)

def test_phi_special_values():
    d = 0.02
    assert O.phi(0.0, 0.0, d) == 0.5
    assert abs(O.phi(0.3, 0.3, d) - 0.5) < 1e-16          # centred on tm
    assert abs(O.phi(d * math.atanh(0.5), 0.0, d) - 0.75) < 1e-15
    for th in (-0.05, -0.013, 0.004, 0.031):
        assert abs(O.phi(th, 0.0, d) + O.phi(-th, 0.0, d) - 1.0) < 1e-15
    assert O.phi(-1.0, 0.0, d) < 1e-40 and O.phi(1.0, 0.0, d) == 1.0
    # sharp limit: phi_delta -> Heaviside as delta -> 0
    assert O.phi(1e-3, 0.0, 1e-6) == 1.0 and O.phi(-1e-3, 0.0, 1e-6) == 0.0


def test_dphi_is_derivative_and_integrates_to_one():
    d = 0.01
    for th in (-0.03, -0.004, 0.0, 0.0021, 0.02):
        h = 1e-7
        fd = (O.phi(th + h, 0.0, d) - O.phi(th - h, 0.0, d)) / (2 * h)
        assert abs(O.dphi(th, 0.0, d) - fd) < 1e-6 * max(1.0, abs(fd))
    xs = np.linspace(-0.4, 0.4, 80001)
    vals = np.array([O.dphi(x, 0.0, d) for x in xs])
    integral = np.trapezoid(vals, xs)
    assert abs(integral - 1.0) < 1e-8


# --------------------------------------------------------------------------
# local Newton problem (eq. rhs_fl_2) against brute-force bisection

def _bisect_root(m0, th, ste, delta, tm=0.0):
    """Brute force: 200 halvings of t + phi(t)/Ste - m0 - phi(th)/Ste on a
    wide bracket (F is increasing)."""
    F = lambda t: t + O.phi(t, tm, delta) / ste - m0 - O.phi(th, tm, delta) / ste
    a, b = -10.0 - 2.0 / ste, 10.0 + 2.0 / ste
    assert F(a) < 0 < F(b)
    for _ in range(200):
        m = 0.5 * (a + b)
        if F(m) > 0:
            b = m
        else:
            a = m
    return 0.5 * (a + b)


def test_newton_matches_bisection_random():
    rng = np.random.Generator(np.random.PCG64(7))
    worst = 0.0
    for _ in range(3000):
        ste = math.exp(rng.uniform(math.log(0.01), math.log(1.0)))
        delta = math.exp(rng.uniform(math.log(1e-4), math.log(0.05)))
        th = rng.uniform(-1.0, 1.0)
        m0 = th + rng.uniform(-0.3, 0.3) * rng.choice([1e-3, 1e-1, 1.0])
        ref = _bisect_root(m0, th, ste, delta)
        got, it, conv = O.newton(m0, th, ste, 0.0, delta, 1e-12, 64)
        assert conv, (m0, th, ste, delta)
        worst = max(worst, abs(got - ref))
    assert worst < 2e-12


def test_plain_newton_cycles_and_safeguard_converges():
    # root in the mushy zone, start on the solid plateau, 1/Ste = 20 >> delta:
    # the paper's update jumps between c and c - 1/Ste and never settles.
    ste, delta, th = 0.05, 1e-3, -0.5
    m0 = 10.0 - O.phi(th, 0.0, delta) / ste
    t, it, conv = O.newton(m0, th, ste, 0.0, delta, 1e-12, 20, O.PLAIN)
    assert not conv and it == 20
    t, it, conv = O.newton(m0, th, ste, 0.0, delta, 1e-12, 20, O.SAFEGUARDED)
    assert conv
    assert abs(t - _bisect_root(m0, th, ste, delta)) < 1e-12


# --------------------------------------------------------------------------
# Neumann similarity solution (Section 2) against the Stefan problem itself

@pytest.mark.parametrize("ste", [0.01, 0.05, 0.1, 0.2857, 1.0])
def test_neumann_solution_solves_stefan_problem(ste):
    th0 = -0.5
    lam = O.stefan_lambda(ste, th0)
    t = 0.01
    xf = 2 * lam * math.sqrt(t)
    T = lambda x, tt: O.neumann_T(x, tt, lam, th0)
    assert abs(T(0.0, t) - 1.0) < 1e-14            # hot wall
    assert abs(T(xf * (1 - 1e-12), t)) < 1e-9      # melting temperature at x_f
    assert abs(T(xf * (1 + 1e-12), t)) < 1e-9
    assert abs(T(50.0, t) - th0) < 1e-12           # far field
    # heat equation on both sides (second differences)
    for x in (0.4 * xf, 0.8 * xf, 1.3 * xf, 2.5 * xf):
        h, k = 1e-4 * xf, 1e-6 * t
        Tt = (T(x, t + k) - T(x, t - k)) / (2 * k)
        Txx = (T(x + h, t) - 2 * T(x, t) + T(x - h, t)) / (h * h)
        assert abs(Tt - Txx) < 1e-4 * max(1.0, abs(Tt))
    # Stefan condition: -dT_l/dx + dT_s/dx = (1/Ste) dx_f/dt, one-sided
    h = 1e-7
    dl = (T(xf * (1 - 1e-13), t) - T(xf - h, t)) / h
    ds = (T(xf + h, t) - T(xf * (1 + 1e-13), t)) / h
    rhs = lam / math.sqrt(t) / ste
    assert abs(-dl + ds - rhs) < 2e-5 * rhs


# --------------------------------------------------------------------------
# invariants of the scheme

def _problems_for_invariants():
    rng = np.random.Generator(np.random.PCG64(3))
    out = []
    p1 = synth.stefan_1d(nx=64)
    out.append(p1.with_(T0=np.full((1, 64), -0.5)))
    n, m = 37, 23
    T0 = -0.5 + 0.02 * rng.standard_normal((m, n))
    T0[:, :4] = 0.3
    out.append(synth.Problem(dim=2, q=5, nx=n, ny=m, tau=0.7, ste=0.05,
                             delta=1.0 / (n - 1), bc=DIR2,
                             wall_T=(1.0, -0.5, 0.0, 0.0), T0=T0))
    out.append(synth.Problem(dim=2, q=9, nx=n, ny=m, tau=0.6, ste=0.02,
                             delta=1.5 / (n - 1),
                             bc=("dirichlet", "dirichlet", "bounceback",
                                 "bounceback"),
                             wall_T=(1.0, -0.5, 0.0, 0.0), T0=T0, max_it=32))
    out.append(synth.Problem(dim=2, q=9, nx=n, ny=m, tau=0.9, ste=0.3,
                             delta=0.05, bc=("bounceback",) * 4,
                             wall_T=(0.0,) * 4, T0=T0))
    out.append(synth.Problem(dim=2, q=5, nx=n, ny=m, tau=0.8, ste=0.2,
                             delta=0.03, bc=("periodic",) * 4,
                             wall_T=(0.0,) * 4, T0=T0))
    out.append(synth.Problem(dim=2, q=9, nx=n, ny=m, tau=0.8, ste=0.2,
                             delta=0.03,
                             bc=("dirichlet", "bounceback", "dirichlet",
                                 "bounceback"),
                             wall_T=(1.0, 0.0, 0.5, 0.0),
                             wall_profile=(np.linspace(0.5, 1.5, m), None,
                                           None, None), T0=T0))
    return out


@pytest.mark.parametrize("k", range(6))
def test_enthalpy_balance_every_step(k):
    """Summing the update over nodes: E(n+1) - E(n) = (populations set by
    the boundary closures) - (populations leaving), up to the Newton
    residual (Section 2, eq. eq-H; Section 4.1, eqs. rhs_fl_stag and
    rhs_fl_2)."""
    p = _problems_for_invariants()[k]
    f = O.init(p, p.T0)
    f, st, E, fl = O.run(p, f, 150, trace=True)
    dE = np.diff(E)
    bal = fl[:, 0] - fl[:, 1]
    scale = max(1.0, np.abs(E).max())
    assert np.max(np.abs(dE - bal)) < 2e-13 * p.nodes * scale / 100 + 1e-12
    if p.bc[0] == "periodic" and p.bc[2] == "periodic":
        assert np.all(fl == 0.0)
        assert np.max(np.abs(E - E[0])) < 1e-11 * scale
    assert st["nonconverged"] == 0
    assert st["max_residual"] < 1e-11


def test_residual_below_tolerance_every_node():
    p = synth.planar_2d(n=64, ny=16, nsteps=300, storage="f64")
    f = O.init(p, p.T0)
    f, st = O.run(p, f, 300)
    assert st["nonconverged"] == 0
    # F' >= 1, so |F| <= tol * F' is implied by quadratic convergence;
    # the observed residual is at rounding level of c ~ 1/Ste
    assert st["max_residual"] < 1e-12 * (1.0 + 1.0 / p.ste)
    assert st["max_it"] <= 32


# --------------------------------------------------------------------------
# special cases with closed forms

def test_linear_profile_is_exact_fixed_point():
    """f_i = w_i (theta - tau e_i.grad theta) with linear theta is a fixed
    point of the interior update (collision, pull, Newton with m0 = theta,
    zero source), and the wet-node Dirichlet closure reproduces it."""
    n, tau = 41, 0.73
    ex, ey, w, opp = O.lattice(1, 3)
    x = np.arange(n)
    b = -1.5 / (n - 1)
    th = 1.0 + b * x
    f = np.array([w[i] * (th - tau * ex[i] * b) for i in range(3)])[:, None, :]
    p = _prob1d(n, tau, 0.1, 0.02, th, walls=(1.0, -0.5))
    g, st = O.step(p, f)
    assert np.max(np.abs(g - f)) < 1e-15
    # the same on D2Q5 with bounce-back y walls (adiabatic): uniform in y
    ex, ey, w, opp = O.lattice(2, 5)
    m = 9
    f2 = np.array([w[i] * (th[None, :] - tau * ex[i] * b) * np.ones((m, 1))
                   for i in range(5)])
    p2 = synth.Problem(dim=2, q=5, nx=n, ny=m, tau=tau, ste=0.1, delta=0.02,
                       bc=("dirichlet", "dirichlet", "bounceback",
                           "bounceback"), wall_T=(1.0, -0.5, 0.0, 0.0),
                       T0=np.broadcast_to(th, (m, n)))
    g2, _ = O.step(p2, f2)
    assert np.max(np.abs(g2 - f2)) < 1e-15


def test_long_run_reaches_linear_steady_state():
    n, tau = 24, 1.0
    p = _prob1d(n, tau, 0.3, 0.02, np.full(n, -0.5))
    f = O.init(p, p.T0)
    f, st = O.run(p, f, 60000)
    T = O.temperature(p, f)[0]
    exact = 1.0 - 1.5 * np.arange(n) / (n - 1)
    assert np.max(np.abs(T - exact)) < 1e-12


@pytest.mark.parametrize("xwalls", [("dirichlet", "dirichlet"),
                                    ("dirichlet", "bounceback")])
@pytest.mark.parametrize("q,nx", [(5, 40), (9, 40)])
def test_2d_with_uniform_rows_equals_1d(q, nx, xwalls):
    """With y-uniform data and a periodic y axis, the sums of the D2Q5/D2Q9
    populations sharing an x velocity evolve as D1Q3 (weights 2/3, 1/6,
    1/6), and Dirichlet deficits shared by weight add up to the D1Q3 one.
    With a bounce-back x wall, every D2Q9 diagonal entering through it
    bounces back (its source also crosses the periodic seam at the first
    and last rows, which wraps), as the D1Q3 population does."""
    x = np.arange(nx) / (nx - 1)
    T1 = 0.4 * np.sin(3 * np.pi * x)        # crosses T_m = 0 twice
    bc = xwalls + ("periodic", "periodic")
    p1 = _prob1d(nx, 0.8, 0.1, 0.03, T1).with_(bc=bc)
    f1 = O.init(p1, p1.T0)
    f1, _ = O.run(p1, f1, 400)
    m = 6
    p2 = synth.Problem(dim=2, q=q, nx=nx, ny=m, tau=0.8, ste=0.1, delta=0.03,
                       bc=bc, wall_T=(1.0, -0.5, 0.0, 0.0),
                       T0=np.broadcast_to(T1, (m, nx)))
    f2 = O.init(p2, p2.T0)
    f2, _ = O.run(p2, f2, 400)
    T1f = O.temperature(p1, f1)[0]
    T2f = O.temperature(p2, f2)
    assert np.max(np.abs(T2f - T1f[None, :])) < 1e-13
    assert abs(T1f[-2] - T1[-2]) > 1e-3      # the far wall took part


def test_pure_diffusion_second_order_against_erfc():
    """Without latent heat (1/Ste -> 0) the scheme is BGK diffusion with
    diffusivity (tau - 1/2)/3 in lattice units (Section 5); the erfc
    solution of the heat equation is matched at second order in dx."""
    tau, t0, t_run = 0.8, 0.002, 0.01
    errs = []
    for n in (128, 256):
        dx = 1.0 / (n - 1)
        dt = (tau - 0.5) * dx * dx / 3.0
        x = np.arange(n) * dx
        Te = lambda t: -0.5 + 1.5 * erfc(x / (2.0 * np.sqrt(t)))
        nst = int(round(t_run / dt))
        p = _prob1d(n, tau, 1e12, 0.02, Te(t0))
        f = O.init(p, p.T0)
        f, st = O.run(p, f, nst)
        errs.append(np.max(np.abs(O.temperature(p, f)[0] - Te(t0 + nst * dt))))
    assert errs[1] < 1e-4
    assert 3.4 < errs[0] / errs[1] < 4.6


def test_bounce_back_preserves_mirror_symmetry():
    n, m = 31, 20
    rng = np.random.Generator(np.random.PCG64(11))
    T0 = -0.5 + 0.05 * rng.standard_normal((m, n))
    T0 = 0.5 * (T0 + T0[::-1, :])
    p = synth.Problem(dim=2, q=9, nx=n, ny=m, tau=0.7, ste=0.1,
                      delta=1.5 / (n - 1),
                      bc=("dirichlet", "dirichlet", "bounceback",
                          "bounceback"), wall_T=(1.0, -0.5, 0.0, 0.0),
                      T0=T0)
    f = O.init(p, p.T0)
    f, _ = O.run(p, f, 200)
    T = O.temperature(p, f)
    assert np.max(np.abs(T - T[::-1, :])) < 1e-13
    assert T[:, 1].max() > 0.0          # melting started near the hot wall


# --------------------------------------------------------------------------
# the paper's own 1D case (Section 6.1)

@pytest.mark.slow
def test_paper_1d_case_matches_printed_errors():
    g = json.load(open(os.path.join(GOLDEN, "paper_1d_case.json")))
    ste, th0, N, tau, delta = g["ste"], g["theta0"], g["nodes"], g["tau"], g["delta"]
    t_end = g["t_end_seconds"] * g["alpha_m2_per_s"] / g["length_m"] ** 2
    lam = O.stefan_lambda(ste, th0)
    t0 = (g["x_front_initial"] / (2 * lam)) ** 2
    dx = 1.0 / (N - 1)
    dt = (tau - 0.5) * dx * dx / 3.0
    nsteps = int(round((t_end - t0) / dt))
    x = np.arange(N) * dx
    p = _prob1d(N, tau, ste, delta, O.neumann_T(x, t0, lam, th0),
                walls=(1.0, th0))
    f = O.init(p, p.T0)
    f, st = O.run(p, f, nsteps)
    t = t0 + nsteps * dt
    err = np.max(np.abs(O.temperature(p, f)[0] - O.neumann_T(x, t, lam, th0)))
    assert abs(err / g["irebm_max_temperature_error"] - 1.0) < 0.15
    xf = O.front(p, f)[0]
    rel = abs(xf - 2 * lam * math.sqrt(t)) / (2 * lam * math.sqrt(t))
    lo, hi = g["irebm_front_error_band"]
    assert 0.8 * lo < rel < 1.2 * hi
    assert st["nonconverged"] == 0


@pytest.mark.slow
def test_regularization_converges_to_sharp_front():
    """delta -> 0: the front of the regularized problem approaches the sharp
    Neumann front (Section 6.1, effect of delta), and the temperature
    error shrinks with delta until the resolution floor."""
    n, tau, ste, th0 = 512, 0.8, 0.1, -0.5
    lam = O.stefan_lambda(ste, th0)
    dx = 1.0 / (n - 1)
    dt = (tau - 0.5) * dx * dx / 3.0
    nsteps = int(round(0.02 / dt))
    t = nsteps * dt
    x = np.arange(n) * dx
    xe = 2 * lam * math.sqrt(t)
    front_err, t_err = [], []
    for delta in (0.04, 0.02, 0.01, 0.005):
        p = _prob1d(n, tau, ste, delta, np.full(n, th0), walls=(1.0, th0))
        f = O.init(p, p.T0)
        f, st = O.run(p, f, nsteps)
        front_err.append(abs(O.front(p, f)[0] - xe))
        t_err.append(np.max(np.abs(O.temperature(p, f)[0] -
                                   O.neumann_T(x, t, lam, th0))))
    assert all(a > b for a, b in zip(front_err, front_err[1:])), front_err
    assert t_err[0] > t_err[1] > t_err[2], t_err
    # first order in delta away from the floor
    assert 1.5 < t_err[0] / t_err[1] < 2.5
