"""Pins of the oracle's Neumann closure (Section 4.2, eq. Neu_on_q) and
of the paper's 2D freezing case (Section 6.2), for both schemes.

eq. Neu_on_q fixes the zeroth moment of the pulled populations at a
Neumann wall node to the one at the interior neighbour across the wall
(the mirror node; the diagonal one at the corner of two Neumann walls).
Pinned by: the moment identity itself after one step, the reduction of
y-uniform D2Q5 data to D1Q3, the x <-> y symmetry of the quarter cavity,
the exact enthalpy balance, the uniform steady state, refusal of mixed
Neumann / bounce-back walls, and the paper's statement that the EEBM and
IREBM -5 C isotherms coincide in the 2D case.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

SCHEMES = ("irebm", "eebm")


def _quarter(n, q, scheme, T0=None, **kw):
    p = synth.freezing_cavity_2d(n=n, q=q, scheme=scheme, **kw)
    return p if T0 is None else p.with_(T0=T0)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q", [5, 9])
def test_wall_moment_equals_mirror_moment(q, scheme):
    """One step from a field that is equal across the Neumann walls: the
    new temperature of every Neumann wall node equals that of its mirror
    node (eq. Neu_on_q; for IREBM because phi(T) is then equal on both
    sides, for EEBM because the enthalpies are)."""
    n = 23
    rng = np.random.Generator(np.random.PCG64(3 + q))
    T0 = 0.6 * rng.standard_normal((n, n))
    T0[:, -1] = T0[:, -2]
    T0[-1, :] = T0[-2, :]
    T0[-1, -1] = T0[-2, -2]
    p = _quarter(n, q, scheme, T0=T0, delta=0.3)
    f, _ = O.step(p, O.init(p, T0))
    T = O.temperature(p, f)
    # x+ wall (x = n-1) and y+ wall, Dirichlet corners excluded
    assert np.max(np.abs(T[1:-1, -1] - T[1:-1, -2])) < 1e-13
    assert np.max(np.abs(T[-1, 1:-1] - T[-2, 1:-1])) < 1e-13
    assert abs(T[-1, -1] - T[-2, -2]) < 1e-13
    # and the closure is not a bounce-back or copy in disguise: the
    # temperature of the mirror differs from its own previous value
    assert np.max(np.abs(T[1:-1, -2] - T0[1:-1, -2])) > 1e-3


@pytest.mark.parametrize("scheme", SCHEMES)
def test_uniform_rows_with_neumann_y_walls_equal_1d(scheme):
    """y-uniform D2Q5 data between Neumann y walls: the closure returns
    the interior value of the unknown population, so the run equals D1Q3
    (weights 2/3, 1/6, 1/6 after summing equal x velocities); with a
    Neumann x+ wall on both."""
    nx, m = 37, 7
    lam = O.stefan_lambda(0.2, -0.5)
    x = np.arange(nx) / (nx - 1)
    T1 = O.neumann_T(x, 0.004, lam, -0.5)
    p1 = synth.Problem(dim=1, q=3, nx=nx, ny=1, tau=0.8, ste=0.2, delta=0.03,
                       bc=("dirichlet", "neumann", "periodic", "periodic"),
                       wall_T=(1.0, 0.0, 0.0, 0.0), T0=T1[None, :],
                       scheme=scheme)
    f1, _ = O.run(p1, O.init(p1, p1.T0), 400)
    p2 = synth.Problem(dim=2, q=5, nx=nx, ny=m, tau=0.8, ste=0.2, delta=0.03,
                       bc=("dirichlet", "neumann", "neumann", "neumann"),
                       wall_T=(1.0, 0.0, 0.0, 0.0),
                       T0=np.broadcast_to(T1, (m, nx)), scheme=scheme)
    f2, _ = O.run(p2, O.init(p2, p2.T0), 400)
    T1f = O.temperature(p1, f1)[0]
    assert np.max(np.abs(O.temperature(p2, f2) - T1f[None, :])) < 1e-13
    # the x+ Neumann wall held the front away from a fixed temperature
    assert abs(T1f[-1] - T1f[-2]) < 0.05 * abs(T1f[0] - T1f[-1])


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q", [5, 9])
def test_quarter_cavity_is_symmetric_about_the_diagonal(q, scheme):
    """Walls and data symmetric under x <-> y give a transposed-symmetric
    field: the closures treat the x and y walls alike (corner mirror on
    the diagonal, Dirichlet corners at the same temperature)."""
    n = 31
    rng = np.random.Generator(np.random.PCG64(17))
    T0 = 1.0 + 0.2 * rng.standard_normal((n, n))
    T0 = 0.5 * (T0 + T0.T)
    p = _quarter(n, q, scheme, T0=T0)
    f, _ = O.run(p, O.init(p, T0), 300)
    T = O.temperature(p, f)
    assert np.max(np.abs(T - T.T)) < 1e-12
    assert T.min() < 0.0 < T.max()          # a front is present


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q", [5, 9])
def test_enthalpy_balance_every_step(q, scheme):
    p = _quarter(29, q, scheme)
    f, st, E, fl = O.run(p, O.init(p, p.T0), 200, trace=True)
    dE = np.diff(E)
    assert np.max(np.abs(dE - (fl[:, 0] - fl[:, 1]))) < 1e-14 * np.abs(E).max()
    assert dE.sum() < 0.0                    # the cavity loses heat


@pytest.mark.parametrize("scheme", SCHEMES)
def test_freezing_reaches_the_uniform_wall_temperature(scheme):
    """Two walls at -2 and two Neumann walls: the steady state is uniform
    -2 (the liquid freezes completely)."""
    p = _quarter(9, 5, scheme, tau=1.0)
    f, _ = O.run(p, O.init(p, p.T0), 60000)
    T = O.temperature(p, f)
    assert np.max(np.abs(T + 2.0)) < 1e-12


def test_neumann_and_bounce_back_do_not_mix():
    p = _quarter(9, 5, "irebm").with_(
        bc=("dirichlet", "neumann", "bounceback", "bounceback"))
    with pytest.raises(ValueError):
        O.init(p, p.T0)
    with pytest.raises(ValueError):
        O.init(p.with_(scheme="eebm"), p.T0)


def _diag_isotherm(p, T, level):
    """Distance from the cold corner, along x = y, where T first rises
    through `level` (linear interpolation)."""
    d = np.diag(T)
    s = np.arange(p.nx) * p.dx * math.sqrt(2.0)
    k = int(np.argmax(d > level))
    return s[k - 1] + (s[k] - s[k - 1]) * (level - d[k - 1]) / (d[k] - d[k - 1])


@pytest.mark.slow
@pytest.mark.parametrize("q", [5, 9])
def test_paper_2d_case_eebm_and_irebm_isotherms_coincide(q):
    """Section 6.2, N = 201, t = 20 h: the -5 C isotherm (theta = -0.5) is
    the same for both methods (read as: within one cell along the
    diagonal), and both have it well inside the cavity."""
    pos = {}
    for scheme in SCHEMES:
        p = _quarter(201, q, scheme)
        f, st = O.run(p, O.init(p, p.T0), p.nsteps)
        T = O.temperature(p, f)
        pos[scheme] = _diag_isotherm(p, T, -0.5)
        assert T.min() >= -2.0 - 1e-12 and T.max() <= 1.0 + 1e-9
    d = abs(pos["irebm"] - pos["eebm"])
    print(f"D2Q{q}: isotherm -5 C on the diagonal at {pos}, |d| = {d:.2e}")
    assert d < p.dx
    assert 5 * p.dx < pos["irebm"] < 0.5 * p.nx * p.dx
