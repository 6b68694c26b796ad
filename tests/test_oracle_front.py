"""Pins of the oracle's zero-crossing front ("position of the interface",
Section 6.1): the first place along x, from x = 0, where T - T_m goes from
> 0 to <= 0, linearly interpolated between the two nodes; 0 when
T(0) <= T_m, and (nx - 1) dx when T stays above T_m.

The front functions only read the temperature of each node (the sum of
its populations, through Theta(H) in the explicit scheme), so each pin
builds a state whose temperature is a profile with a known crossing: a
linear profile (linear interpolation is then exact), integer-valued
profiles that touch T_m at a node or cross it more than once, the edge
rules, and the Neumann similarity solution of Section 2 (eq. exact
solution), both sampled on the lattice and approached by a run of the
scheme under refinement.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

DIR2 = ("dirichlet", "dirichlet", "periodic", "periodic")


def _state_2d(prob, T, seed=5):
    """Populations whose per-node sum is T (shape (ny, nx)): T split over
    the q planes by random positive fractions, so that a wrong plane
    stride or a transposed index changes the sums."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.2, 1.0, prob.q)
    a /= a.sum()
    return np.array([a[i] * T for i in range(prob.q)])


def _prob2d(q, nx, ny, tm=0.0, scheme="irebm", ste=0.1):
    return synth.Problem(dim=2, q=q, nx=nx, ny=ny, tau=0.7, ste=ste,
                         delta=0.01, bc=DIR2, wall_T=(1.0, -0.5, 0.0, 0.0),
                         tm=tm, scheme=scheme)


def _linear_rows(nx, ny, tm, seed=9):
    """Rows T = T_m + s (c - x) with crossing c inside (0, 1) and slope s
    drawn per row; returns (T, c)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.05, 0.95, ny)
    s = rng.uniform(0.3, 4.0, ny)
    x = np.arange(nx) / (nx - 1)
    return tm + s[:, None] * (c[:, None] - x[None, :]), c


@pytest.mark.parametrize("q", [5, 9])
@pytest.mark.parametrize("tm", [0.0, 0.25, -0.3])
def test_linear_rows_exact_crossing(q, tm):
    nx, ny = 41, 13
    p = _prob2d(q, nx, ny, tm=tm)
    T, c = _linear_rows(nx, ny, tm)
    xf = O.front(p, _state_2d(p, T), O.FRONT_CROSSING)
    assert xf.shape == (ny,)
    assert np.max(np.abs(xf - c)) < 1e-13


def test_linear_profile_1d():
    nx = 256
    x = np.arange(nx) / (nx - 1)
    T = 1.0 - 1.5 * x                       # crosses 0 at x = 2/3
    p = synth.stefan_1d(nx=nx)
    ex, ey, w, opp = O.lattice(1, 3)
    f = np.array([w[i] * T for i in range(3)])[:, None, :]
    xf = O.front(p, f, O.FRONT_CROSSING)
    assert abs(xf[0] - 2.0 / 3.0) < 1e-14


def test_node_touch_and_first_crossing_rule():
    """Integer profiles (exact sums): a crossing that lands on a node
    (T = T_m there) is that node; with several crossings the first one from
    x = 0 counts; the rows are independent."""
    nx = 16
    k = np.arange(nx, dtype=float)
    rows = [
        (k - 3.0) * (k - 7.0),               # zero at nodes 3 and 7
        -(k - 3.5) * (k - 7.5) * (k - 12.5),  # + - + - : three crossings
        -(k - 4.0) * (k - 9.5),              # starts at -36 (solid wall)
        5.0 - k,                             # zero at node 5
        np.where(k < 6, 2.0, -1.0),          # a step between nodes 5, 6
    ]
    T = np.array(rows)
    p = _prob2d(5, nx, len(rows))
    dx = p.dx
    xf = O.front(p, _state_2d(p, T), O.FRONT_CROSSING)
    # row 1: between nodes 3 and 4, T(3) = 0.5*4.5*9.5 = 21.375 and
    # T(4) = -(0.5*3.5*8.5) = -14.875
    t3, t4 = 21.375, -14.875
    expect = [3 * dx, (3 + t3 / (t3 - t4)) * dx, 0.0, 5 * dx,
              (5 + 2.0 / 3.0) * dx]
    assert np.max(np.abs(xf - np.array(expect))) < 1e-14


@pytest.mark.parametrize("tm", [0.0, 0.4])
def test_edge_rules(tm):
    nx = 21
    x = np.arange(nx) / (nx - 1)
    T = np.array([
        tm + 1.0 + x,              # stays above T_m: the far end
        tm - 0.5 + 0.0 * x,        # all below: 0
        tm + 0.0 * x,              # at T_m everywhere: T(0) <= T_m gives 0
        tm - 0.2 + 2.0 * x,        # cold at x = 0, warm inside: still 0
        tm + 1.0 - (x == 1.0) * 1.0,   # reaches T_m only at the last node
    ])
    p = _prob2d(9, nx, T.shape[0], tm=tm)
    xf = O.front(p, _state_2d(p, T), O.FRONT_CROSSING)
    dx = p.dx
    assert xf[0] == pytest.approx((nx - 1) * dx, abs=1e-15)
    assert xf[1] == 0.0 and xf[2] == 0.0 and xf[3] == 0.0
    assert xf[4] == pytest.approx((nx - 1) * dx, abs=1e-14)


def test_eebm_crossing_uses_theta_of_H():
    """Explicit scheme: the state carries the enthalpy H, and the front is
    that of Theta(H) (Section 3.4).  H = T + 1/Ste above T_m and H = T
    below gives Theta(H) = T, so a linear T crosses where it does; a
    plateau of mushy nodes (Theta = T_m) starts the front at its first
    node."""
    nx, ny, ste, tm = 41, 9, 0.05, 0.1
    p = _prob2d(5, nx, ny, tm=tm, scheme="eebm", ste=ste)
    T, c = _linear_rows(nx, ny, tm, seed=21)
    H = T + (T > tm) / ste
    xf = O.front(p, _state_2d(p, H), O.FRONT_CROSSING)
    assert np.max(np.abs(xf - c)) < 1e-12
    # mushy plateau on nodes 7..12 after liquid nodes
    H = np.full((ny, nx), tm - 0.3)
    H[:, :7] = tm + 1.0 / ste + 0.2
    H[:, 7:13] = tm + 0.5 / ste
    xf = O.front(p, _state_2d(p, H), O.FRONT_CROSSING)
    assert np.max(np.abs(xf - 7 * p.dx)) < 1e-14


@pytest.mark.parametrize("q", [7, 19])
@pytest.mark.parametrize("scheme", ["irebm", "eebm"])
def test_3d_rows_z_major(q, scheme):
    """3D: one front value per row along x, rows ordered [z][y]."""
    nx, ny, nz, ste, tm = 33, 4, 3, 0.2, 0.0
    p = synth.Problem(dim=3, q=q, nx=nx, ny=ny, nz=nz, tau=0.7, ste=ste,
                      delta=0.01, bc=DIR2, bc_z=("periodic", "periodic"),
                      wall_T=(1.0, -0.5, 0.0, 0.0), scheme=scheme)
    T, c = _linear_rows(nx, ny * nz, tm, seed=33)
    H = T + (T > tm) / ste if scheme == "eebm" else T
    ex, ey, ez, w, opp = O.lattice3(q)
    f = np.array([w[i] * H for i in range(q)]).reshape(q, nz, ny, nx)
    xf = O.front(p, f, O.FRONT_CROSSING)
    assert xf.shape == (nz, ny)
    assert np.max(np.abs(xf.reshape(-1) - c)) < 1e-12


@pytest.mark.parametrize("n", [256, 1024, 4096])
def test_sampled_neumann_profile_crossing(n):
    """The Neumann solution (Section 2) sampled on the nodes crosses 0
    between the two nodes around 2 lambda sqrt(t); the interpolated
    crossing lies in that cell, so within dx of the exact front."""
    ste, th0, t = 0.1, -0.5, 0.02
    lam = O.stefan_lambda(ste, th0)
    x = np.arange(n) / (n - 1)
    T = O.neumann_T(x, t, lam, th0)
    p = synth.stefan_1d(nx=n)
    ex, ey, w, opp = O.lattice(1, 3)
    f = np.array([w[i] * T for i in range(3)])[:, None, :]
    xe = 2 * lam * math.sqrt(t)
    k = int(math.floor(xe * (n - 1)))
    xf = O.front(p, f, O.FRONT_CROSSING)[0]
    assert k * p.dx <= xf <= (k + 1) * p.dx
    assert abs(xf - xe) < p.dx


def test_scheme_crossing_approaches_neumann_front():
    """A run of the scheme from the solid state (hot wall 1, far wall and
    initial temperature -1/2, Ste 0.1, delta four cells): the crossing front
    at t = 0.02 approaches 2 lambda sqrt(t) under refinement and stays
    within half a cell of it."""
    tau, ste, th0 = 0.8, 0.1, -0.5
    lam = O.stefan_lambda(ste, th0)
    errs = []
    for n in (128, 256, 512):
        dx = 1.0 / (n - 1)
        dt = (tau - 0.5) * dx * dx / 3.0
        nsteps = int(round(0.02 / dt))
        t = nsteps * dt
        p = synth.Problem(dim=1, q=3, nx=n, ny=1, tau=tau, ste=ste,
                          delta=4.0 * dx, bc=DIR2,
                          wall_T=(1.0, th0, 0.0, 0.0),
                          T0=np.full((1, n), th0), max_it=32)
        f = O.init(p, p.T0)
        f, st = O.run(p, f, nsteps)
        assert st["nonconverged"] == 0
        err = abs(O.front(p, f, O.FRONT_CROSSING)[0] - 2 * lam * math.sqrt(t))
        assert err < 0.5 * dx, (n, err, dx)
        errs.append(err)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 5e-4
