"""Pins of the oracle's 3D lattices (D3Q7, D3Q19) for IREBM (Algorithm 3)
and EEBM (Algorithm 2) to facts outside the 3D code.

The enthalpy formulation holds in 3D (Section 2) and the schemes are
written for DdQq lattices whose weights give the second moment T/3 times
the identity (Section 5, eq. lambda2).  Pinned by:
  * the moment conditions of the weight tables themselves;
  * reductions to the pinned 2D and 1D oracles: z-uniform data on a
    periodic z axis evolves exactly as on D2Q5 / D2Q9 (populations that
    share (e_x, e_y) sum to the 2D ones, weights included), and x, y
    uniform data between z walls as on D1Q3 (so the z closures are those
    of the 1D oracle);
  * invariance under a cyclic permutation of the axes;
  * the exact enthalpy balance of every step;
  * a linear temperature with an oblique gradient and its first-order
    populations, which the interior update must return unchanged;
  * the decay rate of a Fourier mode in the solid (pure diffusion with
    diffusivity (tau - 1/2)/3, along an axis and along the diagonal);
  * the Neumann closure's moment identity (eq. Neu_on_q) and the symmetry
    of the freezing octant.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

SCHEMES = ("irebm", "eebm")
Q2 = {7: 5, 19: 9}


def _tol(T, ste=1.0):
    """rounding bar of a run: both sides sum the same terms in different
    orders, and the latent heat enters with the factor 1/Ste"""
    return 1e-13 * max(1.0, float(np.abs(T).max())) * (1.0 + 1.0 / ste)


@pytest.mark.parametrize("q", [7, 19])
def test_weights_meet_the_moment_conditions(q):
    ex, ey, ez, w, opp = O.lattice3(q)
    e = np.stack([ex, ey, ez], axis=1)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    M2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(M2, np.eye(3) / 3.0, atol=1e-15)
    # every velocity once, opposites paired
    assert len({tuple(v) for v in e}) == q
    assert np.array_equal(e[opp], -e)
    assert np.all(np.abs(e).sum(axis=1) <= 2)
    if q == 19:
        # fourth moment of the standard D3Q19 set: isotropic w_i e^4 sum
        assert abs(np.sum(w * ex ** 4) - 1.0 / 3.0) < 1e-15
        assert abs(np.sum(w * ex ** 2 * ey ** 2) - 1.0 / 9.0) < 1e-15
    else:
        # D3Q7 is the rest velocity and the six faces of D3Q19
        e19 = np.stack(O.lattice3(19)[:3], axis=1)
        assert np.array_equal(e, e19[:7])


def _as_3d(p2, nz, **kw):
    """the 2D problem p2 as a 3D one, uniform along a periodic z axis"""
    T0 = np.broadcast_to(np.asarray(p2.T0, float).reshape(p2.ny, p2.nx),
                         (nz, p2.ny, p2.nx))
    return p2.with_(dim=3, q={5: 7, 9: 19}[p2.q], nz=nz,
                    bc_z=("periodic", "periodic"), T0=T0, **kw)


def _melt2d(p, seed=8):
    x = np.arange(p.nx) / (p.nx - 1)
    y = np.arange(p.ny) / p.ny
    T0 = 0.3 * np.sin(2 * np.pi * 2 * x)[None, :] * \
        np.cos(2 * np.pi * 1.5 * y)[:, None]
    T0 = T0 + synth.node_noise(seed, p.nodes, 0.05).reshape(p.ny, p.nx)
    return p.with_(T0=T0)


WALLS_2D = {
    "dirichlet_bounceback": lambda q: _melt2d(synth.cavity_2d(
        n=17, ny=11, storage="f64").with_(q=q, ste=0.2, delta=0.05)),
    "dirichlet_neumann": lambda q: _melt2d(synth.freezing_cavity_2d(
        n=13, q=q).with_(ny=9, tm=0.05)),
    "periodic_y": lambda q: _melt2d(synth.planar_2d(
        n=16, ny=8, storage="f64").with_(q=q, ste=0.3, delta=0.04)),
}


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("walls", sorted(WALLS_2D))
@pytest.mark.parametrize("q3", [7, 19])
def test_z_uniform_data_equal_2d(q3, walls, scheme):
    p2 = WALLS_2D[walls](Q2[q3]).with_(scheme=scheme)
    p3 = _as_3d(p2, nz=4)
    f2, s2 = O.run(p2, O.init(p2, p2.T0), 40)
    f3, s3 = O.run(p3, O.init(p3, p3.T0), 40)
    T2, T3 = O.temperature(p2, f2), O.temperature(p3, f3)
    assert np.max(np.abs(T3 - T2[None])) < _tol(T2, p2.ste)
    # the front sums liquid fractions, whose slope is at most 1/(2 delta)
    assert np.max(np.abs(O.front(p3, f3) - O.front(p2, f2)[None])) < \
        p2.dx * p2.nx * _tol(T2, p2.ste) / p2.delta
    for k in ("flux_in", "flux_out"):
        assert abs(s3[k] - 4 * s2[k]) < 1e-12 * max(1.0, abs(s2[k]))
    assert s3["max_it"] == s2["max_it"]
    assert s3["nonconverged"] == s2["nonconverged"] == 0
    assert np.ptp(T2) > 0.1                  # the field did evolve


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("zwalls", [("dirichlet", "dirichlet"),
                                    ("dirichlet", "neumann"),
                                    ("bounceback", "dirichlet")])
@pytest.mark.parametrize("q3", [7, 19])
def test_xy_uniform_data_between_z_walls_equal_1d(q3, zwalls, scheme):
    """The z closures are the 1D ones: data uniform in x and y, periodic x
    and y, walls on z, against D1Q3 along z."""
    nz = 23
    lam = O.stefan_lambda(0.2, -0.5)
    zc = np.arange(nz) / (nz - 1)
    T1 = O.neumann_T(zc, 0.004, lam, -0.5)
    wT = (1.0, -0.5)
    p1 = synth.Problem(dim=1, q=3, nx=nz, ny=1, tau=0.8, ste=0.2, delta=0.03,
                       bc=zwalls + ("periodic", "periodic"),
                       wall_T=wT + (0.0, 0.0), T0=T1[None, :], scheme=scheme)
    p3 = synth.Problem(dim=3, q=q3, nx=4, ny=3, nz=nz, tau=0.8, ste=0.2,
                       delta=0.03, bc=("periodic",) * 4, wall_T=(0.0,) * 4,
                       bc_z=zwalls, wall_T_z=wT, scheme=scheme,
                       T0=np.broadcast_to(T1[:, None, None], (nz, 3, 4)),
                       dx=1.0 / (nz - 1))
    f1, s1 = O.run(p1, O.init(p1, p1.T0), 300)
    f3, s3 = O.run(p3, O.init(p3, p3.T0), 300)
    T1f = O.temperature(p1, f1)[0]
    T3 = O.temperature(p3, f3)
    assert np.max(np.abs(T3 - T1f[:, None, None])) < _tol(T1f, p1.ste)
    assert s3["max_it"] == s1["max_it"]
    assert abs(T1f[1] - T1[1]) > 1e-3         # the profile moved


def _rotate(p, T0):
    """the same problem with axes renamed x -> z, y -> x, z -> y"""
    bc = (p.bc[2], p.bc[3], p.bc_z[0], p.bc_z[1])
    wT = (p.wall_T[2], p.wall_T[3], p.wall_T_z[0], p.wall_T_z[1])
    return p.with_(nx=p.ny, ny=p.nz, nz=p.nx, bc=bc, wall_T=wT,
                   bc_z=(p.bc[0], p.bc[1]),
                   wall_T_z=(p.wall_T[0], p.wall_T[1]),
                   T0=np.transpose(T0, (2, 0, 1)))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("walls", ["dirichlet_bounceback", "neumann"])
@pytest.mark.parametrize("q", [7, 19])
def test_cyclic_axis_permutation(q, walls, scheme):
    nx, ny, nz = 9, 7, 6
    T0 = 0.4 * synth.node_noise(31, nx * ny * nz, 1.0).reshape(nz, ny, nx)
    if walls == "neumann":
        bc, bcz = ("dirichlet", "neumann", "neumann", "neumann"), \
            ("periodic", "periodic")
    else:
        bc, bcz = ("dirichlet", "dirichlet", "bounceback", "bounceback"), \
            ("periodic", "periodic")
    p = synth.Problem(dim=3, q=q, nx=nx, ny=ny, nz=nz, tau=0.7, ste=0.3,
                      delta=0.05, bc=bc, wall_T=(0.9, -0.6, 0.0, 0.0),
                      bc_z=bcz, T0=T0, scheme=scheme, tm=0.02)
    pr = _rotate(p, T0)
    f, s = O.run(p, O.init(p, p.T0), 30)
    fr, sr = O.run(pr, O.init(pr, pr.T0), 30)
    T, Tr = O.temperature(p, f), O.temperature(pr, fr)
    assert np.max(np.abs(Tr - np.transpose(T, (2, 0, 1)))) < _tol(T, p.ste)
    for k in ("flux_in", "flux_out"):
        assert abs(s[k] - sr[k]) < 1e-12 * max(1.0, abs(s[k]))


WALLS_3D = {
    "cavity": dict(bc=("dirichlet", "dirichlet", "bounceback", "bounceback"),
                   bc_z=("bounceback", "bounceback")),
    "freezing": dict(bc=("dirichlet", "neumann", "dirichlet", "neumann"),
                     bc_z=("dirichlet", "neumann")),
    "mixed_periodic": dict(bc=("periodic", "periodic", "dirichlet",
                               "neumann"), bc_z=("neumann", "dirichlet")),
}


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("walls", sorted(WALLS_3D))
@pytest.mark.parametrize("q", [7, 19])
def test_enthalpy_balance_every_step(q, walls, scheme):
    n = 8
    T0 = 0.5 * synth.node_noise(5, n * n * (n + 1), 1.0).reshape(n + 1, n, n)
    p = synth.Problem(dim=3, q=q, nx=n, ny=n, nz=n + 1, tau=0.75, ste=0.25,
                      delta=0.06, wall_T=(1.0, -0.5, -0.8, 0.0),
                      wall_T_z=(0.7, -0.3), T0=T0, scheme=scheme,
                      **WALLS_3D[walls])
    f, st, E, fl = O.run(p, O.init(p, p.T0), 40, trace=True)
    dE = np.diff(E)
    assert np.max(np.abs(dE - (fl[:, 0] - fl[:, 1]))) < 1e-13 * np.abs(E).max()
    assert np.max(np.abs(dE)) > 1e-3
    assert st["nonconverged"] == 0


@pytest.mark.parametrize("q", [7, 19])
def test_linear_field_is_a_fixed_point_of_the_interior_update(q):
    """theta = a + g.x crossing T_m, f_i = w_i (theta - tau e_i.g): one
    step returns f unchanged at every node off the walls (the pulls are
    collisions of the same linear state; the Newton root is theta)."""
    ex, ey, ez, w, _ = O.lattice3(q)
    n, tau = 9, 0.83
    g = np.array([-0.11, 0.07, 0.05])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                          indexing="ij")
    th = 0.05 + g[0] * (x - 4) + g[1] * (y - 4) + g[2] * (z - 4)
    f = np.stack([w[i] * (th - tau * (ex[i] * g[0] + ey[i] * g[1] +
                                      ez[i] * g[2])) for i in range(q)])
    p = synth.Problem(dim=3, q=q, nx=n, ny=n, nz=n, tau=tau, ste=0.2,
                      delta=0.05, bc=("dirichlet",) * 4, wall_T=(0.3,) * 4,
                      bc_z=("dirichlet", "dirichlet"), wall_T_z=(0.3, 0.3),
                      T0=th)
    out, st = O.step(p, f)
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.max(np.abs(out[inner] - f[inner])) < 1e-15
    assert th.min() < 0.0 < th.max()
    # a wall node does change (its closure targets 0.3)
    assert np.max(np.abs(out - f)) > 1e-2


def _mode_rate(q, kvec, n, tau, steps=(100, 300)):
    """decay rate per step / |k|^2 of a small Fourier mode in the solid"""
    nz, ny, nx = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    ph = 2 * np.pi * (kvec[0] * x / nx + kvec[1] * y / ny + kvec[2] * z / nz)
    k2 = sum((2 * np.pi * kvec[a] / n[2 - a]) ** 2 for a in range(3))
    p = synth.Problem(dim=3, q=q, nx=nx, ny=ny, nz=nz, tau=tau, ste=0.1,
                      delta=0.02, bc=("periodic",) * 4, wall_T=(0.0,) * 4,
                      T0=-10.0 + 1e-3 * np.cos(ph))
    f = O.init(p, p.T0)
    amps = []
    done = 0
    for s in steps:
        f, _ = O.run(p, f, s - done)
        done = s
        amps.append(np.sum((O.temperature(p, f) + 10.0) * np.cos(ph)))
    return math.log(amps[0] / amps[1]) / (steps[1] - steps[0]) / k2


@pytest.mark.parametrize("q", [7, 19])
def test_fourier_mode_decays_with_diffusivity_tau_minus_half_over_3(q):
    """In the solid the step is BGK diffusion; a long-wave mode decays as
    exp(-D k^2 t) with D = (tau - 1/2)/3 (the tau relation of Section 5),
    along an axis and along the cube diagonal (isotropy), up to O(k^2)
    lattice corrections (0.1% and 0.6% here; a face weight of 1/8, or
    swapped D3Q19 weights, would be off by 25% or more)."""
    tau = 0.9
    D = (tau - 0.5) / 3.0
    axial = _mode_rate(q, (0, 0, 1), (32, 3, 3), tau)
    diag = _mode_rate(q, (1, 1, 1), (24, 24, 24), tau, steps=(60, 160))
    assert abs(axial / D - 1.0) < 0.015, axial / D
    assert abs(diag / D - 1.0) < 0.02, diag / D


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q", [7, 19])
def test_neumann_wall_moment_equals_mirror_moment(q, scheme):
    """One step from a field equal across the x+, y+ and z+ Neumann faces:
    every Neumann node off the Dirichlet faces gets the temperature of its
    mirror (eq. Neu_on_q), edges and the corner included."""
    n = 9
    rng = np.random.Generator(np.random.PCG64(7 + q))
    T0 = 0.6 * rng.standard_normal((n, n, n))
    T0[:, :, -1] = T0[:, :, -2]
    T0[:, -1, :] = T0[:, -2, :]
    T0[-1, :, :] = T0[-2, :, :]
    p = synth.freezing_cube_3d(n=n, q=q, scheme=scheme, delta=0.3).with_(
        T0=T0)
    T = O.temperature(p, O.step(p, O.init(p, T0))[0])
    i = slice(1, None)
    assert np.max(np.abs(T[i, i, -1] - T[i, i, -2])) < 1e-13
    assert np.max(np.abs(T[i, -1, i] - T[i, -2, i])) < 1e-13
    assert np.max(np.abs(T[-1, i, i] - T[-2, i, i])) < 1e-13
    assert abs(T[-1, -1, -1] - T[-2, -2, -2]) < 1e-13
    assert np.max(np.abs(T[1:-1, 1:-1, -2] - T0[1:-1, 1:-1, -2])) > 1e-3


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q", [7, 19])
def test_freezing_octant_is_symmetric_under_axis_permutations(q, scheme):
    n = 11
    p = synth.freezing_cube_3d(n=n, q=q, scheme=scheme)
    f, st = O.run(p, O.init(p, p.T0), 60)
    T = O.temperature(p, f)
    for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)):
        assert np.max(np.abs(T - np.transpose(T, perm))) < 1e-12
    assert T.min() < 0.0 < T.max()
    assert st["nonconverged"] == 0


def test_invalid_3d_problems_are_refused():
    p = synth.freezing_cube_3d(n=5, q=7)
    bad = [p.with_(nz=2), p.with_(q=9), p.with_(bc_z=("periodic", "dirichlet")),
           p.with_(bc_z=("bounceback", "neumann")),
           p.with_(wall_profile=(np.ones(5), None, None, None)),
           p.with_(scheme="ilfbm")]
    for b in bad:
        with pytest.raises(ValueError):
            O.init(b, np.zeros(b.field_shape))
