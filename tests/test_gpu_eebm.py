"""GPU parity of the explicit enthalpy based method (EEBM, Section 3.4,
Algorithm 2), called through the C ABI, against the CPU FP64 oracle.

The kernel keeps the post-collision populations between steps; the
oracle keeps Algorithm 2's f.  Both start from the equilibrium, which the
collision leaves unchanged, so after n steps the GPU state equals the
oracle's collision of its state (oracle.eebm_collide): the planes are
compared element by element, with the temperature, energy, fronts and
boundary fluxes.

Bars: FP64 storage, 1e-12 relative to the stored zeroth moment (the
enthalpy H, which holds the latent heat 1/Ste as well as T); FP32 storage
(per-node math in FP64), 1e-5 relative to it, and fronts within one cell.
"""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _eebm(prob):
    return prob.with_(scheme="eebm")


def _gpu_run(prob, nsteps, variant=-1, state=None):
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob, variant=variant)
    if state is not None:
        g.set_state(state)
    st = g.step(nsteps, stats=True)
    out = {
        "state": g.state().astype(np.float64),
        "T": g.temperature(),
        "front": g.front("integral"),
        "cross": g.front("crossing"),
        "energy": g.energy(),
        "stats": st,
    }
    g.close()
    return out


def _oracle_run(prob, nsteps, f=None):
    f = O.init(prob, prob.T0) if f is None else f
    f, st = O.run(prob, f, nsteps)
    return {
        "state": O.eebm_collide(prob, f),
        "H": f.sum(axis=0),
        "T": O.temperature(prob, f),
        "front": O.front(prob, f, O.FRONT_INTEGRAL),
        "cross": O.front(prob, f, O.FRONT_CROSSING),
        "energy": O.energy(prob, f),
        "stats": st,
    }


def _crossing_well_posed(prob, T, cross, err):
    """Rows whose zero-crossing front is a continuous function of T at
    the observed error: no node up to the crossing cell within a few
    errors of T_m, unless it sits exactly on the mushy plateau on both
    sides (Theta is then T_m exactly)."""
    ok = np.ones(prob.ny, dtype=bool)
    margin = 8.0 * max(err, 1e-16)
    for y in range(prob.ny):
        k = int(min(prob.nx - 1, np.floor(cross[y] / prob.dx) + 1))
        d = np.abs(T[y, :k + 1] - prob.tm)
        if np.any((d <= margin) & (d > 0.0)):
            ok[y] = False
    return ok


def _compare(prob, g, o, tol):
    Hs = max(1.0, np.max(np.abs(o["H"])))
    dS = np.max(np.abs(g["state"] - o["state"]))
    dT = np.max(np.abs(g["T"] - o["T"]))
    print(f"{prob.name}: max|dOmega| = {dS:.3e}, max|dT| = {dT:.3e} "
          f"(H scale {Hs:.3g})", flush=True)
    assert dS <= tol * Hs
    assert dT <= tol * Hs
    st = g["stats"]
    assert st["max_newton_it"] == 0 and st["nonconverged"] == 0
    assert st["max_residual"] == 0.0
    # the liquid-fraction integral moves by at most dx Ste sum_x w_x |dH|
    dH = np.abs(g["state"].sum(axis=0) - o["H"])
    w = np.ones(prob.nx)
    w[[0, -1]] = 0.5
    bound = prob.dx * prob.ste * (dH * w[None, :]).sum(axis=1)
    fr = np.abs(g["front"] - o["front"])
    assert np.all(fr <= 2 * bound + 1e-13 * np.maximum(np.abs(o["front"]),
                                                        prob.dx))
    ok = _crossing_well_posed(prob, o["T"], o["cross"], dT)
    assert ok.sum() >= prob.ny // 2
    cr = np.abs(g["cross"] - o["cross"])
    if prob.storage == "f64":
        assert np.all(cr[ok] <= 1e-9 * np.maximum(np.abs(o["cross"][ok]),
                                                  prob.dx))
        assert abs(g["energy"] - o["energy"]) <= \
            10 * TOL64 * max(1.0, abs(o["energy"]))
        # each step's boundary flux sums about q * perimeter populations of
        # size up to H, in different orders on the two sides: rounding of
        # at most steps * terms * eps * H, far above 1e-12 of a flux whose
        # inflow and outflow nearly cancel (all bounce-back walls)
        terms = prob.q * (2 * (prob.nx + prob.ny) if prob.dim == 2 else 2)
        fbar = max(1, st["steps"]) * terms * 2.2e-16 * Hs
        for k in ("flux_in", "flux_out"):
            a, b = st[k], o["stats"][k]
            assert abs(a - b) <= fbar + 1e-12 * abs(b), (k, a, b)
    else:
        assert np.all(cr[ok] <= prob.dx), cr[ok].max()
        assert abs(g["energy"] - o["energy"]) <= tol * Hs * prob.nodes


def _melt_field(prob, seed=5):
    """Stress input: smooth field around T_m plus seeded noise, so that
    nodes sit in all three branches of Theta (solid, mushy plateau,
    liquid) and cross between them during the run."""
    x = np.arange(prob.nx) / (prob.nx - 1)
    y = np.arange(prob.ny) / prob.ny
    T0 = (prob.tm + 0.2 * np.sin(2 * np.pi * 2 * x)[None, :] *
          np.cos(2 * np.pi * 3 * y)[:, None])
    T0 = T0 + synth.node_noise(seed, prob.nodes, 0.05).reshape(prob.ny,
                                                              prob.nx)
    return prob.with_(T0=T0)


CASES = [
    ("d1q3_stefan", lambda s: synth.stefan_1d(nx=257).with_(storage=s), 3000),
    ("d2q5_planar_ragged", lambda s: synth.planar_2d(n=131, ny=67,
                                                     storage=s), 600),
    ("d2q9_cavity_ragged", lambda s: synth.cavity_2d(n=150, ny=77,
                                                     storage=s), 600),
    ("d2q9_melt_all_bounceback", lambda s: _melt_field(synth.cavity_2d(
        n=97, ny=70, storage=s)).with_(bc=("bounceback",) * 4), 300),
    ("d2q5_melt_all_periodic", lambda s: _melt_field(synth.planar_2d(
        n=70, ny=45, storage=s)).with_(bc=("periodic",) * 4), 300),
    ("d2q9_melt_mixed_profile", lambda s: _melt_field(synth.cavity_2d(
        n=90, ny=66, storage=s)).with_(
            bc=("dirichlet", "bounceback", "dirichlet", "bounceback"),
            tm=0.1,
            wall_profile=(0.5 + 0.4 * np.sin(np.linspace(0, 3, 66)), None,
                          0.1 * np.cos(np.linspace(0, 5, 90)), None)), 300),
    ("d2q9_melt_bounceback_x_periodic_y", lambda s: _melt_field(
        synth.cavity_2d(n=81, ny=46, storage=s)).with_(
            bc=("bounceback", "bounceback", "periodic", "periodic")), 300),
    ("d2q5_tiny_3x3", lambda s: synth.planar_2d(n=3, ny=3, storage=s), 40),
]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_small_lattices_against_oracle(case, storage):
    name, make, steps = CASES[case]
    prob = _eebm(make(storage)).with_(name=f"eebm_{name}_{storage}")
    _compare(prob, _gpu_run(prob, steps), _oracle_run(prob, steps),
             TOL64 if storage == "f64" else TOL32)


@pytest.mark.parametrize("q", [3, 5, 9])
def test_one_step_from_random_states(q):
    """One step from random populations: enthalpies spread over the
    solid branch, the mushy plateau and the liquid branch of Theta (and
    exactly on its ends), Dirichlet walls on both sides of T_m."""
    rng = np.random.Generator(np.random.PCG64(100 + q))
    if q == 3:
        prob = synth.stefan_1d(nx=203)
    else:
        prob = (synth.planar_2d if q == 5 else synth.cavity_2d)(
            n=133, ny=71, storage="f64")
        prob = prob.with_(bc=("dirichlet", "bounceback", "dirichlet",
                              "bounceback"),
                          wall_profile=(rng.uniform(-0.3, 0.3, prob.ny), None,
                                        rng.uniform(-0.3, 0.3, prob.nx), None))
    prob = _eebm(prob).with_(name=f"eebm_random_q{q}", tm=0.05)
    ex, ey, w, opp = O.lattice(prob.dim, q)
    H = prob.tm + rng.uniform(-1.0, 1.0 + 2.0 / prob.ste, (prob.ny, prob.nx))
    H.flat[rng.integers(0, H.size, 40)] = prob.tm
    H.flat[rng.integers(0, H.size, 40)] = prob.tm + 1.0 / prob.ste
    f = np.array([w[i] * H + 0.05 * rng.standard_normal(H.shape)
                  for i in range(q)])
    f[0] += H - f.sum(axis=0)
    o = _oracle_run(prob, 1, f=f)
    g = _gpu_run(prob, 1, state=O.eebm_collide(prob, f))
    _compare(prob, g, o, TOL64)


def test_variants_bitwise_identical():
    """The per-node arithmetic does not depend on the tile shape or on
    the two-step kernel (odd step count: the last launch single)."""
    from paper_2505_13097_amd import variant_names
    prob = _eebm(_melt_field(synth.cavity_2d(n=300, ny=131, storage="f64")))
    ref = None
    for v in range(len(variant_names(9, "f64"))):
        S = _gpu_run(prob, 41, variant=v)["state"]
        if ref is None:
            ref = S
        assert np.array_equal(S, ref), v


def _two_step_variants(q, storage):
    from paper_2505_13097_amd import variant_names
    return [i for i, n in enumerate(variant_names(q, storage)) if "/t2/" in n]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", [1, 2, 3, 4, 5, 6])
def test_two_step_variants_against_oracle(case, storage):
    name, make, steps = CASES[case]
    prob = _eebm(make(storage)).with_(name=f"eebm_{name}_{storage}_t2")
    o = _oracle_run(prob, steps + 1)
    for v in _two_step_variants(prob.q, storage):
        _compare(prob, _gpu_run(prob, steps + 1, variant=v), o,
                 TOL64 if storage == "f64" else TOL32)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_full_size_cavity_sampled_windows(storage):
    """The 8192 x 8192 D2Q9 cavity lattice in the launch configuration the
    bench times, from a field crossing the melting band everywhere; after
    6 steps, 16 windows (walls, corners, interior) against the oracle."""
    from test_gpu_parity import _check_windows, _windows
    prob = _eebm(_melt_field(synth.cavity_2d(storage=storage), seed=9))
    prob = prob.with_(name=f"eebm_cavity8192_{storage}")
    Hs = 1.0 + 1.0 / prob.ste + np.abs(prob.T0).max()
    tol = (TOL64 if storage == "f64" else TOL32) * Hs
    _check_windows(prob, 6, _windows(prob.nx, prob.ny, 72, 40, 3, 8), tol)


def test_full_size_planar_properties():
    """The 2048 x 2048 D2Q5 planar workload run 10k steps: exact enthalpy
    balance through the walls, temperatures within the wall values, and a
    y-uniform front."""
    from paper_2505_13097_amd import Stefan
    prob = _eebm(synth.planar_2d())
    g = Stefan(prob)
    E0 = g.energy()
    st = g.step(prob.nsteps, stats=True)
    T = g.temperature()
    assert T.min() >= -0.5 - 1e-3 - 1e-5 and T.max() <= 1.0 + 1e-5
    dE = st["energy"] - E0
    assert abs(dE - (st["flux_in"] - st["flux_out"])) < 1e-3 * abs(dE)
    cross = g.front("crossing")
    assert cross.max() - cross.min() < 2 * prob.dx
    g.close()


def test_batch_members_equal_single_runs_and_oracle():
    from paper_2505_13097_amd import Stefan, StefanBatch
    probs = [_eebm(p) for p in synth.batch_table(
        count=6, seed=21, sizes=[64, 128, 192], storage="f64", nsteps=300)]
    probs[1] = probs[1].with_(ny=probs[1].nx // 2 + 16,
                              T0=probs[1].T0[:probs[1].nx // 2 + 16])
    probs[2] = probs[2].with_(wall_profile=(
        0.8 + 0.4 * np.sin(np.arange(probs[2].ny) / 7.0), None, None, None))
    for sched in ((-1, 0), (3, 2)):
        b = StefanBatch(probs)
        b.set_schedule(variant=sched[0], blocks_per_cu=sched[1])
        b.step(301)
        for k, p in enumerate(probs):
            g = Stefan(p)
            g.step(301)
            assert np.array_equal(b.temperature(k), g.temperature()), (sched, k)
            g.close()
        b.close()
    p = probs[0]
    o = _oracle_run(p, 301)
    b = StefanBatch(probs[:1])
    b.step(301)
    assert np.max(np.abs(b.temperature(0) - o["T"])) <= TOL64 * max(
        1.0, np.abs(o["H"]).max())
    b.close()


def test_batch_two_step_variant_equals_single_steps():
    from paper_2505_13097_amd import StefanBatch, variant_names
    probs = [_eebm(p) for p in synth.batch_table(
        count=5, seed=22, sizes=[64, 128, 192], storage="f32", nsteps=300)]
    names = variant_names(5, "f32")
    ref = StefanBatch(probs)
    ref.set_schedule(variant=3)
    ref.step(25)
    b = StefanBatch(probs)
    b.set_schedule(variant=names.index("128x2/t2/r16/nt"))
    b.step(25)
    for k in range(len(probs)):
        assert np.array_equal(b.temperature(k), ref.temperature(k)), k
    b.close()
    ref.close()


def test_reverse_mode_refused():
    """The reverse mode differentiates the IREBM step only."""
    from paper_2505_13097_amd import Stefan
    from paper_2505_13097_amd import _lib as C
    with pytest.raises(Exception, match="IREBM"):
        Stefan(_eebm(synth.planar_2d(n=64, ny=32)), flags=C.FLAG_ADJOINT)
