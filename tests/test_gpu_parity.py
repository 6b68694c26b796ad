"""GPU parity: the gfx950 IREBM step, called through the C ABI, against
the CPU FP64 oracle on the same seeded inputs.

Bars: FP64 storage, ||T_gpu - T_orc||_inf <= max(1e-12 max(||T_orc||_inf,
1), K s_T) and fronts within max(1e-12 max(x_f, dx), K s_front), with s the
measured spread between the oracle and its other rounding of phi on the
same input and K = 10 (parity_cases: the spread is below the 1e-12 terms on
well-conditioned inputs and sets the bar on the hard ones); the
zero-crossing front, on rows where it is a continuous function of T, also
within its first-order sensitivity dx bar_T / (T_x - T_x+1) to the
temperatures of its cell.  FP32 storage (per-node math in FP64),
||dT||_inf <= 1e-5 and the zero-crossing front within one cell; the
energy is an FP64 sum in both precisions.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity_cases import (CASES, HARD_CASES, K_SPREAD, oracle_result,
                          shift_tm, smooth_mushy, spreads)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _gpu_run(prob, nsteps, variant=-1):
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob, variant=variant)
    st = g.step(nsteps, stats=True)
    out = {
        "T": g.temperature(),
        "front": g.front("integral"),
        "cross": g.front("crossing"),
        "energy": g.energy(),
        "stats": st,
    }
    g.close()
    return out


def _oracle_run(prob, nsteps):
    return oracle_result(prob, nsteps)


def _compare(prob, g, o, tol, sp=None):
    """GPU result g against the oracle's o; sp: spreads() of the input
    (FP64 storage: computed here when not given)."""
    scale = max(1.0, np.max(np.abs(o["T"])))
    err = np.max(np.abs(g["T"] - o["T"]))
    assert g["stats"]["nonconverged"] == 0 and o["stats"]["nonconverged"] == 0
    if prob.storage != "f64":
        print(f"{prob.name}: max|dT| = {err:.3e} (bar {tol:.0e})", flush=True)
        assert err <= tol * scale
        cr = np.abs(g["cross"] - o["cross"])
        assert np.all(cr <= prob.dx), cr.max()
        assert abs(g["energy"] - o["energy"]) <= 1e-5 * prob.nodes
        return
    if sp is None:
        sp = spreads(prob, o["nsteps"], ref=o)
    bar_T = max(tol * scale, K_SPREAD * sp["T"])
    # fronts (reading A13 of the scope: 1e-12 max(x_f, dx)), unless the
    # spread of this input says otherwise
    a13 = lambda xf: 1e-12 * np.maximum(np.abs(xf), prob.dx)
    fr = np.abs(g["front"] - o["front"])
    bar_f = np.maximum(a13(o["front"]), K_SPREAD * sp["front"])
    cr = np.abs(g["cross"] - o["cross"])
    ok, dcell = _crossing_well_posed(prob, o["T"], o["cross"],
                                     max(err, sp["T"]))
    bar_c = np.maximum(np.maximum(a13(o["cross"]), K_SPREAD * sp["cross"]),
                       2.0 * prob.dx * bar_T / np.maximum(dcell, 1e-300))
    print(f"{prob.name}: max|dT| = {err:.3e} (bar {bar_T:.2e}, spread "
          f"{sp['T']:.2e}); front {fr.max():.2e} (worst err/bar "
          f"{np.max(fr / bar_f):.3f}); crossing {cr[ok].max() if ok.any() else 0:.2e}"
          f" on {ok.sum()}/{ok.size} rows", flush=True)
    assert err <= bar_T
    assert np.all(fr <= bar_f)
    assert ok.sum() >= 0.9 * ok.size
    assert np.all(cr[ok] <= bar_c[ok])
    assert abs(g["energy"] - o["energy"]) <= max(
        1e-11 * max(1.0, abs(o["energy"])), K_SPREAD * sp["energy"])
    for k in ("flux_in", "flux_out"):
        a, b = g["stats"][k], o["stats"][k]
        assert abs(a - b) <= 1e-11 * max(1.0, abs(b)), (k, a, b)
    assert g["stats"]["max_residual"] < 1e-10


def _crossing_well_posed(prob, T, cross, err):
    """Rows whose zero-crossing front is a continuous function of T at
    the given error: the first crossing from x = 0 jumps to another cell
    when T - T_m at a node before it (or at the crossing cell's ends) is
    within a few times the error of zero.  Also returns each row's
    T_x - T_x+1 across its crossing cell (inf where the row has none)."""
    ok = np.ones(prob.ny, dtype=bool)
    dcell = np.full(prob.ny, np.inf)
    margin = 8.0 * max(err, 1e-16)
    for y in range(prob.ny):
        k = int(min(prob.nx - 1, np.floor(cross[y] / prob.dx) + 1))
        if np.any(np.abs(T[y, :k + 1] - prob.tm) <= margin):
            ok[y] = False
        if 1 <= k <= prob.nx - 1 and cross[y] > 0.0:
            dcell[y] = T[y, k - 1] - T[y, k]
    return ok, dcell


_smooth_mushy = smooth_mushy
_shift_tm = shift_tm


def test_stefan_1d_full_run_fp64():
    """The 1D workload at full length: D1Q3, N = 256, 20k steps, FP64."""
    prob = synth.stefan_1d()
    g = _gpu_run(prob, prob.nsteps)
    o = _oracle_run(prob, prob.nsteps)
    _compare(prob, g, o, TOL64)
    # energy balance through the boundaries, in both implementations
    dE = g["energy"] - o["E0"]
    assert abs(dE - (g["stats"]["flux_in"] - g["stats"]["flux_out"])) < 1e-9


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_small_lattices_against_oracle(case, storage):
    name, make, steps = CASES[case]
    prob = make(storage).with_(name=f"{name}_{storage}")
    g = _gpu_run(prob, steps)
    o = _oracle_run(prob, steps)
    _compare(prob, g, o, TOL64 if storage == "f64" else TOL32)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(HARD_CASES)))
def test_hard_lattices_against_oracle(case, storage):
    """Fields just below the melting temperature next to a suddenly heated
    wall (a hot wall profile from 0.5 to 1.5 in the mixed case): the FP64
    bar is the larger of 1e-12 and ten times the two-rounding spread of the
    oracle on the same input."""
    name, make, steps = HARD_CASES[case]
    prob = make(storage).with_(name=f"{name}_{storage}")
    g = _gpu_run(prob, steps)
    o = _oracle_run(prob, steps)
    _compare(prob, g, o, TOL64 if storage == "f64" else TOL32)


def test_variants_bitwise_identical():
    """The per-node arithmetic does not depend on the tile shape."""
    from paper_2505_13097_amd import variant_names
    prob = _smooth_mushy(synth.cavity_2d(n=300, ny=131, storage="f64"))
    ref = None
    for v in range(len(variant_names(9, "f64"))):
        T = _gpu_run(prob, 40, variant=v)["T"]
        if ref is None:
            ref = T
        assert np.array_equal(T, ref), v


def _two_step_variants(q, storage):
    from paper_2505_13097_amd import variant_names
    return [i for i, n in enumerate(variant_names(q, storage)) if "/t2/" in n]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", [0, 1, 3, 4, 5, 6, 7])
def test_two_step_variants_against_oracle(case, storage):
    """Two steps per launch (rings of rows in LDS): the same bars against
    the oracle, on ragged, periodic, all-bounce-back, mixed-wall and 3x3
    lattices, with an odd step count (the last step single)."""
    name, make, steps = CASES[case]
    prob = make(storage).with_(name=f"{name}_{storage}_t2")
    o = _oracle_run(prob, steps + 1)
    sp = spreads(prob, steps + 1, ref=o) if storage == "f64" else None
    for v in _two_step_variants(prob.q, storage):
        g = _gpu_run(prob, steps + 1, variant=v)
        _compare(prob, g, o, TOL64 if storage == "f64" else TOL32, sp)


def test_two_step_variants_bitwise_equal_single_steps():
    """Each node update of the two-step kernel is the single-step code on
    the same operands: equal states after an odd number of steps."""
    prob = _smooth_mushy(synth.planar_2d(n=600, ny=333, storage="f32")).with_(
        bc=("dirichlet", "bounceback", "periodic", "periodic"))
    ref = _gpu_run(prob, 25, variant=3)["T"]
    for v in _two_step_variants(5, "f32"):
        assert np.array_equal(_gpu_run(prob, 25, variant=v)["T"], ref), v


def test_zero_steps_and_state_roundtrip():
    from paper_2505_13097_amd import Stefan
    prob = synth.planar_2d(n=64, ny=32, storage="f64")
    g = Stefan(prob)
    T0 = g.temperature()
    expect = prob.T0.copy()
    expect[:, 0] = 1.0
    expect[:, -1] = -0.5
    assert np.max(np.abs(T0 - expect)) < 1e-15
    s = g.state()
    g.step(5)
    g.set_state(s)
    assert np.array_equal(g.temperature(), T0)
    st = g.step(0, stats=True)
    assert st["steps"] == 5
    g.close()


def _window_problem(prob, x0, y0, w, h):
    """Window [x0, x0+w) x [y0, y0+h) of prob as a lattice of its own.
    Sides on the real boundary keep its closure; artificial sides get
    bounce-back (which leaves the initial state alone)."""
    bc = (prob.bc[0] if x0 == 0 else "bounceback",
          prob.bc[1] if x0 + w == prob.nx else "bounceback",
          prob.bc[2] if y0 == 0 else "bounceback",
          prob.bc[3] if y0 + h == prob.ny else "bounceback")
    assert "periodic" not in bc
    prof = tuple(None if a is None else
                 (a[y0:y0 + h] if k < 2 else a[x0:x0 + w])
                 for k, a in enumerate(prob.wall_profile))
    T0 = np.broadcast_to(0.0 if prob.T0 is None else prob.T0,
                         (prob.ny, prob.nx))[y0:y0 + h, x0:x0 + w]
    return prob.with_(nx=w, ny=h, bc=bc, wall_profile=prof, T0=T0,
                      dx=prob.dx), bc


def _check_windows(prob, steps, windows, tol, variant=-1):
    """variant: a kernel variant id, -1 for the library default, or
    "autotune" for the one the autotuner picks on this lattice (as the
    bench does)."""
    from paper_2505_13097_amd import Stefan, variant_names
    g = Stefan(prob, variant=-1 if variant == "autotune" else variant)
    if variant == "autotune":
        variant, _ = g.autotune(steps=4)
    vname = variant_names(prob.q, prob.storage)[variant] if variant >= 0 \
        else "default"
    print(f"{prob.name}: kernel variant {variant} ({vname})", flush=True)
    st = g.step(steps, stats=True)
    T = g.temperature()
    g.close()
    assert st["nonconverged"] == 0
    worst = 0.0
    for (x0, y0, w, h) in windows:
        sub, bc = _window_problem(prob, x0, y0, w, h)
        f = O.init(sub, sub.T0)
        f, _ = O.run(sub, f, steps)
        To = O.temperature(sub, f)
        # nodes within `steps` cells of an artificial side are not exact
        xa = 0 if x0 == 0 else steps
        xb = w if x0 + w == prob.nx else w - steps
        ya = 0 if y0 == 0 else steps
        yb = h if y0 + h == prob.ny else h - steps
        d = np.abs(T[y0 + ya:y0 + yb, x0 + xa:x0 + xb] - To[ya:yb, xa:xb])
        worst = max(worst, d.max())
    print(f"{prob.name} [{vname}]: {len(windows)} windows, "
          f"max|dT| = {worst:.3e}", flush=True)
    assert worst <= tol * max(1.0, np.abs(T).max())


def _windows(nx, ny, w, h, seed, count, avoid_y_edges=False):
    """Corners, wall midpoints and seeded interior windows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ylo = h if avoid_y_edges else 0
    yhi = ny - 2 * h if avoid_y_edges else ny - h
    out = [(0, ylo, w, h), (nx - w, yhi, w, h),
           (0, (ylo + yhi) // 2, w, h), (nx - w, (ylo + yhi) // 2, w, h)]
    if not avoid_y_edges:
        out += [(0, 0, w, h), (nx - w, ny - h, w, h), (nx // 2, 0, w, h),
                (nx // 3, ny - h, w, h)]
    for _ in range(count):
        out.append((int(rng.integers(0, nx - w)), int(rng.integers(ylo, yhi)),
                    w, h))
    return out


def _full_size_variants(q):
    """the default one-step variant, every two-step variant, the variant
    the bench times on this lattice (unless asked to autotune: the cavity's
    128x4/t2/r32/nt, the planar step's 128x2/npt2) and the autotuner's
    pick"""
    import bench
    from paper_2505_13097_amd import variant_names
    names = variant_names(q, "f32")
    out = [-1] + [i for i, n in enumerate(names) if "/t2/" in n]
    timed = names.index(bench.DEFAULT_VARIANTS["cavity" if q == 9
                                               else "planar"])
    if timed not in out:
        out.append(timed)
    return out + ["autotune"]


@pytest.mark.parametrize("variant", _full_size_variants(9))
@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", TOL32)])
def test_full_size_cavity_sampled_windows(storage, tol, variant):
    """The 8192 x 8192 D2Q9 cavity lattice, from a smooth field in the
    mushy band plus seeded noise (nearly every node runs a multi-iteration
    Newton solve), in each launch configuration the bench can time (the
    two-step kernels and the autotuner's pick) and the default one; after
    6 steps, 16 windows (walls, corners, interior) against the oracle."""
    prob = _smooth_mushy(synth.cavity_2d(storage=storage))
    T0 = prob.T0 + synth.node_noise(7, prob.nodes, 0.2 * prob.delta).reshape(
        prob.ny, prob.nx)
    prob = prob.with_(T0=T0, name=f"cavity8192_{storage}")
    _check_windows(prob, 6, _windows(prob.nx, prob.ny, 72, 40, 3, 8), tol,
                   variant)


@pytest.mark.parametrize("variant", _full_size_variants(5))
@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", TOL32)])
def test_full_size_planar_sampled_windows(storage, tol, variant):
    """The 2048 x 2048 D2Q5 planar lattice (periodic y) in the mushy band
    with its seeded noise scaled to a fraction of delta; 12 windows after
    10 steps, in the default, every two-step and the autotuned variant."""
    base = synth.planar_2d(storage=storage)
    prob = _smooth_mushy(base)
    prob = prob.with_(T0=prob.T0 + (base.T0 + 0.5) * (0.2 * prob.delta / 1e-3),
                      name=f"planar2048_{storage}")
    _check_windows(prob, 10, _windows(prob.nx, prob.ny, 80, 48, 4, 8,
                                      avoid_y_edges=True), tol, variant)


@pytest.mark.parametrize("storage,tol", [("f32", TOL32), ("f64", TOL64)])
def test_cavity_as_benched_hundred_step_windows(storage, tol):
    """The roofline-graded cavity exactly as the bench runs it (8192 x 8192
    D2Q9, its initial state and walls, the bench's two-step variant) for a
    100-step window, then 8 windows rerun by the oracle: the hot wall where
    the front forms (both corners and two stretches of the wall), the cold
    corner and wall, the top wall and the interior.  Each window keeps the
    nodes more than 100 cells from its artificial sides."""
    import bench
    from paper_2505_13097_amd import variant_names
    prob = synth.cavity_2d(storage=storage).with_(
        name=f"cavity8192_as_benched_{storage}")
    v = variant_names(9, storage).index(bench.DEFAULT_VARIANTS["cavity"])
    n, e, s_ = prob.nx, 164, 232
    wins = [(0, 0, e, e), (0, n - e, e, e), (0, n // 2 - s_ // 2, e, s_),
            (0, n // 3, e, s_), (n - e, 0, e, e), (n - e, n // 2, e, s_),
            (n // 2, n - e, s_, e), (n // 2 - s_ // 2, n // 2 - s_ // 2, s_, s_)]
    _check_windows(prob, 100, wins, tol, v)


def test_full_size_planar_properties():
    """The 2048 x 2048 D2Q5 planar workload at full length (10k steps):
    energy balance through the walls, bounded temperatures, Newton within
    its cap, and a y-uniform front (the initial noise has diffused)."""
    prob = synth.planar_2d()
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob)
    E0 = g.energy()
    st = g.step(prob.nsteps, stats=True)
    T = g.temperature()
    assert st["nonconverged"] == 0
    assert T.min() >= -0.5 - 1e-3 - 1e-6 and T.max() <= 1.0 + 1e-6
    dE = st["energy"] - E0
    assert abs(dE - (st["flux_in"] - st["flux_out"])) < 1e-3 * abs(dE)
    cross = g.front("crossing")
    assert cross.max() - cross.min() < 2 * prob.dx
    g.close()


@pytest.mark.parametrize("max_it", [1, 2, 3])
def test_newton_iteration_cap_against_oracle(max_it):
    """A tight iteration cap: the same nodes stop unconverged on both sides
    (the counts may differ only where rounding moves an iterate across
    the tolerance), the largest iteration count agrees, and converged
    nodes still match the oracle."""
    for make in (lambda: synth.cavity_2d(n=150, ny=77, storage="f64"),
                 lambda: _smooth_mushy(synth.planar_2d(n=131, ny=67,
                                                       storage="f64"))):
        prob = make().with_(max_it=max_it)
        g = _gpu_run(prob, 60)
        o = _oracle_run(prob, 60)
        gs, os_ = g["stats"], o["stats"]
        print(f"{prob.name} cap {max_it}: nonconverged {gs['nonconverged']}"
              f" vs {os_['nonconverged']}, max it {gs['max_newton_it']}"
              f" vs {os_['max_it']}", flush=True)
        assert gs["max_newton_it"] == os_["max_it"]
        assert abs(gs["nonconverged"] - os_["nonconverged"]) <= \
            1e-3 * prob.nodes * 60
        if os_["nonconverged"] == 0:
            assert gs["nonconverged"] == 0
            err = np.max(np.abs(g["T"] - o["T"]))
            assert err <= TOL64 * max(1.0, np.max(np.abs(o["T"])))
