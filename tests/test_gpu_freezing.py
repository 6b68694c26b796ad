"""GPU parity of the Neumann closure (Section 4.2, eq. Neu_on_q) and the
paper's 2D freezing case (Section 6.2), both schemes, through the C ABI.

Bars as for the other parity tests: FP64 storage 1e-12 relative to the
stored zeroth moment (T for IREBM, H for EEBM), FP32 storage 1e-5
relative to it.  The mesh-refinement test has no oracle at N = 801 (the
oracle would take minutes): it checks the properties the paper reports
(the -5 C isotherm of both methods coincides, and refining the mesh moves
it less and less).
"""
import math

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


def _gpu_run(prob, nsteps, variant=-1):
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob, variant=variant)
    st = g.step(nsteps, stats=True)
    out = {"T": g.temperature(), "state": g.state().astype(np.float64),
           "energy": g.energy(), "stats": st}
    g.close()
    return out


def _oracle_run(prob, nsteps):
    f, st = O.run(prob, O.init(prob, prob.T0), nsteps)
    scale = np.abs(f.sum(axis=0)).max()      # stored zeroth moment
    return {"T": O.temperature(prob, f), "energy": O.energy(prob, f),
            "stats": st, "scale": max(1.0, scale),
            "state": O.eebm_collide(prob, f) if prob.scheme == "eebm" else f}


def _compare(prob, g, o, tol):
    dT = np.max(np.abs(g["T"] - o["T"]))
    print(f"{prob.name}: max|dT| = {dT:.3e} (scale {o['scale']:.3g})",
          flush=True)
    assert dT <= tol * o["scale"]
    if prob.scheme == "eebm":
        # planes element by element (the kernel keeps the collision of
        # the oracle's state)
        assert np.max(np.abs(g["state"] - o["state"])) <= tol * o["scale"]
    if prob.storage == "f64":
        assert abs(g["energy"] - o["energy"]) <= \
            10 * TOL64 * max(1.0, abs(o["energy"]))
    else:
        assert abs(g["energy"] - o["energy"]) <= tol * o["scale"] * prob.nodes
    assert g["stats"]["nonconverged"] == 0


def _melt(prob, seed=4):
    """A field crossing the melting band."""
    x = np.arange(prob.nx) / (prob.nx - 1)
    y = np.arange(prob.ny) / prob.ny
    T0 = 0.3 * np.sin(2 * np.pi * 2 * x)[None, :] * \
        np.cos(2 * np.pi * 1.5 * y)[:, None]
    T0 = T0 + synth.node_noise(seed, prob.nodes, 0.05).reshape(prob.ny,
                                                              prob.nx)
    return prob.with_(T0=T0)


CASES = [
    # the paper's quarter cavity, small
    ("quarter_d2q5", lambda s, sc: synth.freezing_cavity_2d(
        n=61, q=5, storage=s, scheme=sc), 300),
    ("quarter_d2q9", lambda s, sc: synth.freezing_cavity_2d(
        n=61, q=9, storage=s, scheme=sc), 300),
    # ragged, Neumann on three walls, melting field, tm != 0
    ("ragged_d2q9_three_neumann", lambda s, sc: synth.freezing_cavity_2d(
        n=131, q=9, storage=s, scheme=sc).with_(
            ny=67, T0=None, bc=("dirichlet", "neumann", "neumann", "neumann"),
            wall_T=(0.8, 0.0, 0.0, 0.0), tm=0.05), 300),
    # Neumann y walls across a periodic x axis
    ("periodic_x_d2q5", lambda s, sc: synth.freezing_cavity_2d(
        n=96, q=5, storage=s, scheme=sc).with_(
            ny=45, T0=None, bc=("periodic", "periodic", "neumann",
                                "dirichlet"), wall_T=(0.0, 0.0, 0.0, -1.0)),
     300),
    # 1D: Dirichlet hot wall, Neumann far wall
    ("d1q3_neumann", lambda s, sc: synth.stefan_1d(nx=203).with_(
        storage=s, scheme=sc, bc=("dirichlet", "neumann", "periodic",
                                  "periodic")), 2000),
    # all four walls Neumann on a 5 x 4 lattice (every node a wall node
    # or the mirror of one)
    ("all_neumann_5x4", lambda s, sc: synth.freezing_cavity_2d(
        n=5, q=9, storage=s, scheme=sc).with_(
            ny=4, T0=None, bc=("neumann",) * 4), 60),
]


def _make(case, storage, scheme):
    name, make, steps = CASES[case]
    prob = make(storage, scheme)
    if prob.T0 is None:
        prob = _melt(prob)
    return prob.with_(name=f"{name}_{scheme}_{storage}"), steps


@pytest.mark.parametrize("scheme", ["irebm", "eebm"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_neumann_lattices_against_oracle(case, storage, scheme):
    prob, steps = _make(case, storage, scheme)
    _compare(prob, _gpu_run(prob, steps), _oracle_run(prob, steps),
             TOL64 if storage == "f64" else TOL32)


@pytest.mark.parametrize("scheme", ["irebm", "eebm"])
def test_variants_bitwise_identical(scheme):
    """Every variant, the two-step ones included (a Neumann lattice runs
    them as single steps), gives the same bits."""
    from paper_2505_13097_amd import variant_names
    prob, _ = _make(2, "f64", scheme)
    ref = None
    for v in range(len(variant_names(9, "f64"))):
        T = _gpu_run(prob, 31, variant=v)["T"]
        if ref is None:
            ref = T
        assert np.array_equal(T, ref), v


@pytest.mark.parametrize("scheme", ["irebm", "eebm"])
@pytest.mark.parametrize("q", [5, 9])
def test_paper_case_full_run_n101(q, scheme):
    """The Section 6.2 case at N = 101 to t = 20 h (500 steps) against the
    oracle, FP64."""
    prob = synth.freezing_cavity_2d(n=101, q=q, scheme=scheme)
    _compare(prob, _gpu_run(prob, prob.nsteps), _oracle_run(prob, prob.nsteps),
             TOL64)


def _diag_isotherm(p, T, level):
    d = np.diag(T)
    s = np.arange(p.nx) * p.dx * math.sqrt(2.0)
    k = int(np.argmax(d > level))
    return s[k - 1] + (s[k] - s[k - 1]) * (level - d[k - 1]) / (d[k] - d[k - 1])


@pytest.mark.parametrize("q", [5, 9])
def test_paper_case_mesh_refinement(q):
    """Section 6.2 at N = 201, 401, 801, t = 20 h: the -5 C isotherm of
    EEBM and IREBM coincides within a cell at each N, and refining the
    mesh moves it less each time (delta fixed at 0.02)."""
    from paper_2505_13097_amd import Stefan
    pos = {}
    for n in (201, 401, 801):
        for scheme in ("irebm", "eebm"):
            p = synth.freezing_cavity_2d(n=n, q=q, scheme=scheme)
            g = Stefan(p)
            st = g.step(p.nsteps, stats=True)
            T = g.temperature()
            g.close()
            assert st["nonconverged"] == 0
            assert T.min() >= -2.0 - 1e-12 and T.max() <= 1.0 + 1e-9
            pos[n, scheme] = _diag_isotherm(p, T, -0.5)
        print(f"D2Q{q} N={n} ({p.nsteps} steps): isotherm -5 C on the "
              f"diagonal IREBM {pos[n, 'irebm']:.5f} EEBM "
              f"{pos[n, 'eebm']:.5f}", flush=True)
        assert abs(pos[n, "irebm"] - pos[n, "eebm"]) < p.dx
    d1 = abs(pos[401, "irebm"] - pos[201, "irebm"])
    d2 = abs(pos[801, "irebm"] - pos[401, "irebm"])
    assert d2 < d1


def test_batch_refuses_neumann_instances():
    from paper_2505_13097_amd import StefanBatch
    probs = [synth.freezing_cavity_2d(n=64, q=5)] * 2
    with pytest.raises(Exception, match="Neumann"):
        StefanBatch(probs)
