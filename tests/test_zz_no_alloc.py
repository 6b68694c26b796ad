"""lbm_stefan_step_noalloc (no workspace, nothing allocated; its scratch is
a fixed device array) against lbm_stefan_step on a handle made from the
same params: the same state bit for bit and the same statistics, on calls
in a row whose lattices shrink, so each call must clear what the last one
left in the shared scratch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _mushy(prob, seed=3):
    """a field in the melting band with seeded noise: multi-iteration
    Newton solves at most nodes"""
    if prob.dim == 3:
        shape = (prob.nz, prob.ny, prob.nx)
    else:
        shape = (prob.ny, prob.nx)
    x = np.arange(prob.nx) / (prob.nx - 1)
    T0 = 2.0 * prob.delta * np.sin(6 * np.pi * x) + 0.3 * prob.delta
    T0 = np.broadcast_to(T0, shape) + synth.node_noise(
        seed, int(np.prod(shape)), 0.5 * prob.delta).reshape(shape)
    return prob.with_(T0=T0)


CASES = [
    # largest first: each later call has fewer statistics slots (1170,
    # 102, 80, 36, 2) and fewer nodes than the one before
    ("d2q9_cavity_f64", lambda: _mushy(synth.cavity_2d(
        n=1031, ny=517, storage="f64"))),
    ("d2q5_planar_f32", lambda: _mushy(synth.planar_2d(
        n=300, ny=133, storage="f32"))),
    ("d3q19_cube_f32", lambda: _mushy(synth.cavity_3d(
        n=70, ny=37, nz=29, q=19, storage="f32")).with_(ste=0.3)),
    ("d2q9_periodic_eebm_f64", lambda: _mushy(synth.cavity_2d(
        n=131, ny=70, storage="f64")).with_(
            bc=("periodic",) * 4, scheme="eebm")),
    ("d1q3_f64", lambda: _mushy(synth.stefan_1d(nx=333))),
]

KEYS = ("max_newton_it", "nonconverged", "max_residual", "energy",
        "flux_in", "flux_out")


def _one(prob, label):
    import torch
    from paper_2505_13097_amd import Stefan, step_noalloc
    print(f"no-alloc {label}: {prob.name} q{prob.q} "
          f"{prob.nx}x{prob.ny}x{prob.nz if prob.dim == 3 else 1}",
          flush=True)
    # the handle in the one-step kernel the call runs (a small D1Q3
    # lattice would default to the resident kernel)
    g = Stefan(prob, variant=0 if prob.dim == 1 else -1)
    nbytes = prob.q * prob.nodes * (8 if prob.storage == "f64" else 4)
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    src.copy_(torch.as_tensor(g.state().reshape(-1).view(np.uint8)))
    st = step_noalloc(prob, src, dst, stats=True)
    ref = g.step(1, stats=True)
    want = g.state()
    g.close()
    got = dst.cpu().numpy().view(want.dtype).reshape(want.shape)
    assert np.array_equal(got, want), label
    for k in KEYS:
        assert st[k] == ref[k], (label, k, st[k], ref[k])
    assert st["steps"] == 1
    assert st["max_newton_it"] >= 2 or prob.scheme == "eebm"
    return st


def test_noalloc_matches_handle_step_on_shrinking_lattices():
    for label, make in CASES:
        _one(make(), label)
    # the first lattice again after the small ones, then a repeat call
    _one(CASES[0][1](), "d2q9_cavity_f64 again")
    _one(CASES[1][1](), "d2q5_planar_f32 again")


def test_noalloc_without_stats_and_refusals():
    import torch
    from paper_2505_13097_amd import Stefan, LbmError, _lib, step_noalloc
    prob = _mushy(synth.planar_2d(n=200, ny=90, storage="f32"))
    g = Stefan(prob)
    nbytes = prob.q * prob.nodes * 4
    src = torch.as_tensor(g.state().reshape(-1).view(np.uint8)).cuda()
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    assert step_noalloc(prob, src, dst) is None
    torch.cuda.synchronize()
    g.step(1)
    want = g.state()
    got = dst.cpu().numpy().view(np.float32).reshape(want.shape)
    assert np.array_equal(got, want)
    g.close()
    # refused before any device work: a wall profile, the same buffer
    with pytest.raises(LbmError) as e:
        step_noalloc(prob.with_(wall_profile=(np.ones(prob.ny), None, None,
                                              None)), src, dst)
    assert e.value.code == _lib.EINVAL
    with pytest.raises(LbmError) as e:
        step_noalloc(prob, src, src)
    assert e.value.code == _lib.EINVAL
