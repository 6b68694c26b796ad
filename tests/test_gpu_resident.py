"""The resident D1Q3 kernel (many steps per launch in one workgroup, both
states in LDS) against the one-step kernel, bit for bit: the same per-node
code on the same operands, so every state, every Newton counter and the
largest residual are equal; the boundary-flux sums, added up in another
order, agree to rounding.  Lattices the resident kernel does not take run
the variant as the one-step default."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RES = "resident2048"


def _res_index():
    from paper_2505_13097_amd import variant_names
    return variant_names(3, "f64").index(RES)


def _run(prob, chunks, variant):
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob, variant=variant)
    for n in chunks:
        g.step(n)
    st = g.stats()
    out = {"T": g.temperature(), "state": g.state(), "stats": st}
    g.close()
    return out


def _same(a, b, label):
    assert np.array_equal(a["state"], b["state"]), label
    assert np.array_equal(a["T"], b["T"]), label
    for k in ("steps", "max_newton_it", "nonconverged", "max_residual",
              "energy"):
        assert a["stats"][k] == b["stats"][k], (label, k, a["stats"][k],
                                                b["stats"][k])
    for k in ("flux_in", "flux_out"):
        x, y = a["stats"][k], b["stats"][k]
        assert abs(x - y) <= 1e-12 * max(1.0, abs(x), abs(y)), (label, k, x, y)


def _wave(n):
    x = np.arange(n) / n
    return (0.3 * np.sin(2 * np.pi * x) - 0.05).reshape(1, n)


CASES = {
    "hot_wall_f64": lambda: synth.stefan_1d(nx=256),
    "hot_wall_f32": lambda: synth.stefan_1d(nx=256).with_(storage="f32"),
    "hot_wall_plain": lambda: synth.stefan_1d(nx=256).with_(
        newton_mode="plain"),
    "hot_wall_eebm": lambda: synth.stefan_1d(nx=256).with_(scheme="eebm"),
    "bounceback_x+": lambda: synth.stefan_1d(nx=301).with_(
        bc=("dirichlet", "bounceback", "periodic", "periodic")),
    "periodic": lambda: synth.stefan_1d(nx=200).with_(
        bc=("periodic", "periodic", "periodic", "periodic"), T0=_wave(200),
        dx=1.0 / 200),
    "largest_2048": lambda: synth.stefan_1d(nx=2048).with_(delta=0.002),
    "ragged_1025": lambda: synth.stefan_1d(nx=1025).with_(storage="f32"),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("chunks", [(1,), (2,), (37,), (1000, 4200)])
def test_resident_equals_one_step_kernel(case, chunks):
    prob = CASES[case]()
    print(f"resident {case} chunks {chunks}", flush=True)
    a = _run(prob, chunks, 0)
    b = _run(prob, chunks, _res_index())
    _same(a, b, (case, chunks))


def test_resident_is_the_default_for_small_1d_lattices():
    prob = synth.stefan_1d(nx=256)
    a = _run(prob, (500,), -1)
    b = _run(prob, (500,), _res_index())
    _same(a, b, "default")


def test_resident_variant_falls_back_beyond_2048_nodes():
    prob = synth.stefan_1d(nx=2049).with_(delta=0.002)
    a = _run(prob, (300,), 0)
    b = _run(prob, (300,), _res_index())
    _same(a, b, "2049 nodes")


def test_autotune_on_1d_keeps_the_state():
    from paper_2505_13097_amd import Stefan
    prob = synth.stefan_1d(nx=256)
    ref = _run(prob, (30,), 0)
    g = Stefan(prob)
    g.step(10)
    v, ms = g.autotune(steps=20)
    assert ms > 0
    g.step(20)
    T = g.temperature()
    g.close()
    assert np.array_equal(T, ref["T"]), v


def test_batch_rejects_the_resident_variant():
    from paper_2505_13097_amd import StefanBatch
    b = StefanBatch([synth.stefan_1d(nx=64), synth.stefan_1d(nx=96)])
    with pytest.raises(Exception, match="single lattices"):
        b.set_schedule(_res_index(), 0, 0)
    b.step(4)
    b.close()
