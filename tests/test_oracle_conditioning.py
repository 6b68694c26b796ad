"""How strongly the parity inputs amplify rounding: the oracle against a
second build of itself whose only difference is how phi is rounded
(tanh(z) evaluated as 2/(1 + exp(-2z)) - 1 instead of libm's tanh), run on
the same inputs.  The spread between the two is what two correct FP64
implementations of the scheme may differ by on an input; the GPU parity
tests take ten times it as their FP64 bar where it exceeds the 1e-12 of
the scheme's arithmetic (tests/parity_cases.py).  The measured values are
listed in the design doc (readings, conditioning).
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from parity_cases import CASES, HARD_CASES, spreads


def test_alternate_build_rounds_phi_differently():
    """The second build evaluates the same function: phi agrees to a few
    ulp everywhere and differs in the last bits somewhere."""
    xs = np.linspace(-0.1, 0.1, 2001)
    a = np.array([O.phi(x, 0.0, 0.01) for x in xs])
    with O.alternate_rounding():
        b = np.array([O.phi(x, 0.0, 0.01) for x in xs])
        assert O.phi(0.0, 0.0, 0.01) == 0.5
    assert np.max(np.abs(a - b)) < 4e-16
    assert np.any(a != b)
    # and the default build is back after the block
    assert np.array_equal(a, [O.phi(x, 0.0, 0.01) for x in xs])


def _measure(cases):
    out = {}
    for name, make, steps in cases:
        prob = make("f64")
        sp = spreads(prob, steps)
        out[name] = sp
        print(f"{name}: spread T {sp['T']:.2e} front {sp['front']:.2e} "
              f"crossing {sp['cross']:.2e} energy {sp['energy']:.2e}",
              flush=True)
    return out


@pytest.mark.slow
def test_spreads_of_the_parity_inputs():
    """The well-conditioned inputs (the workloads' own states, smooth
    fields inside the band with the walls inside it too) spread below the
    1e-12 bar; a field just below the melting temperature next to a
    suddenly heated wall spreads above it, and every hard input spreads
    below 1e-11, so that ten times its spread is still a tight bar."""
    easy = _measure(CASES)
    assert max(sp["T"] for sp in easy.values()) < 1e-12 / 4
    hard = _measure(HARD_CASES)
    assert max(sp["T"] for sp in hard.values()) > 1e-12
    assert max(sp["T"] for sp in hard.values()) < 1e-11
    for sp in list(easy.values()) + list(hard.values()):
        assert sp["front"] < 1e-11 and sp["cross"] < 1e-10


@pytest.mark.slow
@pytest.mark.parametrize("q", [7, 19])
def test_spread_of_the_freezing_octant_at_the_papers_delta(q):
    """The 3D freezing octant at delta 0.02 (Section 6.2) after 80 steps:
    the sudden freezing at the cold corner spreads the two roundings by
    1e-13 to 1e-11, against ~1e-14 at delta 0.3."""
    sp = {}
    for delta in (0.02, 0.3):
        prob = synth.freezing_cube_3d(n=25, q=q, storage="f64", delta=delta)
        f = O.init(prob, prob.T0)
        a, _ = O.run(prob, f, 80)
        with O.alternate_rounding():
            b, _ = O.run(prob, O.init(prob, prob.T0), 80)
        sp[delta] = float(np.max(np.abs(O.temperature(prob, a) -
                                        O.temperature(prob, b))))
        print(f"D3Q{q} freezing octant delta {delta}: spread T "
              f"{sp[delta]:.2e}", flush=True)
    assert 1e-13 < sp[0.02] < 1e-10
    assert sp[0.3] < sp[0.02] and sp[0.3] < 1e-12
    assert math.isfinite(sp[0.3])
