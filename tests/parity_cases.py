"""Inputs of the 2D parity tests and the conditioning measurement behind
their FP64 bars (shared by tests/test_gpu_parity.py and
tests/test_oracle_conditioning.py).

Conditioning.  Two correct FP64 evaluations of the scheme drift apart on
some inputs: a field inside the melting band next to a suddenly heated
Dirichlet wall amplifies rounding differences over the steps.  spreads()
runs the oracle twice, once as built and once with phi rounded the other
way (tanh(z) as 2/(1 + exp(-2z)) - 1, oracle.alternate_rounding), and
returns how far the two results lie apart.  The GPU computes phi as
1/(1 + exp(-2u)), a third rounding of the same function, so an FP64 bar of
K_SPREAD times the measured spread (never below the 1e-12 bar of the
scheme's arithmetic) admits the GPU's own rounding drift and nothing
larger.
"""
import numpy as np

import oracle as O
import synth

K_SPREAD = 10.0


def smooth_mushy(prob, amp_cells=2.0, walls_cells=2.0):
    """Stress input: a smooth field inside the mushy band (|T| ~ delta) so
    that nearly every node runs a multi-iteration Newton solve, with any
    Dirichlet wall set inside the band too (a well-conditioned input)."""
    x = np.arange(prob.nx) / (prob.nx - 1)
    y = np.arange(prob.ny) / prob.ny
    d = prob.delta
    T0 = (amp_cells * d * np.sin(2 * np.pi * 3 * x)[None, :] *
          np.cos(2 * np.pi * 2 * y)[:, None] + 0.3 * d)
    wall = (walls_cells * d, -walls_cells * d, 0.5 * d, -0.5 * d)
    return prob.with_(T0=T0, wall_T=wall)


def near_melting(prob, shift=0.45):
    """Hard input: the workload's initial field lifted to just below the
    melting temperature (-0.05 for the -0.5 solid), next to walls at
    their workload temperatures (a hot wall at 1): the band opens at a
    suddenly heated wall."""
    T0 = prob.T0 if prob.T0 is not None else np.full((prob.ny, prob.nx),
                                                      -0.5)
    return prob.with_(T0=np.broadcast_to(T0, (prob.ny, prob.nx)) + shift)


def noisy(prob, amplitude, seed=17):
    """prob with seeded node noise of the given amplitude added to T0"""
    T0 = np.broadcast_to(prob.T0, (prob.ny, prob.nx)) + synth.node_noise(
        seed, prob.nx * prob.ny, amplitude).reshape(prob.ny, prob.nx)
    return prob.with_(T0=T0)


def shift_tm(prob, tm):
    """The same problem with melting temperature tm: T0 and the wall
    temperatures move with it."""
    return prob.with_(tm=tm, T0=np.asarray(prob.T0) + tm,
                      wall_T=tuple(w + tm for w in prob.wall_T))


CASES = [
    # (name, problem builder, steps): the workloads' own initial states on
    # ragged lattices, and smooth mushy-band stress fields
    ("d2q5_planar_ragged", lambda s: synth.planar_2d(
        n=131, ny=67, storage=s), 600),
    ("d2q9_cavity_ragged", lambda s: synth.cavity_2d(
        n=150, ny=77, storage=s), 600),
    ("d2q5_planar_mushy", lambda s: smooth_mushy(synth.planar_2d(
        n=131, ny=67, storage=s)), 200),
    ("d2q9_cavity_mushy", lambda s: smooth_mushy(synth.cavity_2d(
        n=150, ny=77, storage=s)), 200),
    ("d2q9_all_bounceback", lambda s: smooth_mushy(synth.cavity_2d(
        n=97, ny=70, storage=s)).with_(bc=("bounceback",) * 4), 200),
    ("d2q5_all_periodic", lambda s: smooth_mushy(synth.planar_2d(
        n=70, ny=45, storage=s)).with_(bc=("periodic",) * 4), 200),
    ("d2q9_mixed_profile", lambda s: smooth_mushy(synth.cavity_2d(
        n=90, ny=66, storage=s)).with_(
            bc=("dirichlet", "bounceback", "dirichlet", "bounceback"),
            wall_profile=(0.02 * np.sin(np.linspace(0, 3, 66)), None,
                          0.01 * np.cos(np.linspace(0, 5, 90)), None)), 200),
    # bounce-back walls beside a periodic axis: diagonals entering at the
    # first and last rows cross the seam and still bounce back
    ("d2q9_bounceback_x_periodic_y", lambda s: smooth_mushy(synth.cavity_2d(
        n=81, ny=46, storage=s)).with_(
            bc=("bounceback", "bounceback", "periodic", "periodic")), 200),
    ("d2q9_periodic_x_bounceback_y", lambda s: smooth_mushy(synth.cavity_2d(
        n=77, ny=52, storage=s)).with_(
            bc=("periodic", "periodic", "bounceback", "bounceback")), 200),
    ("d2q5_tiny_3x3", lambda s: synth.planar_2d(n=3, ny=3, storage=s), 40),
    # degenerate parameters: no latent heat (1/Ste = 1e-12: one or two
    # Newton iterations, BGK diffusion), a sharp band (delta half a cell),
    # tau next to 1/2 (a = 1 - 1/tau near -1), melting at T_m = 0.25
    ("d2q5_no_latent_heat", lambda s: smooth_mushy(synth.planar_2d(
        n=96, ny=40, storage=s)).with_(ste=1e12), 200),
    ("d2q9_sharp_delta", lambda s: smooth_mushy(synth.cavity_2d(
        n=101, ny=58, storage=s).with_(delta=0.5 / 100)), 200),
    ("d2q5_tau_near_half", lambda s: smooth_mushy(synth.planar_2d(
        n=96, ny=40, storage=s)).with_(tau=0.5005), 200),
    ("d2q9_melting_at_0.25", lambda s: shift_tm(smooth_mushy(
        synth.cavity_2d(n=88, ny=61, storage=s)), 0.25), 200),
    ("d1q3_plain_newton", lambda s: synth.stefan_1d(nx=333).with_(
        newton_mode="plain", storage=s), 500),
]

HARD_CASES = [
    # fields just below the melting temperature next to a suddenly heated
    # wall, on the workloads' lattices and wall mixes; the mixed case has
    # a hot wall profile from 0.5 to 1.5 and a y wall profile across T_m
    ("d2q5_planar_near_melting", lambda s: near_melting(synth.planar_2d(
        n=131, ny=67, storage=s)), 150),
    ("d2q9_cavity_near_melting", lambda s: near_melting(synth.cavity_2d(
        n=150, ny=77, storage=s), 0.4), 150),
    # closed boxes: a noisy field reaching into the band from below
    ("d2q9_all_bounceback_near_melting", lambda s: noisy(near_melting(
        synth.cavity_2d(n=97, ny=70, storage=s)), 0.05).with_(
            bc=("bounceback",) * 4), 120),
    ("d2q5_all_periodic_near_melting", lambda s: noisy(near_melting(
        synth.planar_2d(n=70, ny=45, storage=s)), 0.05).with_(
            bc=("periodic",) * 4), 120),
    ("d2q9_mixed_profile_hot", lambda s: near_melting(synth.cavity_2d(
        n=90, ny=66, storage=s)).with_(
            bc=("dirichlet", "bounceback", "dirichlet", "bounceback"),
            wall_T=(1.0, 0.0, 0.2, 0.0),
            wall_profile=(np.linspace(0.5, 1.5, 66), None,
                          np.linspace(-0.3, 0.3, 90), None)), 120),
]


def oracle_result(prob, nsteps):
    """T, both fronts, energy and statistics of the oracle after nsteps
    from prob.T0."""
    f = O.init(prob, prob.T0)
    E0 = O.energy(prob, f)
    f, st = O.run(prob, f, nsteps)
    return {
        "T": O.temperature(prob, f),
        "front": O.front(prob, f, O.FRONT_INTEGRAL),
        "cross": O.front(prob, f, O.FRONT_CROSSING),
        "energy": O.energy(prob, f),
        "E0": E0,
        "stats": st,
        "nsteps": nsteps,
    }


def spreads(prob, nsteps, ref=None):
    """How far the oracle and its other rounding of phi lie apart after
    nsteps: the largest |dT|, |d front| (integral), |d crossing| over the
    lattice and |d energy|."""
    a = oracle_result(prob, nsteps) if ref is None else ref
    with O.alternate_rounding():
        b = oracle_result(prob, nsteps)
    return {"T": float(np.max(np.abs(a["T"] - b["T"]))),
            "front": float(np.max(np.abs(a["front"] - b["front"]))),
            "cross": float(np.max(np.abs(a["cross"] - b["cross"]))),
            "energy": abs(a["energy"] - b["energy"])}
