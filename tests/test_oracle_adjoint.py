"""Pins of the oracle's reverse mode.

The reverse step differentiates the Newton root by the implicit-function
theorem.  It is pinned against (i) the complex-step tangent of the same
forward step (dot-product test <J v, w> = <v, J^T w>, exact to rounding
for the state and for the Ste, delta and wall-profile directions),
(ii) the complex-step derivative of the whole front-misfit loss and
(iii) central finite differences of the forward loss in FP64.
"""
import numpy as np
import pytest

import oracle as O
import synth

H = 1e-30   # complex-step size


def _state_with_front(prob, nsteps):
    f = O.init(prob, prob.T0)
    f, st = O.run(prob, f, nsteps)
    assert st["nonconverged"] == 0
    return f


def _cases():
    n, m = 24, 10
    prof = 1.0 + 0.1 * np.sin(2 * np.pi * np.arange(m) / m)
    d2q5 = synth.Problem(dim=2, q=5, nx=n, ny=m, tau=0.8, ste=0.2,
                         delta=1.5 / (n - 1),
                         bc=("dirichlet", "dirichlet", "periodic", "periodic"),
                         wall_T=(1.0, -0.5, 0.0, 0.0),
                         wall_profile=(prof, None, None, None),
                         T0=np.full((m, n), -0.5), max_it=40)
    d2q9 = synth.Problem(dim=2, q=9, nx=n, ny=m, tau=0.65, ste=0.1,
                         delta=1.5 / (n - 1),
                         bc=("dirichlet", "dirichlet", "bounceback",
                             "bounceback"),
                         wall_T=(1.0, -0.5, 0.0, 0.0),
                         wall_profile=(prof, None, None, None),
                         T0=np.full((m, n), -0.5), max_it=40)
    d1q3 = synth.stefan_1d(nx=48).with_(max_it=40)
    return [("d2q5", d2q5, 40), ("d2q9", d2q9, 40), ("d1q3", d1q3, 300)]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_adjoint_step_dot_product(case):
    name, prob, warm = _cases()[case]
    f = _state_with_front(prob, warm)
    T = O.temperature(prob, f)
    # the state must straddle the melting temperature for a real test
    assert (np.abs(T) < 3 * prob.delta).any()
    rng = np.random.Generator(np.random.PCG64(100 + case))
    v = rng.standard_normal(f.shape)
    w = rng.standard_normal(f.shape)
    # state direction
    _, jv = O.cs_step(prob, f, f_im=H * v)
    fb, gw, gs, gd = O.adjoint_step(prob, f, w)
    lhs = np.sum(jv / H * w)
    rhs = np.sum(v * fb)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs)), (lhs, rhs)
    # parameter directions: Ste, delta and the x- wall profile
    _, js = O.cs_step(prob, f, ste_im=H)
    assert abs(np.sum(js / H * w) - gs) < 1e-11 * max(1.0, abs(gs))
    _, jd = O.cs_step(prob, f, delta_im=H)
    assert abs(np.sum(jd / H * w) - gd) < 1e-11 * max(1.0, abs(gd))
    u = rng.standard_normal(prob.ny)
    _, jw = O.cs_step(prob, f, wall_im=H * u)
    assert abs(np.sum(jw / H * w) - gw @ u) < 1e-11 * max(1.0, abs(gw @ u))


def _loss_case():
    n, m = 20, 8
    prob = synth.adjoint_2d(n=n, ny=m, nsteps=60, storage="f64").with_(
        max_it=40)
    tw_star = synth.wall_target_profile(m)
    target = O.front(prob.with_(wall_profile=(tw_star, None, None, None)),
                     O.run(prob.with_(wall_profile=(tw_star, None, None,
                                                    None)),
                           O.init(prob.with_(wall_profile=(tw_star, None,
                                                           None, None)),
                                  prob.T0), prob.nsteps)[0])
    return prob, target


def test_front_loss_gradient_matches_complex_step():
    prob, target = _loss_case()
    L, gw, gs, gd = O.front_loss_grad(prob, prob.T0, prob.nsteps, target)
    assert L > 0
    Lr, Li = O.cs_front_loss(prob, prob.T0, prob.nsteps, target, ste_im=H)
    assert abs(Lr - L) < 1e-15 * max(1, L) + 1e-18
    assert abs(Li / H - gs) < 1e-10 * abs(gs), (Li / H, gs)
    _, Li = O.cs_front_loss(prob, prob.T0, prob.nsteps, target, delta_im=H)
    assert abs(Li / H - gd) < 1e-10 * abs(gd), (Li / H, gd)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(3):
        u = rng.standard_normal(prob.ny)
        _, Li = O.cs_front_loss(prob, prob.T0, prob.nsteps, target,
                                wall_im=H * u)
        assert abs(Li / H - gw @ u) < 1e-10 * max(abs(gw @ u), 1e-12)


def test_front_loss_gradient_matches_central_differences():
    prob, target = _loss_case()
    L, gw, gs, gd = O.front_loss_grad(prob, prob.T0, prob.nsteps, target)
    def loss(**kw):
        return O.front_loss(prob.with_(**kw), prob.T0, prob.nsteps, target)
    h = 1e-6
    fd = (loss(ste=prob.ste * (1 + h)) - loss(ste=prob.ste * (1 - h))) / (
        2 * h * prob.ste)
    assert abs(fd - gs) < 1e-6 * abs(gs)
    fd = (loss(delta=prob.delta * (1 + h)) -
          loss(delta=prob.delta * (1 - h))) / (2 * h * prob.delta)
    assert abs(fd - gd) < 1e-6 * abs(gd)
    base = prob.wall_profile[0]
    for y in (0, 3, 7):
        e = np.zeros(prob.ny)
        e[y] = h
        fd = (loss(wall_profile=(base + e, None, None, None)) -
              loss(wall_profile=(base - e, None, None, None))) / (2 * h)
        assert abs(fd - gw[y]) < 1e-6 * max(abs(gw).max(), 1e-12)
