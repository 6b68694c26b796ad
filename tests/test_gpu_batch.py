"""GPU tests of the batched form: many uneven lattices in one persistent
launch per step must evolve exactly as each lattice stepped alone (same
per-node arithmetic), match the CPU oracle, survive hipGraph replays and
autotuning without any change of state."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _mixed(storage, count=7, seed=11):
    probs = synth.batch_table(count=count, seed=seed, sizes=[64, 128, 192],
                              storage=storage, nsteps=300)
    # uneven: one non-square, one with a wall profile, one plain Newton
    ny1 = probs[1].nx // 2 + 16
    probs[1] = probs[1].with_(ny=ny1, T0=probs[1].T0[:ny1])
    probs[2] = probs[2].with_(wall_profile=(
        0.8 + 0.4 * np.sin(np.arange(probs[2].ny) / 7.0), None, None, None))
    probs[3] = probs[3].with_(newton_mode="plain")
    return probs


def _single(prob, steps):
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob)
    g.step(steps)
    T = g.temperature()
    g.close()
    return T


def test_batch_members_equal_single_runs_and_oracle():
    from paper_2505_13097_amd import StefanBatch
    probs = _mixed("f64")
    # plain Newton cannot share a batch with safeguarded instances
    probs = [p for p in probs if p.newton_mode == "safeguarded"]
    b = StefanBatch(probs)
    b.step(300)
    st = b.stats()
    for k, p in enumerate(probs):
        T = b.temperature(k)
        assert np.array_equal(T, _single(p, 300)), k
        assert st[k]["nonconverged"] == 0
    for k in (0, 1, 2):
        p = probs[k]
        f, _ = O.run(p, O.init(p, p.T0), 300)
        err = np.abs(b.temperature(k) - O.temperature(p, f)).max()
        print(f"batch member {k} ({p.nx}x{p.ny}): max|dT| vs oracle {err:.2e}")
        assert err <= 1e-12
    b.close()


def test_batch_fp32_against_oracle():
    from paper_2505_13097_amd import StefanBatch
    probs = [p for p in _mixed("f32") if p.newton_mode == "safeguarded"]
    b = StefanBatch(probs)
    b.step(300)
    for k in (0, 2, 4):
        p = probs[k]
        f, _ = O.run(p, O.init(p, p.T0), 300)
        To = O.temperature(p, f)
        assert np.abs(b.temperature(k) - To).max() <= 1e-5
        cr = np.abs(b.front(k, "crossing") - O.front(p, f, O.FRONT_CROSSING))
        assert cr.max() <= p.dx
    b.close()


def test_batch_plain_newton_batch():
    from paper_2505_13097_amd import StefanBatch
    probs = [p.with_(newton_mode="plain") for p in _mixed("f64", count=4)]
    b = StefanBatch(probs)
    b.step(200)
    for k, p in enumerate(probs):
        assert np.array_equal(b.temperature(k), _single(p, 200))
    b.close()


@pytest.mark.parametrize("graph_steps", [2, 6])
def test_graph_replays_equal_eager_steps(graph_steps):
    from paper_2505_13097_amd import StefanBatch
    probs = [p for p in _mixed("f64") if p.newton_mode == "safeguarded"]
    eager = StefanBatch(probs)
    graph = StefanBatch(probs)
    graph.set_schedule(-1, 0, graph_steps)
    done = 0
    for rnd, n in enumerate([graph_steps, graph_steps + 1, 3 * graph_steps, 1]):
        graph.step(n)
        eager.step(n)
        done += n
        # eager work between replays (queries launch kernels of their own)
        for k in range(len(probs)):
            assert np.array_equal(graph.temperature(k), eager.temperature(k)), (rnd, k)
        graph.front(0)
    sg, se = graph.stats(), eager.stats()
    for a, c in zip(sg, se):
        assert a["energy"] == c["energy"]
        assert a["steps"] == c["steps"] == done
    graph.close()
    eager.close()


@pytest.mark.parametrize("variant,bpc", [(3, 2), (9, 0), (8, 4), (13, 0), (17, 2)])
def test_schedules_bitwise_identical(variant, bpc):
    """Persistent or one-block-per-tile, reversed sweeps, non-temporal
    stores: the per-node arithmetic is the same."""
    from paper_2505_13097_amd import StefanBatch
    probs = [p for p in _mixed("f64") if p.newton_mode == "safeguarded"]
    a = StefanBatch(probs)
    ref = StefanBatch(probs)
    a.set_schedule(variant, bpc, 0)
    a.step(41)
    ref.step(41)
    for k in range(len(probs)):
        assert np.array_equal(a.temperature(k), ref.temperature(k))
    a.close()
    ref.close()


def test_autotune_keeps_state_and_result():
    from paper_2505_13097_amd import StefanBatch
    probs = [p for p in _mixed("f32") if p.newton_mode == "safeguarded"]
    a = StefanBatch(probs)
    ref = StefanBatch(probs)
    a.step(20)
    ref.step(20)
    before = [a.temperature(k) for k in range(len(probs))]
    v, bpc, ms = a.autotune(steps=3)
    print(f"autotune: variant {v}, {bpc} blocks/CU, {ms:.4f} ms/step")
    assert ms > 0
    for k in range(len(probs)):
        assert np.array_equal(a.temperature(k), before[k])
    a.step(30)
    ref.step(30)
    for k in range(len(probs)):
        assert np.array_equal(a.temperature(k), ref.temperature(k))
    a.close()
    ref.close()


def test_single_lattice_autotune_keeps_state():
    from paper_2505_13097_amd import Stefan
    prob = synth.cavity_2d(n=300, ny=200, storage="f32")
    g = Stefan(prob)
    r = Stefan(prob)
    g.step(10)
    r.step(10)
    T = g.temperature()
    v, ms = g.autotune(steps=3)
    assert np.array_equal(g.temperature(), T)
    g.step(25)
    r.step(25)
    assert np.array_equal(g.temperature(), r.temperature())
    g.close()
    r.close()


def test_batch_energy_balance_per_instance():
    from paper_2505_13097_amd import StefanBatch
    probs = [p for p in _mixed("f64") if p.newton_mode == "safeguarded"]
    b = StefanBatch(probs)
    E0 = [b.energy(k) for k in range(len(probs))]
    b.step(200)
    for k, s in enumerate(b.stats()):
        dE = s["energy"] - E0[k]
        assert abs(dE - (s["flux_in"] - s["flux_out"])) < 1e-9 * max(1, abs(dE))
    b.close()


@pytest.mark.parametrize("name", ["128x2/t2/r16/nt", "128x4/t2/r32/nt"])
def test_batch_two_step_variants_equal_single_steps(name):
    """Two steps per launch in the batched form (odd step counts end with a
    one-step launch of the same kernel; graphs of an odd number of
    launches flip the buffers): states and statistics as one-step runs."""
    from paper_2505_13097_amd import StefanBatch, variant_names
    probs = [p for p in _mixed("f64") if p.newton_mode == "safeguarded"]
    v = variant_names(5, "f64").index(name)
    a = StefanBatch(probs)
    ref = StefanBatch(probs)
    a.set_schedule(v, 0, 6)
    done = 0
    for n in (6, 7, 1, 12, 3):
        a.step(n)
        ref.step(n)
        done += n
        for k in range(len(probs)):
            assert np.array_equal(a.temperature(k), ref.temperature(k)), (n, k)
    for sa, sr in zip(a.stats(), ref.stats()):
        assert sa["steps"] == sr["steps"] == done
        assert sa["max_newton_it"] == sr["max_newton_it"]
        assert sa["nonconverged"] == sr["nonconverged"] == 0
        assert abs(sa["flux_in"] - sr["flux_in"]) <= 1e-12 * max(1.0, abs(sr["flux_in"]))
    a.close()
    ref.close()



def _split_mix(storage, q=5):
    """Instances for the split two-step schedule: heated at x = 0 (front
    strip), heated at x = 1 only (its front in the last strip: the quiet
    pass flags those items), heated at both walls, a field just below
    melting everywhere (every item flagged), a wall profile, a non-square
    lattice, and sizes from one strip (64) to three (300)."""
    probs = synth.batch_table(count=6, seed=23, sizes=[64, 192, 300],
                              storage=storage, nsteps=40)
    p = [x.with_(q=q) for x in probs]
    p[1] = p[1].with_(wall_T=(-0.5, 1.0, 0.0, 0.0))
    p[2] = p[2].with_(wall_T=(1.0, 1.0, 0.0, 0.0))
    p[3] = p[3].with_(T0=np.full((p[3].ny, p[3].nx), -2.0 * p[3].delta))
    p[4] = p[4].with_(wall_profile=(
        0.8 + 0.4 * np.sin(np.arange(p[4].ny) / 5.0), None, None, None))
    ny5 = p[5].nx // 2 + 9
    p[5] = p[5].with_(ny=ny5, T0=p[5].T0[:ny5])
    return p


def test_split_two_step_schedule_d2q9():
    """The split schedule on D2Q9 instances (diagonal pulls in the front
    kernel's LDS rows and in the quiet pass), FP64 and FP32: states equal
    one-step launches bit for bit."""
    from paper_2505_13097_amd import StefanBatch, variant_names
    for storage in ("f64", "f32"):
        probs = _split_mix(storage, q=9)
        v = variant_names(9, storage).index("128x2/t2s/r96/nt")
        a = StefanBatch(probs)
        ref = StefanBatch(probs)
        a.set_schedule(v, 0, 4)
        for n in (4, 5, 2):
            a.step(n)
            ref.step(n)
            for k in range(len(probs)):
                assert np.array_equal(a.temperature(k), ref.temperature(k)), \
                    (storage, n, k)
        for sa, sr in zip(a.stats(), ref.stats()):
            assert sa["max_newton_it"] == sr["max_newton_it"]
            assert sa["nonconverged"] == sr["nonconverged"]
        a.close()
        ref.close()


@pytest.mark.parametrize("name", ["128x2/t2s/r16/nt", "128x4/t2s/r32/nt",
                                  "128x2/t2s/r96/nt",
                                  "128x2/t2s/r64/nt"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_split_two_step_schedule_equals_single_steps(name, storage):
    """The split two-step schedule (front strips by two column-limited
    one-step passes, quiet pass, full pass over flagged items) gives the
    states of one-step launches bit for bit, in eager launches and graph
    replays, with odd step counts, and the same statistics."""
    from paper_2505_13097_amd import StefanBatch, variant_names
    probs = _split_mix(storage)
    v = variant_names(5, storage).index(name)
    a = StefanBatch(probs)
    ref = StefanBatch(probs)
    a.set_schedule(v, 0, 6)
    done = 0
    for n in (6, 7, 1, 12, 3, 2):
        a.step(n)
        ref.step(n)
        done += n
        for k in range(len(probs)):
            assert np.array_equal(a.temperature(k), ref.temperature(k)), (n, k)
    for k, (sa, sr) in enumerate(zip(a.stats(), ref.stats())):
        assert sa["steps"] == sr["steps"] == done
        assert sa["max_newton_it"] == sr["max_newton_it"], k
        assert sa["nonconverged"] == sr["nonconverged"], k
        assert sa["max_residual"] == sr["max_residual"], k
        for f in ("flux_in", "flux_out"):
            assert abs(sa[f] - sr[f]) <= 1e-12 * max(1.0, abs(sr[f])), (k, f)
    a.close()
    ref.close()


@pytest.mark.parametrize("schedule", ["bench", "autotune"])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_full_table_of_512_instances_against_oracle(storage, schedule):
    """The batched workload itself: the 512-instance table of the bench
    (sizes 64^2 to 1024^2, about 2.1e8 nodes, a workspace above 8 GB in
    FP32) in the bench's schedule (its fixed kernel variant, one block per
    work item, hipGraph replays of two steps) or the autotuner's pick, six
    steps; the 8 smallest and the 2 largest instances against the oracle
    in full (T, both fronts, energy, Newton counters)."""
    import bench
    from paper_2505_13097_amd import StefanBatch, variant_names
    probs = synth.batch_table(count=512, storage=storage)
    nodes = np.array([p.nodes for p in probs])
    order = np.argsort(nodes, kind="stable")
    picks = list(order[:8]) + list(order[-2:])
    b = StefanBatch(probs)
    ws = b.workspace.numel()
    names = variant_names(5, storage)
    if schedule == "bench":
        v, bpc = names.index(bench.DEFAULT_VARIANTS["batched"]), 0
    else:
        v, bpc, _ = b.autotune(steps=2)
    b.set_schedule(v, bpc, 2)
    print(f"batch512 {storage}: {nodes.sum()} nodes, workspace "
          f"{ws / 2**30:.2f} GiB, variant {names[v]}, blocks per CU {bpc}",
          flush=True)
    assert ws > (8 if storage == "f32" else 16) * 10**9 * 0.95
    steps = 6
    b.step(steps)
    st = b.stats()
    tol = 1e-12 if storage == "f64" else 1e-5
    worst = 0.0
    for k in picks:
        p = probs[k]
        f, ost = O.run(p, O.init(p, p.T0), steps)
        To = O.temperature(p, f)
        T = b.temperature(k)
        err = np.abs(T - To).max()
        worst = max(worst, err)
        assert err <= tol * max(1.0, np.abs(To).max()), (k, p.nx, err)
        cr = np.abs(b.front(k, "crossing") - O.front(p, f, O.FRONT_CROSSING))
        fr = np.abs(b.front(k, "integral") - O.front(p, f, O.FRONT_INTEGRAL))
        assert cr.max() <= (1e-12 if storage == "f64" else p.dx)
        assert fr.max() <= tol * p.nx * p.dx / p.delta + 1e-13
        E = O.energy(p, f)
        assert abs(b.energy(k) - E) <= (1e-11 if storage == "f64" else 1e-5
                                        ) * max(1.0, abs(E))
        assert st[k]["nonconverged"] == 0 and ost["nonconverged"] == 0
        # FP32 states round the temperatures the solves start from
        assert abs(st[k]["max_newton_it"] - ost["max_it"]) <= \
            (1 if storage == "f64" else 2)
    print(f"batch512 {storage} [{names[v]}]: instances {picks} "
          f"(sizes {[probs[k].nx for k in picks]}), max|dT| {worst:.3e}",
          flush=True)
    b.close()
