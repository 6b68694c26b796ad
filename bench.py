"""Benchmark of the IREBM step on one MI355X.

A step is one IREBM time step (collision, pull streaming, boundary
closures, local Newton solve, source and update, per-tile Newton and flux
statistics) over the whole lattice: one kernel launch.  Inputs are
resident in HBM before the timed region.

Default workload: the 8192 x 8192 D2Q9 cavity (FP32 populations, FP64
per-node arithmetic), heated at x = 0, adiabatic y walls, Ste drawn from
the seed, delta = 1.5 cells, tau = 0.6, Newton tol 1e-12.

Prints one JSON line.  Roofline: algorithmic bytes per launch
(2 q sizeof(population) per node: each population read once and written
once) over the average launch time measured with HIP events on the stream
the kernels run on.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "MLUPS and HBM GB/s (% roofline), plain vs batched vs adjoint, fixed tol"


def workload(name):
    import synth
    if name == "cavity":
        return synth.cavity_2d()
    if name == "planar":
        return synth.planar_2d()
    if name == "stefan1d":
        return synth.stefan_1d()
    raise SystemExit(f"unknown workload {name}")


KERNEL_SOURCES = ("irebm_node.hpp", "kernels.hpp", "host_util.hpp",
                  "lbm_stefan.hip")


def kernel_source_hash():
    """sha256 of the sources that define the single-lattice step kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2505_13097_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload, variant_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken with the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("sources_sha256") != kernel_source_hash() or
            rec.get("workload") != workload or
            rec.get("kernel_variant") != variant_name):
        return None
    return rec.get("bytes_per_launch")


def bytes_per_node(prob):
    s = 8 if prob.storage == "f64" else 4
    return 2 * prob.q * s


def time_plain(prob, steps, warmup, variant=-1, autotune=True):
    import torch
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob, variant=variant)
    stream = torch.cuda.current_stream()
    tuned = None
    if autotune and variant < 0:
        v, ms = g.autotune(steps=10)
        tuned = {"variant": v, "ms_per_step": round(ms, 4)}
        variant = v
    g.step(warmup)
    g.reset_stats()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    g.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gpu_ms = ev0.elapsed_time(ev1)
    st = g.stats()
    front = g.front("integral")
    g.close()
    return {"wall_s": t1 - t0, "gpu_ms": gpu_ms, "stats": st,
            "front_mean": float(front.mean()), "variant": variant,
            "tuned": tuned}


def time_batched(probs, steps, warmup, autotune=True, graph_steps=100,
                 variant=-1, bpc=0):
    """The batched form: all instances advanced by one persistent launch
    per step, replayed from a captured hipGraph of graph_steps launches."""
    import torch
    from paper_2505_13097_amd import StefanBatch, variant_names
    b = StefanBatch(probs)
    tuned = None
    v = variant
    if autotune:
        v, bpc, ms = b.autotune(steps=3)
        tuned = {"variant": variant_names(probs[0].q, probs[0].storage)[v],
                 "blocks_per_cu": bpc, "ms_per_step": round(ms, 4)}
    b.set_schedule(v, bpc, graph_steps)
    b.step(warmup)
    b.reset_stats()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    b.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = b.stats()
    b.close()
    nodes = sum(p.nodes for p in probs)
    bpn = bytes_per_node(probs[0])
    gpu_ms = ev0.elapsed_time(ev1)
    return {
        "workload": f"batch{len(probs)}_d2q5_{probs[0].storage}",
        "instances": len(probs), "nodes": nodes, "steps": steps,
        "value": round(nodes * steps / (t1 - t0) / 1e6, 1), "unit": "MLUPS",
        "hbm_gbps_algorithmic": round(nodes * bpn * steps / (gpu_ms * 1e-3) / 1e9, 1),
        "frac_of_peak": round(nodes * bpn * steps / (gpu_ms * 1e-3) / 1e9 /
                              HBM_PEAK_GBPS, 4),
        "ms_per_step": round(gpu_ms / steps, 4),
        "graph_steps": graph_steps, "autotune": tuned,
        "nonconverged": int(sum(s["nonconverged"] for s in st)),
        "max_newton_it": int(max(s["max_newton_it"] for s in st)),
    }


def time_adjoint(prob, interval):
    """The reverse mode: forward run keeping a checkpoint tape, then the
    reverse sweep (segment recompute + reverse steps) giving dL/dT_wall
    (512 values), dL/dSte and dL/ddelta for L = 1/2 sum (xf - xf*)^2,
    with xf* the front of a twin run with a seeded wall profile."""
    import numpy as np
    import torch
    import synth as S
    from paper_2505_13097_amd import Stefan, _lib
    twin = Stefan(prob.with_(wall_profile=(S.wall_target_profile(prob.ny),
                                           None, None, None)))
    twin.step(prob.nsteps)
    target = twin.front("integral")
    twin.close()
    s = Stefan(prob, flags=_lib.FLAG_ADJOINT)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    tape = s.forward_tape(prob.nsteps, interval)
    ev[1].record(stream)
    xf = s.front("integral")
    walls, gs, gd = s.backward_tape(xf - target, tape)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.close()
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[1].elapsed_time(ev[2])
    lups = prob.nodes * prob.nsteps
    return {
        "workload": prob.name, "steps": prob.nsteps,
        "checkpoint_interval": interval,
        "value": round(lups / (bwd_ms * 1e-3) / 1e6, 1),
        "unit": "MLUPS (reverse sweep: recompute + reverse steps)",
        "forward_tape_mlups": round(lups / (fwd_ms * 1e-3) / 1e6, 1),
        "total_s": round(t1 - t0, 4),
        "loss": float(0.5 * np.sum((xf - target) ** 2)),
        "grad_norms": {"wall": float(np.linalg.norm(walls["x-"])),
                       "ste": gs, "delta": gd},
    }


def cpu_baseline(prob, steps=1):
    """The oracle, as it stands, on `steps` steps of the same lattice from
    the same initial state (single thread)."""
    import oracle as O
    f = O.init(prob, prob.T0)
    t0 = time.perf_counter()
    O.run(prob, f, steps)
    dt = time.perf_counter() - t0
    return {"value": prob.nodes * steps / dt / 1e6, "unit": "MLUPS",
            "cores": 1, "kind": "oracle",
            "sample": f"{steps} step(s) of the full {prob.nx}x{prob.ny} "
                      f"{prob.name} lattice from its initial state, "
                      f"single-threaded C oracle, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cavity",
                    choices=["cavity", "planar", "stefan1d"])
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--forms", default="plain,batched,adjoint",
                    help="comma list of extra forms to time: batched, adjoint")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-variant", type=int, default=-1)
    ap.add_argument("--batch-bpc", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                          "--gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth  # noqa: F401
    from paper_2505_13097_amd import variant_names
    torch.cuda.set_device(0)

    prob = workload(args.workload)
    print(f"[bench] workload {prob.name}: {prob.nx}x{prob.ny} D2Q{prob.q} "
          f"steps {args.steps} warmup {args.warmup}", file=sys.stderr,
          flush=True)
    r = time_plain(prob, args.steps, args.warmup, args.variant,
                   autotune=not args.no_autotune)
    print(f"[bench] timed region done: {r['gpu_ms']:.1f} ms", file=sys.stderr,
          flush=True)
    ms_per_step = r["wall_s"] * 1e3 / args.steps
    mlups = prob.nodes * args.steps / r["wall_s"] / 1e6
    launch_ms = r["gpu_ms"] / args.steps
    bpn = bytes_per_node(prob)
    achieved = prob.nodes * bpn / (launch_ms * 1e-3) / 1e9
    v = r["variant"] if r["variant"] >= 0 else (0 if prob.q == 3 else 3)
    vname = variant_names(prob.q, prob.storage)[v]

    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": prob.name,
            "lattice": f"D{prob.dim}Q{prob.q}",
            "nx": prob.nx, "ny": prob.ny,
            "storage": prob.storage,
            "tau": prob.tau, "ste": round(prob.ste, 6),
            "delta_cells": round(prob.delta / prob.dx, 4),
            "newton_tol": prob.tol, "newton_max_it": prob.max_it,
            "bc": list(prob.bc),
            "kernel_variant": vname,
            "kernel_variant_id": v,
            "autotuned": r["tuned"] is not None,
        },
        "hbm_gbps_algorithmic": round(achieved, 1),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(prob.name, vname),
            "kernel": "step_kernel",
            "bytes_per_node": bpn,
            "avg_launch_us": round(launch_ms * 1e3, 2),
        },
        "newton": {
            "max_it": r["stats"]["max_newton_it"],
            "nonconverged": r["stats"]["nonconverged"],
            "max_residual": r["stats"]["max_residual"],
        },
    }
    forms = {}
    if "batched" in args.forms.split(","):
        import synth as S
        print(f"[bench] batched form: {args.batch_count} instances, "
              f"{args.batch_steps} steps", file=sys.stderr, flush=True)
        probs = S.batch_table(count=args.batch_count, nsteps=args.batch_steps)
        forms["batched"] = time_batched(
            probs, args.batch_steps, 10, autotune=not args.no_autotune,
            variant=args.batch_variant, bpc=args.batch_bpc)
        print("[bench] batched done", file=sys.stderr, flush=True)
    if "adjoint" in args.forms.split(","):
        import synth as S
        print("[bench] adjoint form", file=sys.stderr, flush=True)
        forms["adjoint"] = time_adjoint(S.adjoint_2d(), 64)
        print("[bench] adjoint done", file=sys.stderr, flush=True)
    if forms:
        out["forms"] = forms
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, 1 if prob.nodes > 1e6 else 200)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
