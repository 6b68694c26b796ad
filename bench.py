"""Benchmark of the IREBM step on one MI355X.

A step is one IREBM time step (collision, pull streaming, boundary
closures, local Newton solve, source and update, per-item Newton and flux
statistics) over the whole lattice: one kernel launch, or half of one for
the temporally blocked variants that advance two steps per launch.  Inputs
are resident in HBM before the timed region.

Default workload: the 8192 x 8192 D2Q9 cavity (FP32 populations, FP64
per-node arithmetic), heated at x = 0, adiabatic y walls, Ste drawn from
the seed, delta = 1.5 cells, tau = 0.6, Newton tol 1e-12.

Further forms in "forms" (--forms): the batched form (512 D2Q5 lattices,
64^2 to 1024^2), the reverse mode (512^2 D2Q5, 4096 steps), the explicit
scheme on the same cavity, the 2048^2 D2Q5 planar front (10,000 steps,
both schemes), the paper's 2D freezing case and 1D case with
the three schemes, the 512^3 cube on D3Q19 and D3Q7, and the freezing
case taken to 3D.

Prints one JSON line.  Roofline: algorithmic bytes per launch
(2 q sizeof(population) per lattice update: each population read once and
written once, times the updates one launch performs) over the average
launch time measured with HIP events on the stream the kernels run on.  A
two-step launch moves about half of those bytes (roofline.traffic, from
the counter runs), so its achieved rate can exceed what HBM delivers.
"""
import argparse
import json
import math
import os
import re
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
                  "launch.hpp", "k_step_safeguarded.hip")


def kernel_source_hash():
    """sha256 of the sources that define the single-lattice step kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2505_13097_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def measured_traffic(workload, variant_name):
    """HBM bytes per launch of the step kernel in this variant, from the
    committed rocprofv3 counter summary, if it was taken with the current
    kernel sources, else None."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("sources_sha256") != kernel_source_hash() or
            rec.get("workload") != workload):
        return None
    v = rec.get("variants", {}).get(variant_name)
    return None if v is None else v.get("bytes_per_launch")


KERNEL3_SOURCES = ("irebm_node.hpp", "kernels.hpp", "lattice3d.hpp",
                   "launch3.hpp", "k_step3_safeguarded.hip")
TRAFFIC3_JSON = os.path.join(ROOT, "profiles", "step3_kernel_traffic.json")


def kernel3_source_hash():
    """sha256 of the sources that define the 3D step kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2505_13097_amd", "csrc")
    for name in KERNEL3_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic3(workload, variant_name):
    """HBM bytes per launch of the 3D step kernel, from the committed
    counter summary when it matches the current sources, else None."""
    try:
        with open(TRAFFIC3_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel3_source_hash():
        return None
    v = rec.get("lattices", {}).get(workload, {}).get(variant_name)
    return None if v is None else v.get("bytes_per_launch")


# Kernel variants the bench times unless --autotune is given: the fastest
# of the autotuner's sweeps on these lattices, fixed so that a run and the
# committed rocprofv3 summaries name the same kernel.
DEFAULT_VARIANTS = {
    "cavity": "128x4/t2/r32/nt",
    "cavity_eebm": "256x2/t2/r32/nt",
    "planar": "128x2/npt2",
    "planar_eebm": "128x2/npt2",
    "stefan1d": "resident2048",
    "batched": "128x2/t2s/r96/nt",
    "adjoint": "256x1/npt1",
    "cube3d_19": "256x1/npt2/z4/nt",
    "cube3d_7": "64x4/npt1/z8/nt/s",
}


def variant_id(q, storage, name):
    """index of a kernel variant by its name"""
    from paper_2505_13097_amd import variant_names
    names = variant_names(q, storage)
    if name not in names:
        raise SystemExit(f"no kernel variant {name} for q = {q}")
    return names.index(name)


def bytes_per_node(prob):
    s = 8 if prob.storage == "f64" else 4
    return 2 * prob.q * s


def time_plain(prob, steps, warmup, variant=-1, autotune=False):
    """W untimed steps, then K steps timed with HIP events on the stream
    the kernels run on (torch's current stream, which the handle uses)."""
    import torch
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob, variant=variant)
    stream = torch.cuda.current_stream()
    tuned = None
    if autotune:
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


def time_batched(probs, steps, warmup, autotune=False, graph_steps=100,
                 variant=-1, bpc=0):
    """The batched form: all instances advanced by one persistent launch
    per step, replayed from a captured hipGraph of graph_steps launches."""
    import torch
    from paper_2505_13097_amd import StefanBatch, variant_names
    b = StefanBatch(probs)
    tuned = None
    v = variant
    if v < 0 and not autotune:
        v = variant_id(probs[0].q, probs[0].storage, DEFAULT_VARIANTS["batched"])
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


def time_eebm(prob, steps, warmup, autotune, irebm_ms_per_step, variant=-1,
              key=None):
    """The explicit enthalpy based method (Algorithm 2) on the same
    lattice, same kernels and state layout, no Newton solve; the paper's
    timing tables report the IREBM/EEBM time ratio."""
    from paper_2505_13097_amd import variant_names
    pe = prob.with_(scheme="eebm", name=prob.name + "_eebm")
    dflt = DEFAULT_VARIANTS.get(f"{key}_eebm")
    if variant < 0 and not autotune and dflt:
        variant = variant_id(pe.q, pe.storage, dflt)
    r = time_plain(pe, steps, warmup, variant, autotune=autotune)
    v = r["variant"] if r["variant"] >= 0 else (0 if pe.q == 3 else 3)
    vname = variant_names(pe.q, pe.storage)[v]
    spl = steps_per_launch(vname)
    launch_ms = r["gpu_ms"] / (steps // spl)
    gbps = pe.nodes * bytes_per_node(pe) * spl / (launch_ms * 1e-3) / 1e9
    ms = r["wall_s"] * 1e3 / steps
    return {
        "workload": pe.name, "steps": steps,
        "value": round(pe.nodes * steps / r["wall_s"] / 1e6, 1),
        "unit": "MLUPS", "ms_per_step": round(ms, 4),
        "kernel_variant": vname,
        "hbm_gbps_algorithmic": round(gbps, 1),
        "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4),
        "time_ratio_irebm_to_eebm": round(irebm_ms_per_step / ms, 3),
    }


def time_planar(steps=10000, warmup=20, autotune=False):
    """The plain step on the 2048^2 planar-front lattice (D2Q5, FP32
    storage, 10,000 steps): both state buffers (2 x 84 MB) fit in the
    memory-side cache, so the algorithmic rate can exceed what HBM alone
    delivers.  The explicit scheme on the same lattice gives the time
    ratio."""
    import synth
    from paper_2505_13097_amd import variant_names
    out = {}
    for scheme in ("irebm", "eebm"):
        prob = synth.planar_2d(nsteps=steps)
        if scheme == "eebm":
            prob = prob.with_(scheme="eebm", name=prob.name + "_eebm")
        v = -1 if autotune else variant_id(
            prob.q, prob.storage,
            DEFAULT_VARIANTS["planar" if scheme == "irebm" else "planar_eebm"])
        r = time_plain(prob, steps, warmup, v, autotune=autotune)
        v = r["variant"] if r["variant"] >= 0 else 3
        vname = variant_names(prob.q, prob.storage)[v]
        spl = steps_per_launch(vname)
        launch_ms = r["gpu_ms"] / (steps // spl)
        gbps = prob.nodes * bytes_per_node(prob) * spl / (launch_ms * 1e-3) / 1e9
        out[scheme] = {
            "workload": prob.name, "steps": steps,
            "value": round(prob.nodes * steps / r["wall_s"] / 1e6, 1),
            "unit": "MLUPS",
            "ms_per_step": round(r["gpu_ms"] / steps, 5),
            "kernel_variant": vname,
            "hbm_gbps_algorithmic": round(gbps, 1),
            "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4),
            "newton_max_it": r["stats"]["max_newton_it"],
            "nonconverged": r["stats"]["nonconverged"],
            "front_mean": round(r["front_mean"], 6),
        }
    irebm = out["irebm"]
    irebm["eebm_ms_per_step"] = out["eebm"]["ms_per_step"]
    irebm["time_ratio_irebm_to_eebm"] = round(
        irebm["ms_per_step"] / out["eebm"]["ms_per_step"], 3)
    return irebm


CUBE3D_N = 512


def time_cube3d(steps=50, warmup=5, autotune=False, variant=-1, n=CUBE3D_N):
    """The 3D lattices (the enthalpy model holds in 3D, Section 2): the
    n^3 cube heated at one face (Dirichlet x faces, bounce-back y and z
    faces), D3Q19 and D3Q7, FP32 populations, IREBM and then EEBM on the
    same kernel variant; algorithmic bytes 2 q s per lattice update."""
    import synth as S
    from paper_2505_13097_amd import variant_names
    rows = []
    for q in (19, 7):
        p = S.cavity_3d(n=n, q=q)
        print(f"[bench] cube3d D3Q{q} {n}^3", file=sys.stderr, flush=True)
        v = variant
        if v < 0 and not autotune:
            v = variant_id(q, p.storage, DEFAULT_VARIANTS[f"cube3d_{q}"])
        r = time_plain(p, steps, warmup, v, autotune=autotune)
        v = r["variant"] if r["variant"] >= 0 else 0
        vname = variant_names(q, p.storage)[v]
        launch_ms = r["gpu_ms"] / steps
        alg = p.nodes * bytes_per_node(p)
        gbps = alg / (launch_ms * 1e-3) / 1e9
        pe = p.with_(scheme="eebm", name=p.name.replace("irebm", "eebm"))
        e = time_plain(pe, steps, warmup, v, autotune=False)
        e_ms = e["gpu_ms"] / steps
        rows.append({
            "workload": p.name, "lattice": f"D3Q{q}", "nodes": p.nodes,
            "steps": steps, "kernel_variant": vname,
            "autotuned": r["tuned"] is not None,
            "value": round(p.nodes * steps / r["wall_s"] / 1e6, 1),
            "unit": "MLUPS",
            "avg_launch_us": round(launch_ms * 1e3, 2),
            "bytes_per_lattice_update": bytes_per_node(p),
            "hbm_gbps_algorithmic": round(gbps, 1),
            "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic3(p.name, vname),
            "newton_max_it": r["stats"]["max_newton_it"],
            "nonconverged": r["stats"]["nonconverged"],
            "eebm_avg_launch_us": round(e_ms * 1e3, 2),
            "eebm_hbm_gbps_algorithmic": round(alg / (e_ms * 1e-3) / 1e9, 1),
            "time_ratio_irebm_to_eebm": round(launch_ms / e_ms, 3),
        })
    return {"unit": "MLUPS per lattice", "runs": rows}


def traffic_sweep3(n=CUBE3D_N):
    """Counter runs of the 3D step kernel: every 3D variant for SWEEP_STEPS
    steps on the D3Q19, then the D3Q7 cube (IREBM), in table order."""
    import torch
    import synth as S
    from paper_2505_13097_amd import Stefan, variant_names
    for q in (19, 7):
        g = Stefan(S.cavity_3d(n=n, q=q))
        for v in range(len(variant_names(q, "f32"))):
            g.set_variant(v)
            g.step(SWEEP_STEPS)
        torch.cuda.synchronize()
        g.close()
        torch.cuda.empty_cache()


def cube3d_kernels(q, vname, mode=0):
    """Trace names of the kernels one 3D step runs under variant vname on
    the cube heated at x = 0 (IREBM mode 0, EEBM mode 2), by role: a split
    variant runs the front strip (variant 0's tiling), the quiet pass and
    the full pass (IREBM)."""
    m = re.fullmatch(r"(\d+)x(\d+)/npt(\d+)/z(\d+)(/nt)?(/s)?", vname)
    npt = int(m.group(3))
    nt = "true" if m.group(5) else "false"
    base = f"step3_kernel<{q}, float, {npt}, {mode}, {nt}"
    if m.group(6) and mode != 2:
        return {"front": f"step3_kernel<{q}, float, 1, {mode}, true, 0>",
                "quiet": base + ", 1>", "full": base + ", 2>"}
    return {"step": base + ", 0>"}


def summarize_profiles3(run, args):
    """profiles/ summaries of the 3D step kernel from run/prof3d (kernel
    trace of bench.py --cube3d-only with a fixed variant) and
    run/pmc3d_fetch, run/pmc3d_write (bench.py --traffic-sweep-3d)."""
    import collections
    import re
    import sqlite3
    import synth as S
    from paper_2505_13097_amd import variant_names

    def short(nm):
        nm = nm.replace("(anonymous namespace)::", "").replace("irebm::", "")
        return nm.split("(")[0].replace("void ", "")

    def db(sub):
        d = os.path.join(run, sub)
        f = [x for x in os.listdir(d) if x.endswith("_results.db")]
        return sqlite3.connect(os.path.join(d, f[0]))

    def kq(k):
        m = re.match(r"step3_kernel<(\d+), float, \d, (\d+),", k)
        return (int(m.group(1)), int(m.group(2))) if m else None

    def vdefault(q):
        if args.variant3d >= 0:
            return variant_names(q, "f32")[args.variant3d]
        return DEFAULT_VARIANTS[f"cube3d_{q}"]

    c = db("prof3d")
    trace = [(short(r[0]), r[1], r[2], r[3], r[4]) for r in c.execute(
        "select name, total_calls, total_duration, average, percentage "
        "from top_kernels")]
    steps = args.steps3d
    # time per step of the timed launches (the last `steps` of each role;
    # a split step's kernels overlap on two streams: first start to last
    # end)
    avg = {}
    roles = {}
    for q in (19, 7):
        for mode in (0, 2):
            ks = cube3d_kernels(q, vdefault(q), mode)
            w = batch_walls(c, short, ks)[-steps:]
            if w:
                avg[(q, mode)] = sum(w) / len(w)
                roles[(q, mode)] = ks

    def counters(sub, cn):
        rows = db(sub).execute(
            "select kernel_name, value from counters_collection where "
            "counter_name=? order by dispatch_id", (cn,)).fetchall()
        return [(short(k), v) for k, v in rows]
    F = counters("pmc3d_fetch", "FETCH_SIZE")
    W = counters("pmc3d_write", "WRITE_SIZE")
    gib_kib = 1024.0 * 1024.0
    copy_f = max(v for k, v in F if "copyBuffer" in k)
    copy_w = max(v for k, v in W if "copyBuffer" in k)
    fs, ws = gib_kib / copy_f, gib_kib / copy_w
    lattices = {}
    src = kernel3_source_hash()
    for q in (19, 7):
        p = S.cavity_3d(n=args.cube3d_n, q=q)
        names = variant_names(q, "f32")
        sf = [v for k, v in F if kq(k) == (q, 0)]
        sw = [v for k, v in W if kq(k) == (q, 0)]
        # dispatches per step: three for a split variant (front strip, quiet
        # and full pass), else one
        per = [3 if nm.endswith("/s") else 1 for nm in names]
        need = SWEEP_STEPS * sum(per)
        if len(sf) != need or len(sw) != len(sf):
            raise SystemExit(f"D3Q{q}: expected {need} "
                             f"dispatches, found {len(sf)} / {len(sw)}")
        alg = p.nodes * bytes_per_node(p)
        rec = {}
        o = 0
        for i, nm in enumerate(names):
            n_ = SWEEP_STEPS * per[i]
            fk = sum(sf[o:o + n_]) / SWEEP_STEPS
            wk = sum(sw[o:o + n_]) / SWEEP_STEPS
            o += n_
            b = fk * 1024 * fs + wk * 1024 * ws
            rec[nm] = {"fetch_kib_per_dispatch": round(fk, 1),
                       "write_kib_per_dispatch": round(wk, 1),
                       "bytes_per_launch": round(b),
                       "bytes_per_lattice_update": round(b / p.nodes, 3),
                       "ratio_to_algorithmic": round(b / alg, 4)}
        lattices[p.name] = rec
    vname = {q: vdefault(q) for q in (19, 7)}
    trace_cmd = (f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof3d -o p3"
                 f" -- python bench.py --cube3d-only"
                 + (f" --variant3d {args.variant3d}" if args.variant3d >= 0
                    else "") + f" --steps3d {steps}")
    pmc_cmd = ("rocprofv3 --pmc {C} -d gpurun_out/{D} -o {O} -- python "
               "bench.py --traffic-sweep-3d")
    lines = [f"# step3_kernel — {args.cube3d_n}^3 cube heated at one face, "
             "D3Q19 and D3Q7, FP32 populations", "",
             "Kernel trace (rocprofv3 on MI355X; run from /tmp with "
             "TMPDIR=/tmp, paths absolute; summary written by bench.py "
             "--summarize-profiles3):", "", "    " + trace_cmd, "",
             "| kernel | calls | total us | average us | % |",
             "|---|---|---|---|---|"]
    for r in trace[:12]:
        lines.append(f"| {r[0]} | {r[1]} | {r[2]:.0f} | {r[3]:.1f} | "
                     f"{r[4]:.2f} |")
    lines += ["", "Timed steps (the last " + str(steps) + " of each "
              "lattice and scheme; mode 0 IREBM, 2 EEBM; a split step's "
              "time runs from its first kernel's start to its last kernel's "
              "end, from the trace's timestamps):", "",
              "| lattice | mode | variant | kernels | us per step | "
              "algorithmic GB/s |", "|---|---|---|---|---|---|"]
    for (q, mode), a in sorted(avg.items(), reverse=True):
        p = S.cavity_3d(n=args.cube3d_n, q=q)
        ks = ", ".join(f"{r}: {k}" for r, k in roles[(q, mode)].items())
        lines.append(f"| D3Q{q} | {mode} | {vname[q]} | {ks} | {a:.1f} | "
                     f"{p.nodes * bytes_per_node(p) / (a * 1e-6) / 1e9:.0f} |")
    lines += ["", "HBM traffic per launch of every variant (IREBM, two "
              "counter runs, one counter each):", "",
              "    " + pmc_cmd.format(C="FETCH_SIZE", D="pmc3d_fetch",
                                      O="fetch"),
              "    " + pmc_cmd.format(C="WRITE_SIZE", D="pmc3d_write",
                                      O="write"), "",
              f"Counter scale from a 1 GiB device copy in the same runs: "
              f"FETCH_SIZE x{fs:.4f}, WRITE_SIZE x{ws:.4f}.", ""]
    for wl, rec in lattices.items():
        lines += [f"{wl}:", "",
                  "| variant | FETCH KiB | WRITE KiB | bytes/launch | "
                  "B per lattice update | / algorithmic |",
                  "|---|---|---|---|---|---|"]
        for nm, r in rec.items():
            lines.append(f"| {nm} | {r['fetch_kib_per_dispatch']:.0f} | "
                         f"{r['write_kib_per_dispatch']:.0f} | "
                         f"{r['bytes_per_launch'] / 1e9:.3f} GB | "
                         f"{r['bytes_per_lattice_update']:.2f} | "
                         f"{r['ratio_to_algorithmic']:.4f} |")
        lines.append("")
    lines += [f"Kernel sources sha256 {src}.", ""]
    fn = f"step3_kernel_cube{args.cube3d_n}_d3q19_d3q7_f32.md"
    with open(os.path.join(ROOT, "profiles", fn), "w") as f:
        f.write("\n".join(lines))
    with open(TRAFFIC3_JSON, "w") as f:
        json.dump({"kernel": "step3_kernel", "sources_sha256": src,
                   "fetch_scale": fs, "write_scale": ws,
                   "lattices": lattices, "source": "profiles/" + fn}, f,
                  indent=1)
    print(f"wrote profiles/{fn}, {os.path.relpath(TRAFFIC3_JSON, ROOT)}")


def _run_seconds(prob, nsteps):
    """Wall time of nsteps steps of a fresh handle (after 5 warm steps),
    and its statistics."""
    import torch
    from paper_2505_13097_amd import Stefan
    g = Stefan(prob)
    g.step(5)
    g.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(nsteps, stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    return dt, st


def time_paper1d(sizes=(201, 401, 801)):
    """The paper's 1D case (Section 6.1) to t = 160 s with the three
    schemes of its 1D timing table (tau 0.62, delta 0.01 for IREBM; D1Q3,
    FP64; ILFBM inner loop to 1e-12, at most 200 iterations)."""
    import numpy as np
    import synth as S
    ste, th0 = 0.2857, -0.5
    t_end = 160.0 * 8e-5
    tau = 0.62
    rows = []
    for n in sizes:
        dx = 1.0 / (n - 1)
        dt = (tau - 0.5) * dx * dx / 3.0
        nsteps = int(round(t_end / dt))
        base = S.Problem(dim=1, q=3, nx=n, ny=1, tau=tau, ste=ste, delta=0.01,
                         bc=("dirichlet", "dirichlet", "periodic", "periodic"),
                         wall_T=(1.0, th0, 0.0, 0.0), tol=1e-12, max_it=200,
                         storage="f64", T0=np.full((1, n), th0))
        r = {"N": n, "steps": nsteps}
        for scheme in ("eebm", "irebm", "ilfbm"):
            sec, st = _run_seconds(base.with_(scheme=scheme), nsteps)
            r[f"{scheme}_s"] = round(sec, 4)
            if scheme == "ilfbm":
                r["ilfbm_max_inner_iterations"] = st["max_newton_it"]
                r["ilfbm_capped_steps"] = st["nonconverged"]
        r["ratio_irebm_to_eebm"] = round(r["irebm_s"] / r["eebm_s"], 3)
        r["ratio_ilfbm_to_irebm"] = round(r["ilfbm_s"] / r["irebm_s"], 3)
        rows.append(r)
    return {"workload": "stefan1d_d1q3_f64_to_160s", "unit": "s per run",
            "runs": rows}


def time_freezing(sizes=(201, 401, 801)):
    """The paper's 2D freezing case (Section 6.2) run to t = 20 h, D2Q5 and
    D2Q9, EEBM and IREBM, FP64 populations: the configuration of the
    paper's 2D timing table, whose IREBM/EEBM ratio is reported beside the
    times (one launch per step: these lattices are small, so the launches,
    not HBM, bound them)."""
    import torch
    from paper_2505_13097_amd import Stefan
    import synth as S
    rows = []
    for q in (5, 9):
        for n in sizes:
            r = {"lattice": f"D2Q{q}", "N": n}
            for scheme in ("eebm", "irebm"):
                p = S.freezing_cavity_2d(n=n, q=q, scheme=scheme)
                g = Stefan(p)
                g.step(20)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.step(p.nsteps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                g.close()
                r["steps"] = p.nsteps
                r[f"{scheme}_s"] = round(dt, 4)
                r[f"{scheme}_glups"] = round(p.nodes * p.nsteps / dt / 1e9, 2)
            r["ratio_irebm_to_eebm"] = round(r["irebm_s"] / r["eebm_s"], 3)
            if q == 9 and n <= 401:
                # ILFBM converges on D2Q9 only (about 80 inner iterations)
                p = S.freezing_cavity_2d(n=n, q=q, scheme="ilfbm").with_(
                    max_it=200)
                sec, st = _run_seconds(p, p.nsteps)
                r["ilfbm_s"] = round(sec, 4)
                r["ilfbm_max_inner_iterations"] = st["max_newton_it"]
                r["ilfbm_capped_steps"] = st["nonconverged"]
            rows.append(r)
    return {"workload": "freeze2d_quarter_cavity_f64_20h",
            "unit": "s per run to 20 h", "runs": rows}


def time_freezing3d(sizes=(101, 201)):
    """The freezing case taken to 3D (the octant of a cube cooled on every
    face, Dirichlet and symmetry faces, the 2D case's parameters), run to
    t = 20 h, D3Q7 and D3Q19, EEBM and IREBM, FP64 populations: the 2D
    timing table's IREBM/EEBM ratio in 3D."""
    import torch
    from paper_2505_13097_amd import Stefan
    import synth as S
    rows = []
    for q in (7, 19):
        for n in sizes:
            r = {"lattice": f"D3Q{q}", "N": n}
            for scheme in ("eebm", "irebm"):
                p = S.freezing_cube_3d(n=n, q=q, scheme=scheme)
                g = Stefan(p)
                g.step(5)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.step(p.nsteps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                g.close()
                r["steps"] = p.nsteps
                r[f"{scheme}_s"] = round(dt, 4)
                r[f"{scheme}_glups"] = round(p.nodes * p.nsteps / dt / 1e9, 2)
            r["ratio_irebm_to_eebm"] = round(r["irebm_s"] / r["eebm_s"], 3)
            rows.append(r)
    return {"workload": "freeze3d_octant_f64_20h",
            "unit": "s per run to 20 h", "runs": rows}


def time_adjoint(prob, interval, autotune=False):
    """The reverse mode: forward run keeping a checkpoint tape, then the
    reverse sweep (segment recompute + reverse steps) giving dL/dT_wall
    (512 values), dL/dSte and dL/ddelta for L = 1/2 sum (xf - xf*)^2,
    with xf* the front of a twin run with a seeded wall profile."""
    import numpy as np
    import torch
    import synth as S
    from paper_2505_13097_amd import Stefan, _lib, variant_names
    twin = Stefan(prob.with_(wall_profile=(S.wall_target_profile(prob.ny),
                                           None, None, None)))
    twin.step(prob.nsteps)
    target = twin.front("integral")
    twin.close()
    s = Stefan(prob, flags=_lib.FLAG_ADJOINT)
    if autotune:
        v, ms = s.autotune(steps=20)
    else:
        v = variant_id(prob.q, prob.storage, DEFAULT_VARIANTS["adjoint"])
        s.set_variant(v)
    tuned = variant_names(prob.q, prob.storage)[v]
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
    del tape
    torch.cuda.empty_cache()
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[1].elapsed_time(ev[2])
    lups = prob.nodes * prob.nsteps
    # algorithmic bytes per node-step of the reverse sweep: the reverse
    # step reads the forward state (q s) and the adjoint arrays of the step
    # after it (q + 1 FP64) and writes them for this step (q + 1 FP64);
    # with checkpoints, the segment recompute adds one forward step (2 q s)
    s_b = 8 if prob.storage == "f64" else 4
    rev_b = prob.q * s_b + 2 * (prob.q + 1) * 8
    bwd_b = rev_b + (2 * prob.q * s_b if interval > 1 else 0)
    bwd_gbps = lups * bwd_b / (bwd_ms * 1e-3) / 1e9
    fwd_gbps = lups * bytes_per_node(prob) / (fwd_ms * 1e-3) / 1e9
    return {
        "workload": prob.name, "steps": prob.nsteps,
        "checkpoint_interval": interval, "forward_variant": tuned,
        "value": round(lups / (bwd_ms * 1e-3) / 1e6, 1),
        "unit": "MLUPS (reverse sweep: recompute + reverse steps)",
        "forward_tape_mlups": round(lups / (fwd_ms * 1e-3) / 1e6, 1),
        "bytes_per_node_step": bwd_b,
        "hbm_gbps_algorithmic": round(bwd_gbps, 1),
        "frac_of_peak": round(bwd_gbps / HBM_PEAK_GBPS, 4),
        "forward_tape_gbps_algorithmic": round(fwd_gbps, 1),
        "note": "both states and adjoint arrays (5.2 MB and 10.5 MB) sit in "
                "the memory-side cache: launch latency, not HBM, bounds "
                "this form",
        "total_s": round(t1 - t0, 4),
        "loss": float(0.5 * np.sum((xf - target) ** 2)),
        "grad_norms": {"wall": float(np.linalg.norm(walls["x-"])),
                       "ste": gs, "delta": gd},
    }


SWEEP_STEPS = 4


RESIDENT_STEPS = 4096   # steps per launch of the resident D1Q3 kernel


def steps_per_launch(variant_name, steps=1):
    """Time steps one launch of this variant advances (two for the
    temporally blocked "/t2" variants; up to RESIDENT_STEPS of a run of
    `steps` for the resident D1Q3 kernel)."""
    if variant_name.startswith("resident"):
        return min(steps, RESIDENT_STEPS)
    return 2 if "/t2" in variant_name else 1


def traffic_sweep(prob):
    """For counter runs: every kernel variant of the workload's lattice for
    SWEEP_STEPS steps each, in table order (the summary maps the step-kernel
    dispatches to variants by that order: SWEEP_STEPS launches of a
    one-step variant, SWEEP_STEPS / 2 of a two-step one)."""
    import torch
    from paper_2505_13097_amd import Stefan, variant_names
    g = Stefan(prob)
    names = variant_names(prob.q, prob.storage)
    for v in range(len(names)):
        g.set_variant(v)
        g.step(SWEEP_STEPS)
    torch.cuda.synchronize()
    g.close()
    return names


BATCH_PROFILE = "batch_step2_kernel_batch512_d2q5_f32.md"


def batch_kernels(vname, mode=0):
    """Trace names of the kernels one batched launch runs under variant
    vname (IREBM mode 0, EEBM mode 2), by role."""
    if "/t2" in vname:
        m = re.fullmatch(r"(\d+)x(\d+)/t2s?(/r\d+)?(/nt)?", vname)
        win, by = int(m.group(1)), int(m.group(2))
        base = f"batch_step2_kernel<5, float, {mode}, {by}, {win}"
        if "/t2s" in vname and mode != 2:
            return {"front": f"batch_front_kernel<5, float, {mode}>",
                    "quiet": base + ", 1>", "full": base + ", 2>"}
        return {"two-step": base + ", 0>"}
    m = re.fullmatch(r"(\d+)x(\d+)/npt(\d+).*", vname)
    npt = int(m.group(3))
    nt = "true" if "/nt" in vname else "false"
    return {"one-step": f"batch_step_kernel<5, float, {npt}, {mode}, {nt}>"}


def batch_walls(c, short, bkern):
    """Wall time (us) of each batched launch in a kernel trace: from the
    first start to the last end of the launch's kernels (one of each role
    per launch, in order)."""
    rows = c.execute("select name, start, end from kernels "
                     "order by start").fetchall()
    per = {role: [(s_, e) for n, s_, e in rows if short(n) == k]
           for role, k in bkern.items()}
    n = min(len(v) for v in per.values())
    return [(max(v[i][1] for v in per.values()) -
             min(v[i][0] for v in per.values())) / 1000.0 for i in range(n)]


def summarize_profiles(run, args):
    """Write the profiles/ summaries from the rocprofv3 databases of a
    GPU run: run/prof_all (kernel trace of the bench with a fixed plain
    variant and batch schedule), run/pmc_fetch and run/pmc_write (one
    counter each, bench --traffic-sweep)."""
    import collections
    import sqlite3
    import synth
    from paper_2505_13097_amd import variant_names

    import re

    def short(n):
        n = n.replace("(anonymous namespace)::", "").replace("irebm::", "")
        return n.split("(")[0].replace("void ", "")

    def step_kernel_of(k, mode):
        """k is a single-lattice step kernel of this lattice in node-update
        mode `mode` (0: IREBM safeguarded Newton, 2: EEBM)."""
        return re.match(rf"(step2_kernel<{prob.q}, float, {mode},|"
                        rf"step_kernel<{prob.q}, float, \d, {mode},)", k)

    def db(sub):
        d = os.path.join(run, sub)
        f = [x for x in os.listdir(d) if x.endswith("_results.db")]
        return sqlite3.connect(os.path.join(d, f[0]))

    prob = workload(args.workload)
    names = variant_names(prob.q, prob.storage)
    bnames = variant_names(5, "f32")
    V, BV, BB = args.variant, args.batch_variant, args.batch_bpc
    vname, bvname = names[V], bnames[BV]
    spl = steps_per_launch(vname)
    launches = args.steps // spl

    c = db("prof_all")
    trace = [(short(r[0]), r[1], r[2], r[3], r[4]) for r in c.execute(
        "select name, total_calls, total_duration, average, percentage "
        "from top_kernels")]
    by = collections.defaultdict(list)
    for name, d in c.execute("select name, duration from kernels "
                             "order by dispatch_id"):
        by[short(name)].append(d / 1000.0)          # ns -> us
    kname = "step2_kernel" if spl == 2 else "step_kernel"
    step_us = by[[k for k in by if step_kernel_of(k, 0) and
                  k.startswith(kname + "<")][0]]
    # the timed launches are the last ones of the step kernel
    step_avg = sum(step_us[-launches:]) / launches
    eebm_k = [k for k in by if step_kernel_of(k, 2) and
              k.startswith(kname + "<")]
    eebm_avg = (sum(by[eebm_k[0]][-launches:]) / launches
                if eebm_k and len(by[eebm_k[0]]) >= launches else None)
    bkern = batch_kernels(bvname)
    blaunch = args.batch_steps // steps_per_launch(bvname)
    bwall = batch_walls(c, short, bkern)[-blaunch:]
    bat_avg = sum(bwall) / len(bwall)          # wall time per launch
    bk_avg = {role: sum(by[k][-blaunch:]) / blaunch
              for role, k in bkern.items() if by.get(k)}

    def counters(sub, cn):
        rows = db(sub).execute(
            "select kernel_name, value from counters_collection where "
            "counter_name=? order by dispatch_id", (cn,)).fetchall()
        return [(short(k), v) for k, v in rows]
    F = counters("pmc_fetch", "FETCH_SIZE")
    W = counters("pmc_write", "WRITE_SIZE")
    gib_kib = 1024.0 * 1024.0
    copy_f = max(v for k, v in F if "copyBuffer" in k)
    copy_w = max(v for k, v in W if "copyBuffer" in k)
    fs, ws = gib_kib / copy_f, gib_kib / copy_w
    def is_step(k):
        return step_kernel_of(k, 0) is not None
    sf = [v for k, v in F if is_step(k)]
    sw = [v for k, v in W if is_step(k)]
    counts = [SWEEP_STEPS // steps_per_launch(nm) for nm in names]
    if len(sf) != sum(counts) or len(sw) != sum(counts):
        raise SystemExit(f"expected {sum(counts)} step-kernel dispatches, "
                         f"found {len(sf)} / {len(sw)}")
    alg = prob.nodes * bytes_per_node(prob)      # per lattice update
    per_var = {}
    o = 0
    for nm, n in zip(names, counts):
        fk = sum(sf[o:o + n]) / n
        wk = sum(sw[o:o + n]) / n
        o += n
        b = fk * 1024 * fs + wk * 1024 * ws
        per_var[nm] = {"steps_per_launch": steps_per_launch(nm),
                       "fetch_kib_per_dispatch": round(fk, 1),
                       "write_kib_per_dispatch": round(wk, 1),
                       "bytes_per_launch": round(b),
                       "bytes_per_lattice_update": round(
                           b / prob.nodes / steps_per_launch(nm), 3),
                       "ratio_to_algorithmic": round(
                           b / (alg * steps_per_launch(nm)), 4)}
    # counters of the batch's last launch in the sweep (IREBM comes first)
    def last_launch(C):
        out = {}
        for role, k in bkern.items():
            vs = [v for kk, v in C if kk == k]
            if vs:
                out[role] = vs[-1]
        return out
    bF, bW = last_launch(F), last_launch(W)
    bf, bw = sum(bF.values()), sum(bW.values())
    bprobs = synth.batch_table(count=args.batch_count, nsteps=args.batch_steps)
    bnodes = sum(p.nodes for p in bprobs)
    bspl = steps_per_launch(bvname)
    balg = bnodes * 40 * bspl
    bfb, bwb = bf * 1024 * fs, bw * 1024 * ws
    src = kernel_source_hash()

    trace_cmd = (f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof_all -o all"
                 f" -- python bench.py --steps {args.steps} --warmup 5 --variant {V}"
                 f" --no-cpu-baseline --forms batched,adjoint,eebm"
                 f" --batch-steps {args.batch_steps}"
                 f" --batch-variant {BV} --batch-bpc {BB}")
    pmc_cmd = ("rocprofv3 --pmc {C} -d gpurun_out/{D} -o {O} -- python bench.py"
               f" --traffic-sweep --batch-steps 4 --batch-variant {BV}"
               f" --batch-bpc {BB}")
    out = os.path.join(ROOT, "profiles")
    cav = step_avg
    lines = [f"# step_kernel — {prob.nx} x {prob.ny} D2Q{prob.q} {args.workload}, "
             f"FP32 populations (variant {vname})", "",
             "Kernel trace (rocprofv3 on MI355X; run from /tmp with TMPDIR=/tmp,",
             "paths absolute; summary written by bench.py --summarize-profiles):",
             "", "    " + trace_cmd, "",
             "| kernel | calls | total us | average us | % |",
             "|---|---|---|---|---|"]
    for r in trace[:16]:
        lines.append(f"| {r[0]} | {r[1]} | {r[2]:.0f} | {r[3]:.1f} | {r[4]:.2f} |")
    lines += ["", f"The {launches} timed launches of the step kernel "
              f"({spl} step(s) each) average {cav:.1f} us (bench.py measures the "
              "same launches with HIP events);",
              f"algorithmic bytes per launch {alg * spl / 1e9:.4f} GB ({prob.nodes:,} "
              f"nodes x {bytes_per_node(prob)} B x {spl} step(s)) -> "
              f"{alg * spl / (cav * 1e-6) / 1e9:.0f} GB/s.",
              "", "HBM traffic per launch of every variant (two counter runs, one "
              "counter each):", "", "    " + pmc_cmd.format(
                  C="FETCH_SIZE", D="pmc_fetch", O="fetch"),
              "    " + pmc_cmd.format(C="WRITE_SIZE", D="pmc_write", O="write"), "",
              f"Counter scale from a 1 GiB hipMemcpy D2D in the same runs: "
              f"FETCH_SIZE reads {copy_f:.0f} KiB (x{fs:.4f}), WRITE_SIZE "
              f"{copy_w:.0f} KiB (x{ws:.4f}).", "",
              "| variant | steps/launch | FETCH KiB | WRITE KiB | bytes/launch | "
              "B per lattice update | / algorithmic |",
              "|---|---|---|---|---|---|---|"]
    for nm, r in per_var.items():
        lines.append(f"| {nm} | {r['steps_per_launch']} | "
                     f"{r['fetch_kib_per_dispatch']:.0f} | "
                     f"{r['write_kib_per_dispatch']:.0f} | "
                     f"{r['bytes_per_launch'] / 1e9:.4f} GB | "
                     f"{r['bytes_per_lattice_update']:.2f} | "
                     f"{r['ratio_to_algorithmic']:.4f} |")
    t = per_var[vname]["bytes_per_launch"]
    lines += ["", f"Timed variant {vname}: {t / 1e9:.4f} GB per launch, "
              f"measured HBM rate {t / (cav * 1e-6) / 1e9:.0f} GB/s.",
              f"Kernel sources sha256 {src}.", ""]
    fn = f"step_kernel_{args.workload}{prob.nx}_d2q{prob.q}_f32.md"
    with open(os.path.join(out, fn), "w") as f:
        f.write("\n".join(lines))
    if eebm_avg is not None:
        fe = f"step_kernel_{args.workload}{prob.nx}_d2q{prob.q}_f32_eebm.md"
        with open(os.path.join(out, fe), "w") as f:
            f.write("\n".join([
                f"# {eebm_k[0]} — {prob.nx} x {prob.ny} D2Q{prob.q} "
                f"{args.workload}, explicit scheme (Algorithm 2), FP32 "
                f"populations (variant "
                f"{DEFAULT_VARIANTS.get(args.workload + '_eebm', vname)})", "",
                f"Same kernel trace as {fn} (the bench's eebm form, same "
                "step count).", "",
                f"The {launches} timed launches ({spl} step(s) each) average "
                f"{eebm_avg:.1f} us, against {cav:.1f} us for the IREBM "
                f"kernel (time ratio IREBM/EEBM {cav / eebm_avg:.3f}); "
                f"algorithmic bytes per launch {alg * spl / 1e9:.4f} GB -> "
                f"{alg * spl / (eebm_avg * 1e-6) / 1e9:.0f} GB/s.", ""]))
    blines = [
        f"# Batched form — {args.batch_count} D2Q5 instances (64^2 ... "
        f"1024^2), FP32, variant {bvname} (blocks per CU {BB})", "",
        f"Same kernel trace as {fn} (the bench's batched form:",
        f"{args.batch_steps} steps replayed from hipGraphs of 100 steps).", ""]
    if "front" in bkern:
        blines += [
            "Split two-step schedule, per launch of two steps: the front "
            "strips (batch_front_kernel, on a stream of its own) beside the "
            "quiet pass (batch_step2_kernel<..., 1>), then the full pass over "
            "flagged items (batch_step2_kernel<..., 2>).", ""]
    blines += ["| kernel | role | average us per launch |", "|---|---|---|"]
    for role, k in bkern.items():
        if role in bk_avg:
            blines.append(f"| {k} | {role} | {bk_avg[role]:.1f} |")
    blines += [
        "", f"Wall time per launch (first kernel start to last kernel end, "
        f"from the trace's timestamps), average over the {len(bwall)} timed "
        f"launches: {bat_avg:.1f} us ({bat_avg / bspl:.1f} us per step); "
        f"{bnodes:,} nodes x 40 B x {bspl} step(s) = {balg / 1e9:.3f} GB "
        f"algorithmic per launch -> {balg / (bat_avg * 1e-6) / 1e9:.0f} GB/s.",
        "", "| kernel | FETCH KiB | WRITE KiB | bytes |", "|---|---|---|---|"]
    for role, k in bkern.items():
        if role in bF and role in bW:
            blines.append(f"| {k} | {bF[role]:.0f} | {bW[role]:.0f} | "
                          f"{(bF[role] * fs + bW[role] * ws) * 1024 / 1e9:.4f}"
                          " GB |")
    blines += ["", f"Counter scale as above (FETCH_SIZE x{fs:.4f}, WRITE_SIZE "
               f"x{ws:.4f}); total {(bfb + bwb) / 1e9:.4f} GB per launch "
               f"({(bfb + bwb) / balg:.4f}x the algorithmic bytes).", ""]
    with open(os.path.join(out, BATCH_PROFILE), "w") as f:
        f.write("\n".join(blines))
    adj = [r for r in trace if "adj_" in r[0] or "front_vjp" in r[0] or
           "init_term" in r[0]]
    with open(os.path.join(out, "adjoint_kernels_adjoint512_d2q5_f32.md"), "w") as f:
        f.write("\n".join(
            ["# Reverse-mode kernels — 512 x 512 D2Q5, FP32 states, FP64 adjoint "
             "arrays, 4096 steps, checkpoints every 64", "",
             f"Same kernel trace as {fn} (the bench's adjoint form:",
             "forward tape, then the reverse sweep with segment recompute).", "",
             "| kernel | calls | total us | average us |", "|---|---|---|---|"] +
            [f"| {r[0]} | {r[1]} | {r[2]:.0f} | {r[3]:.2f} |" for r in adj] + [""]))
    with open(TRAFFIC_JSON, "w") as f:
        json.dump({"kernel": "step_kernel / step2_kernel", "workload": prob.name,
                   "sources_sha256": src, "fetch_scale": fs, "write_scale": ws,
                   "algorithmic_bytes_per_launch": alg, "variants": per_var,
                   "source": "profiles/" + fn}, f, indent=1)
    print(f"wrote profiles/{fn}, batch and adjoint summaries, "
          f"{os.path.relpath(TRAFFIC_JSON, ROOT)}")
    if os.path.isdir(os.path.join(run, "pmc_sq")):
        summarize_sq(run, args, db, short)


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
               "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES")


def summarize_sq(run, args, db, short):
    """profiles/ summary of the SQ counter run (run/pmc_sq, bench
    --traffic-sweep): instructions and wave cycles per dispatch of the
    batched kernel in IREBM and EEBM, and of the timed cavity kernel."""
    import collections
    from paper_2505_13097_amd import variant_names
    rows = db("pmc_sq").execute(
        "select dispatch_id, kernel_name, counter_name, value from "
        "counters_collection order by dispatch_id").fetchall()
    per = collections.OrderedDict()
    for d, k, cn, v in rows:
        per.setdefault((d, short(k)), {})[cn] = v
    bnames = variant_names(5, "f32")
    bv = bnames[args.batch_variant]
    kinds = [(f"batched IREBM, {role}", k)
             for role, k in batch_kernels(bv, 0).items()]
    kinds += [(f"batched EEBM, {role}", k)
              for role, k in batch_kernels(bv, 2).items()]
    lines = ["# SQ counters — batched form (512 D2Q5 instances, FP32, variant "
             f"{bv}) in IREBM and EEBM", "",
             "    rocprofv3 --pmc " + " ".join(SQ_COUNTERS) +
             " -d gpurun_out/pmc_sq -o sq -- python bench.py --traffic-sweep"
             f" --batch-steps 4 --batch-variant {args.batch_variant}"
             f" --batch-bpc {args.batch_bpc}", "",
             "Averages per dispatch (the sweep's 4 steps of each).", "",
             "| kernel | dispatches | " + " | ".join(SQ_COUNTERS) +
             " | VALU per wave | wave cycles per wave |",
             "|---|---|" + "---|" * (len(SQ_COUNTERS) + 2)]
    avg = {}
    for label, pre in kinds:
        ds = [c for (d, k), c in per.items() if k == pre]
        if not ds:
            continue
        a = {cn: sum(c.get(cn, 0.0) for c in ds) / len(ds)
             for cn in SQ_COUNTERS}
        avg[label] = a
        lines.append(f"| {label} | {len(ds)} | " +
                     " | ".join(f"{a[cn]:.4g}" for cn in SQ_COUNTERS) +
                     f" | {a['SQ_INSTS_VALU'] / max(a['SQ_WAVES'], 1):.1f} |"
                     f" {a['SQ_WAVE_CYCLES'] / max(a['SQ_WAVES'], 1):.0f} |")
    irebm = [a for lab, a in avg.items() if lab.startswith("batched IREBM")]
    eebm = [a for lab, a in avg.items() if lab.startswith("batched EEBM")]
    if irebm and eebm:
        tot = {cn: (sum(a[cn] for a in irebm), sum(a[cn] for a in eebm))
               for cn in SQ_COUNTERS}
        lines += ["", "IREBM (all kernels of a launch) / EEBM: VALU "
                  "instructions "
                  f"{tot['SQ_INSTS_VALU'][0] / tot['SQ_INSTS_VALU'][1]:.2f}x,"
                  " wave cycles "
                  f"{tot['SQ_WAVE_CYCLES'][0] / tot['SQ_WAVE_CYCLES'][1]:.2f}x,"
                  " busy cycles "
                  f"{tot['SQ_BUSY_CYCLES'][0] / tot['SQ_BUSY_CYCLES'][1]:.2f}x."]
    lines.append("")
    fn = "batch_step2_kernel_sq_counters_batch512_d2q5_f32.md"
    with open(os.path.join(ROOT, "profiles", fn), "w") as f:
        f.write("\n".join(lines))
    print(f"wrote profiles/{fn}")


RDREQ_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_128B_sum",
                  "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_32B_sum")


def summarize_rdreq(run):
    """profiles/ summary of the read requests by size (run/pmc_rdreq, bench
    --traffic-sweep): bytes read from HBM as 128 x (128-byte requests) +
    64 x (64-byte) + 32 x (32-byte), per dispatch of each kernel, beside
    FETCH_SIZE of the same kernels (run/pmc_fetch) and the 1 GiB copy.
    This counts the bytes with no calibration; FETCH_SIZE, whose formula
    counts a 128-byte request as 64 bytes, is scaled by the copy."""
    import collections
    import sqlite3

    def db(sub):
        d = os.path.join(run, sub)
        f = [x for x in os.listdir(d) if x.endswith("_results.db")]
        return sqlite3.connect(os.path.join(d, f[0]))

    def short(n):
        n = n.replace("(anonymous namespace)::", "").replace("irebm::", "")
        return n.split("(")[0].replace("void ", "")

    per = collections.OrderedDict()
    for d, k, cn, v in db("pmc_rdreq").execute(
            "select dispatch_id, kernel_name, counter_name, value from "
            "counters_collection order by dispatch_id"):
        e = per.setdefault((d, short(k)), {})
        e[cn] = e.get(cn, 0.0) + v
    fetch = collections.defaultdict(list)
    for k, v in db("pmc_fetch").execute(
            "select kernel_name, value from counters_collection where "
            "counter_name='FETCH_SIZE' order by dispatch_id"):
        fetch[short(k)].append(v)
    by = collections.OrderedDict()
    for (d, k), c in per.items():
        b = (128 * c.get(RDREQ_COUNTERS[1], 0) + 64 * c.get(RDREQ_COUNTERS[2], 0)
             + 32 * c.get(RDREQ_COUNTERS[3], 0))
        other = c.get(RDREQ_COUNTERS[0], 0) - sum(
            c.get(x, 0) for x in RDREQ_COUNTERS[1:])
        by.setdefault(k, []).append((b, c.get(RDREQ_COUNTERS[1], 0) /
                                     max(c.get(RDREQ_COUNTERS[0], 0), 1),
                                     other))
    copy_kib = max(fetch["__amd_rocclr_copyBuffer"])
    lines = ["# HBM read bytes by request size — the counter sweep of the "
             "2D step kernels and the batched form", "",
             "    rocprofv3 --pmc " + " ".join(RDREQ_COUNTERS) +
             " -d gpurun_out/pmc_rdreq -o rdreq -- python bench.py "
             "--traffic-sweep --batch-steps 4 --batch-variant 35 "
             "--batch-bpc 0", "",
             "Bytes read = 128 x (128-byte requests) + 64 x (64-byte) + 32 "
             "x (32-byte), no calibration; beside it FETCH_SIZE (same "
             "sweep, its own run) scaled by the 1 GiB copy "
             f"(x{1048576.0 / copy_kib:.4f}).", "",
             "| kernel | dispatches | GB read by request size | 128-byte "
             "share | other requests | FETCH_SIZE x scale, GB | ratio |",
             "|---|---|---|---|---|---|---|"]
    for k, rs in by.items():
        if not (k.startswith("step") or k.startswith("batch") or
                "copyBuffer" in k):
            continue
        b = sum(r[0] for r in rs) / len(rs)
        if b < 1e6:
            continue
        share = sum(r[1] for r in rs) / len(rs)
        oth = sum(r[2] for r in rs) / len(rs)
        fs = fetch.get(k)
        fb = (sum(fs) / len(fs)) * 1024 * 1048576.0 / copy_kib if fs else None
        lines.append(f"| {k} | {len(rs)} | {b / 1e9:.4f} | {share:.4f} | "
                     f"{oth:.0f} | " + (f"{fb / 1e9:.4f} | {fb / b:.4f} |"
                                        if fb else "— | — |"))
    lines.append("")
    fn = "hbm_read_requests_by_size_cavity8192_batch512.md"
    with open(os.path.join(ROOT, "profiles", fn), "w") as f:
        f.write("\n".join(lines))
    print(f"wrote profiles/{fn}")


def cpu_baseline(prob, steps=1, threads=None):
    """The oracle, as it stands, on `steps` steps of the same lattice from
    the same initial state: once on one thread, then on every core this
    process may use (at most 16), the lattice cut into row strips with
    `steps` halo rows each, run side by side (the oracle's C code runs
    outside the GIL).  The strips' own rows must equal the single-thread
    result bit for bit."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle as O
    model, ncores, nproc = host_cpu()
    threads = min(16, ncores) if threads is None else threads
    threads = max(1, min(threads, prob.ny // max(1, 2 * steps)))
    f = O.init(prob, prob.T0)
    t0 = time.perf_counter()
    f1, _ = O.run(prob, f, steps)
    dt1 = time.perf_counter() - t0
    T1 = O.temperature(prob, f1)
    del f, f1
    cuts = np.linspace(0, prob.ny, threads + 1).astype(int)

    def strip(k):
        sub, a = strip_problem(prob, cuts[k], cuts[k + 1], steps)
        g, _ = O.run(sub, O.init(sub, sub.T0), steps)
        T = O.temperature(sub, g)
        return T[cuts[k] - a:cuts[k + 1] - a]

    # the parallel leg times the steps and the strips' set-up alike
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(strip, range(threads)))
    dtn = time.perf_counter() - t0
    same = all(np.array_equal(parts[k], T1[cuts[k]:cuts[k + 1]])
               for k in range(threads))
    return {"value": round(prob.nodes * steps / dtn / 1e6, 2),
            "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} step(s) of the full {prob.nx}x{prob.ny} "
                      f"{prob.name} lattice from its initial state: "
                      f"{threads} row strips ({steps} halo rows each) on "
                      f"{threads} threads, {dtn:.1f} s; one thread on the "
                      f"whole lattice {dt1:.1f} s",
            "single_thread_mlups": round(prob.nodes * steps / dt1 / 1e6, 2),
            "strips_equal_single_thread": bool(same),
            "cpu_model": model, "nproc": nproc, "usable_cores": ncores}


def copy_gbps(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (torch's copy kernel) on the current
    stream, timed with HIP events: 2 nbytes per copy (read and write)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def host_cpu():
    """CPU model (lscpu) and the cores this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True,
                             timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def strip_problem(prob, y0, y1, halo):
    """rows [y0, y1) of prob with `halo` rows around them as a lattice of
    their own (cut sides bounce back; after k <= halo steps the own rows
    equal those of the whole lattice)"""
    import numpy as np
    T0 = np.broadcast_to(-0.5 if prob.T0 is None else prob.T0,
                         (prob.ny, prob.nx))
    if prob.bc[2] == "periodic" and (y0 > 0 or y1 < prob.ny):
        # the halo rows wrap around the periodic axis; both cut sides
        # bounce back
        a, b = y0 - halo, y1 + halo
        rows = np.arange(a, b) % prob.ny
        return prob.with_(ny=b - a, bc=prob.bc[:2] + ("bounceback",) * 2,
                          T0=T0[rows], dx=prob.dx), a
    a, b = max(0, y0 - halo), min(prob.ny, y1 + halo)
    bc = (prob.bc[0], prob.bc[1],
          prob.bc[2] if a == 0 else "bounceback",
          prob.bc[3] if b == prob.ny else "bounceback")
    return prob.with_(ny=b - a, bc=bc, T0=T0[a:b], dx=prob.dx), a


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cavity",
                    choices=["cavity", "planar", "stefan1d"])
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="let the autotuners pick the kernel variants "
                         "(default: the fixed variants of DEFAULT_VARIANTS)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="the default; kept for older profile commands")
    ap.add_argument("--forms",
                    default="batched,adjoint,eebm,planar,cube3d",
                    help="comma list of extra forms to time: batched, "
                         "adjoint, eebm, planar, cube3d; and the paper's "
                         "experiments: freezing, paper1d, freezing3d")
    ap.add_argument("--cube3d-only", action="store_true",
                    help="time the 3D form alone (profile runs)")
    ap.add_argument("--cube3d-n", type=int, default=CUBE3D_N)
    ap.add_argument("--steps3d", type=int, default=50)
    ap.add_argument("--variant3d", type=int, default=-1)
    ap.add_argument("--traffic-sweep-3d", action="store_true",
                    help="counter runs of the 3D kernel: 1 GiB copy, every "
                         f"3D variant for {SWEEP_STEPS} steps; no timing")
    ap.add_argument("--summarize-profiles3", metavar="RUN_DIR",
                    help="write the 3D profiles/ summary (CPU only; "
                         "--variant3d and --steps3d as in the trace run)")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-variant", type=int, default=-1)
    ap.add_argument("--batch-bpc", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter scale)")
    ap.add_argument("--traffic-sweep", action="store_true",
                    help="counter runs: 1 GiB copy, every variant for "
                         f"{SWEEP_STEPS} steps, the batched form; no timing")
    ap.add_argument("--summarize-rdreq", metavar="RUN_DIR",
                    help="write the read-requests-by-size summary from "
                         "RUN_DIR/pmc_rdreq and RUN_DIR/pmc_fetch (CPU only)")
    ap.add_argument("--summarize-profiles", metavar="RUN_DIR",
                    help="write profiles/ from the rocprofv3 output of a run "
                         "(CPU only; --variant, --batch-variant, --batch-bpc, "
                         "--steps and --batch-steps as in the trace run)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args)
        return
    if args.summarize_rdreq:
        summarize_rdreq(args.summarize_rdreq)
        return
    if args.summarize_profiles3:
        summarize_profiles3(args.summarize_profiles3, args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; "
                          "--gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth  # noqa: F401
    from paper_2505_13097_amd import variant_names
    torch.cuda.set_device(0)

    if args.cube3d_only:
        r = time_cube3d(args.steps3d, 5, args.autotune,
                        args.variant3d, args.cube3d_n)
        print(json.dumps({"cube3d": r}), flush=True)
        return
    if args.traffic_sweep_3d:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        del a, b
        traffic_sweep3(args.cube3d_n)
        print(json.dumps({"traffic_sweep_3d": args.cube3d_n,
                          "steps_each": SWEEP_STEPS}), flush=True)
        return

    prob = workload(args.workload)
    if args.traffic_sweep:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        del a, b
        names = traffic_sweep(prob)
        import synth as S
        probs = S.batch_table(count=args.batch_count, nsteps=args.batch_steps)
        # the batched form in IREBM, then in EEBM (instruction counts of the
        # Newton path against the no-Newton scheme in the SQ counter runs)
        for pr in (probs, [p.with_(scheme="eebm") for p in probs]):
            time_batched(pr, args.batch_steps, 0, autotune=False,
                         graph_steps=0, variant=args.batch_variant,
                         bpc=args.batch_bpc)
        print(json.dumps({"traffic_sweep": prob.name, "variants": names,
                          "steps_each": SWEEP_STEPS}), flush=True)
        return
    print(f"[bench] workload {prob.name}: {prob.nx}x{prob.ny} D{prob.dim}Q{prob.q} "
          f"steps {args.steps} warmup {args.warmup}", file=sys.stderr,
          flush=True)
    if args.variant < 0 and not args.autotune:
        args.variant = variant_id(prob.q, prob.storage,
                                  DEFAULT_VARIANTS[args.workload])
    r = time_plain(prob, args.steps, args.warmup, args.variant,
                   autotune=args.autotune)
    print(f"[bench] timed region done: {r['gpu_ms']:.1f} ms", file=sys.stderr,
          flush=True)
    ms_per_step = r["wall_s"] * 1e3 / args.steps
    mlups = prob.nodes * args.steps / r["wall_s"] / 1e6
    v = r["variant"] if r["variant"] >= 0 else (0 if prob.q == 3 else 3)
    vname = variant_names(prob.q, prob.storage)[v]
    resident = vname.startswith("resident")
    spl = steps_per_launch(vname, args.steps)
    if args.steps % 2 and spl == 2:
        raise SystemExit("--steps must be even for a two-step variant")
    launches = -(-args.steps // spl)
    launch_ms = r["gpu_ms"] / launches
    bpn = bytes_per_node(prob)
    # algorithmic bytes per launch: 2 q s per lattice update, times the
    # updates one launch performs (the same rate over the whole run)
    achieved = prob.nodes * bpn * args.steps / (r["gpu_ms"] * 1e-3) / 1e9

    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

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
            "kernel": ("resident1d_kernel" if resident else
                       "step2_kernel" if spl == 2 else "step_kernel"),
            "steps_per_launch": spl,
            "bytes_per_lattice_update": bpn,
            "avg_launch_us": round(launch_ms * 1e3, 2),
        },
        "newton": {
            "max_it": r["stats"]["max_newton_it"],
            "nonconverged": r["stats"]["nonconverged"],
            "max_residual": r["stats"]["max_residual"],
        },
    }
    traffic = out["roofline"]["traffic"]
    if traffic:
        # what HBM actually moved: the counter bytes of one launch of this
        # variant over the same launch time (a two-step launch moves about
        # half of its algorithmic bytes)
        dram = traffic / (launch_ms * 1e-3) / 1e9
        out["roofline"]["dram_gbps"] = round(dram, 1)
        out["roofline"]["dram_frac"] = round(dram / HBM_PEAK_GBPS, 4)
    print("[bench] copy kernel", file=sys.stderr, flush=True)
    out["roofline"]["copy_kernel_gbps"] = copy_gbps()
    if resident:
        out["roofline"]["note"] = (
            "the state stays in LDS between steps: the rate is the "
            "metric's algorithmic bytes, HBM is touched once per launch; "
            "the per-step latency of one workgroup bounds this kernel")
    forms = {}
    if "batched" in args.forms.split(","):
        import synth as S
        print(f"[bench] batched form: {args.batch_count} instances, "
              f"{args.batch_steps} steps", file=sys.stderr, flush=True)
        probs = S.batch_table(count=args.batch_count, nsteps=args.batch_steps)
        forms["batched"] = time_batched(
            probs, args.batch_steps, 10, autotune=args.autotune,
            variant=args.batch_variant, bpc=args.batch_bpc)
        print("[bench] batched done", file=sys.stderr, flush=True)
    if "adjoint" in args.forms.split(","):
        import synth as S
        print("[bench] adjoint form", file=sys.stderr, flush=True)
        adj = S.adjoint_2d()
        forms["adjoint"] = time_adjoint(adj, 64, args.autotune)
        # every state kept (no recompute): 4097 states of 5.2 MB fit in HBM
        forms["adjoint_all_states"] = time_adjoint(adj, 1, args.autotune)
        print("[bench] adjoint done", file=sys.stderr, flush=True)
    if "eebm" in args.forms.split(","):
        print("[bench] eebm form", file=sys.stderr, flush=True)
        forms["eebm"] = time_eebm(prob, args.steps, args.warmup,
                                  args.autotune, ms_per_step,
                                  key=args.workload)
        print("[bench] eebm done", file=sys.stderr, flush=True)
    if "planar" in args.forms.split(","):
        print("[bench] planar form", file=sys.stderr, flush=True)
        forms["planar"] = time_planar(autotune=args.autotune)
        print("[bench] planar done", file=sys.stderr, flush=True)
    if "freezing" in args.forms.split(","):
        print("[bench] freezing form", file=sys.stderr, flush=True)
        forms["freezing"] = time_freezing()
        print("[bench] freezing done", file=sys.stderr, flush=True)
    if "paper1d" in args.forms.split(","):
        print("[bench] paper1d form", file=sys.stderr, flush=True)
        forms["paper1d"] = time_paper1d()
        print("[bench] paper1d done", file=sys.stderr, flush=True)
    if "freezing3d" in args.forms.split(","):
        print("[bench] freezing3d form", file=sys.stderr, flush=True)
        forms["freezing3d"] = time_freezing3d()
        print("[bench] freezing3d done", file=sys.stderr, flush=True)
    if "cube3d" in args.forms.split(","):
        print("[bench] cube3d form", file=sys.stderr, flush=True)
        forms["cube3d"] = time_cube3d(
            args.steps3d, 5, args.autotune, args.variant3d,
            args.cube3d_n)
        print("[bench] cube3d done", file=sys.stderr, flush=True)
    if forms:
        out["forms"] = forms
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)...", file=sys.stderr, flush=True)
        # about 10-30 s of oracle work: one thread, then all usable cores
        out["cpu_baseline"] = cpu_baseline(prob, 3 if prob.nodes > 1e6 else 200)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
