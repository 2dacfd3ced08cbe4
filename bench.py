#!/usr/bin/env python3
"""Throughput of the CV-MC field transfer hot path on one MI355X.

One step is one whole transfer with the inputs resident in HBM:
  ft_sample_points   (node queries + N Philox samples per target element)
  ft_source_eval     (the built-in P1 source answers every point query)
  ft_consume_queries (residual, per-element Monte Carlo sums, node assembly)
  ft_project         (b = alpha M g + b_res, Jacobi-PCG to rtol, conservation report)
Setup (mass matrix, incidence, source bins) is timed separately: it is paid
once per mesh pair.

Prints one JSON line.  Per-phase times come from HIP events recorded on the
stream the library launches on; the dominant kernel's achieved bandwidth is
its algorithmic bytes divided by its average event-measured duration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs at 2.4 GHz, one full-rate wave64 vector
# instruction per SIMD every 4 cycles (16 lanes per cycle) = 614.4e9 wave64
# instructions per second (64 lanes each: 3.93e13 lane operations/s)
VALU_PEAK_G = 256 * 4 * 2.4 / 4
METRIC = "target elements/s and point queries/s per transfer; % HBM roofline vs FP64"
PRECISIONS = {"f64": "FT_F64", "f32": "FT_F32", "split-f16": "FT_SPLIT_F16", "split-bf16": "FT_SPLIT_BF16"}
DTYPES = {"f64": "f64", "f32": "f32", "split-f16": "f32+f16x2", "split-bf16": "f32+bf16x2"}

# device sources each timed kernel is compiled from: a counter record taken on
# other sources no longer describes the kernel and is not reported
KERNEL_SOURCES = {
    "k_emit": ["mc.hip", "adaptive.h", "sampling.h", "common.h"],
    "k_src_eval": ["source.hip", "locate.h", "common.h"],
    "k_consume": ["mc.hip", "adaptive.h", "sampling.h", "common.h"],
    "k_consume_mfma": ["mc_mfma.hip", "sampling.h", "common.h"],
    "k_fused_p1": ["fused.hip", "fused.h", "adaptive.h", "locate.h", "sampling.h", "common.h"],
}
TRAFFIC_RECORDS = os.path.join(ROOT, "profiles", "hbm_traffic.md")
VALU_RECORDS = os.path.join(ROOT, "profiles", "valu_counts.md")
# kernels whose device sources define them (for the record digests)
KERNEL_SOURCES["k_src_eval_many"] = KERNEL_SOURCES["k_src_eval"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_mesh_bytes(dim, F, src):
    """The built-in source read once: element records (128 / 256 B), binary32
    boxes, bin lists; connectivity and nodal values only for F > 1 (one field's
    vertex values sit in the records)."""
    rec, box = (128, 32) if dim == 2 else (256, 48)
    b = src["E"] * (rec + box) + src["n_reg"] * 4 + src["nbins"] * 8
    if F > 1:
        b += src["E"] * (dim + 1) * 4 + src["n"] * F * 8
    return b


def algorithmic_bytes(phase, dim, E, n, N, F, p, src=None):
    """Compulsory HBM bytes of one launch of a phase: what it must read and write
    at least once (points, values, mesh data), not what its caches refetch."""
    Q = n + E * N
    if phase == "emit":
        # write d coordinates per query; read connectivity and vertex coordinates per element
        return Q * dim * p + E * ((dim + 1) * 4 + (dim + 1) * dim * 8) + n * dim * 8
    if phase == "eval":
        # read d coordinates and write F values per query; read the source mesh
        # (coordinates, connectivity, nodal values) once
        return Q * (dim + F) * p + src["n"] * dim * 8 + src["E"] * (dim + 1) * 4 + src["n"] * F * 8
    if phase == "fused":
        # per element: connectivity, vertex coordinates, control values, measure, beta; the source mesh once
        return E * ((dim + 1) * 4 + (dim + 1) * dim * 8 + (dim + 1) * F * 8 + 8 + (dim + 1) * F * 8) \
            + source_mesh_bytes(dim, F, src)
    if phase == "consume":
        # read F values per query; per element connectivity, measure and beta; node assembly
        return Q * F * p + E * ((dim + 1) * 4 + 8 + (dim + 1) * F * 8) + E * (dim + 1) * (4 + F * 8) + n * F * 16
    raise ValueError(phase)


_CPU = {}   # oracle state shared with the forked baseline workers


def _cpu_elements(job):
    """Oracle steps 3-5 (sample, query, residual element sums) for one run of elements."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cvmc

    start, count = job
    c = _CPU
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        els = np.arange(start, start + count)
        lam, X = cvmc.query_points(c["tc"], c["tconn"], c["N"], c["seed"], 0, els)
        y = np.atleast_2d(c["src"](X.reshape(-1, c["tc"].shape[1]))).reshape(c["F"], els.size, c["N"])
        cvmc.element_loads(c["tc"], c["tconn"], c["g"], y, lam, c["alpha"], els)
        return time.perf_counter() - t0


def _cpu_nodes(job):
    """Oracle step 1 (the control: the source at the target nodes) for a range of nodes."""
    from threadpoolctl import threadpool_limits

    start, count = job
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _CPU["src"](_CPU["tc"][start:start + count])
        return time.perf_counter() - t0


def _spread_runs(total, runs, length):
    """`runs` runs of `length` consecutive items spread evenly over [0, total)."""
    length = max(1, min(length, total // runs if total >= runs else total))
    starts = [int(round(k * (total - length) / max(1, runs - 1))) for k in range(runs)]
    return [(s_, length) for s_ in starts]


def cpu_baseline_child(args):
    """The oracle, as it stands, timed on this host for the whole transfer of a
    workload: steps 1 and 3-5 on bounded samples (one core, then every core of
    the process's share with one worker process per core), steps 2, 6 and 7 at
    full size (single-threaded numpy / scipy), scaled to the whole target.
    Setup (the source's search tree, the mass matrix) is excluded, like the
    GPU's setup.  Prints one JSON line."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cvmc, geometry
    from oracle.source import P1Source
    from workloads import configs

    w = configs.WORKLOADS[args.workload]
    tc, tconn = configs.build_mesh(w.target)
    sc, sconn = configs.build_mesh(w.source)
    svals = configs.source_nodal_values(w, sc)
    tconn = np.asarray(tconn, dtype=np.int64)
    src = P1Source(sc, sconn, svals)
    M = geometry.mass_matrix(tc, tconn)
    m = geometry.lumped_mass(tc, tconn)
    E, n, dim = tconn.shape[0], tc.shape[0], tc.shape[1]
    N, F = w.samples_per_elem, svals.shape[0] if svals.ndim == 2 else 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))   # the host share of one GPU
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    _CPU.update(tc=tc, tconn=tconn, src=src, N=N, F=F, seed=w.philox_seed, alpha=w.alpha)
    with threadpool_limits(limits=1):
        # step 1 on one core: a spread sample of the nodes
        node_jobs = _spread_runs(n, 8, max(1, min(n, 200_000) // 8))
        t_n1 = sum(_cpu_nodes(j) for j in node_jobs)
        n_done = sum(c for _, c in node_jobs)
        t_nodes_1 = t_n1 * n / n_done
        g = np.atleast_2d(src(tc))                       # the control for steps 2-5 (untimed)
        _CPU["g"] = g
        # steps 3-5 on one core: a pilot, then about 6 s of element runs
        pilot = _cpu_elements((E // 2, min(E, 200)))
        per_el = pilot / min(E, 200)
        e1 = int(max(64, min(E, 6.0 / per_el)))
        jobs1 = _spread_runs(E, 16, e1 // 16)
        t_e1 = sum(_cpu_elements(j) for j in jobs1)
        e_done1 = sum(c for _, c in jobs1)
        # steps 2, 6, 7 and the report at full size
        t0 = time.perf_counter()
        b_g = cvmc.control_load(tc, tconn, g, w.alpha)
        t_control = time.perf_counter() - t0
        beta = np.zeros((F, E, dim + 1))
        t0 = time.perf_counter()
        b = b_g + cvmc.assemble(tconn, beta, n)
        t_assemble = time.perf_counter() - t0
        t0 = time.perf_counter()
        x = cvmc.solve_mass(M, b, dim)
        cvmc.conservation_report(b, x, m)
        t_solve = time.perf_counter() - t0
    t_global = t_control + t_assemble + t_solve
    # steps 1 and 3-5 on every core of the share: one worker process per core
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_elements, [(0, 8)] * cores)        # warm the workers
        jobsc = _spread_runs(E, 4 * cores, max(1, int(3.0 / per_el) // 4))
        t0 = time.perf_counter()
        pool.map(_cpu_elements, jobsc, chunksize=1)
        t_ec = time.perf_counter() - t0
        e_donec = sum(c for _, c in jobsc)
        t0 = time.perf_counter()
        pool.map(_cpu_nodes, _spread_runs(n, 4 * cores, max(1, min(n, 400_000) // (4 * cores))), chunksize=1)
        t_nc = time.perf_counter() - t0
        n_donec = sum(c for _, c in _spread_runs(n, 4 * cores, max(1, min(n, 400_000) // (4 * cores))))
    t_nodes_c = t_nc * n / n_donec
    T1 = t_nodes_1 + t_e1 * E / e_done1 + t_global
    Tc = t_nodes_c + t_ec * E / e_donec + t_global
    out = {
        "value": E / Tc, "unit": "target elements/s", "cores": cores, "kind": "oracle",
        "sample": (f"whole transfer of {w.name} estimated from the oracle (numpy/scipy, untuned): steps 1 and "
                   f"3-5 timed on spread samples ({n_donec} nodes, {e_donec} of {E} elements x {N} samples on "
                   f"{cores} worker processes; {n_done} nodes and {e_done1} elements on 1 core) and scaled to the "
                   f"whole mesh, steps 2, 6, 7 and the report at full size ({t_global:.1f} s, single-threaded); "
                   f"setup excluded"),
        "seconds_per_transfer": Tc,
        "one_core": {"value": E / T1, "cores": 1, "seconds_per_transfer": T1},
        "phases_s": {"nodes": t_nodes_c, "elements": t_ec * E / e_donec, "control": t_control,
                     "assemble": t_assemble, "solve_and_report": t_solve},
        "host": {"cpu": model, "cores_used": cores, "cpu_count": os.cpu_count()},
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(w):
    """Run the oracle baseline in a child process (it uses no GPU) and return its dict."""
    import subprocess

    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--workload", w.name]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed ({r.returncode}): {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def sources_digest(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2603_00538_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    record of this kernel and workload, or None when there is none or it was
    taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_RECORDS):
        return None
    digest = sources_digest(kernel)
    with open(TRAFFIC_RECORDS) as fh:
        for line in fh:
            line = line.strip()
            if not line.startswith("record "):
                continue
            r = json.loads(line[len("record "):])
            if ((r["kernel"], r["workload"], r["precision"], r["sources"]) == (kernel, workload, precision, digest)
                    and "fetch_bytes" in r):
                return r["fetch_bytes"] + r["write_bytes"]
    return None


def measured_valu(kernel, workload, precision):
    """VALU wave64 instructions per launch from the committed rocprofv3
    SQ_INSTS_VALU record of this kernel and workload, or None when there is
    none or it was taken on other kernel sources."""
    if not os.path.exists(VALU_RECORDS):
        return None
    digest = sources_digest(kernel)
    with open(VALU_RECORDS) as fh:
        for line in fh:
            line = line.strip()
            if not line.startswith("record "):
                continue
            r = json.loads(line[len("record "):])
            if ((r["kernel"], r["workload"], r["precision"], r["sources"]) == (kernel, workload, precision, digest)
                    and "valu_insts" in r):
                return r
    return None


def kernel_roofline(kernel, workload, precision, abytes, avg_ms):
    """Roofline of one kernel: its algorithmic HBM bytes against 8 TB/s and, when
    a counter record exists, its VALU issue rate against 614.4e9 wave64
    instructions/s; the bound is whichever is nearer its peak.  Both use the
    live event-timed average duration."""
    sec = avg_ms * 1e-3
    hbm_ach = abytes / sec / 1e9
    hbm = {"bound": "hbm", "achieved": hbm_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_ach / HBM_PEAK_GBS,
           "algorithmic_bytes": abytes}
    traffic = measured_traffic(kernel, workload, precision)
    rec = measured_valu(kernel, workload, precision)
    alu = None
    if rec is not None:
        ach = rec["valu_insts"] / sec / 1e9
        alu = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_G, "unit": "G wave64 VALU instructions/s",
               "frac": ach / VALU_PEAK_G, "valu_insts": rec["valu_insts"]}
    main, other = (alu, hbm) if alu is not None and alu["frac"] > hbm["frac"] else (hbm, alu)
    out = dict(main)
    out["kernel"] = kernel
    out["traffic"] = traffic
    out["avg_ms"] = avg_ms
    if other is not None:
        out[other["bound"]] = {k: v for k, v in other.items() if k != "bound"}
    return out


def sequential_f64(T, w, tmesh, smesh, svals):
    """The comparator of the many-field form: F one-field FP64 transfers, one
    after another (each field's source set up untimed; emit, eval, consume and
    project timed with events)."""
    import numpy as np
    import torch

    from paper_2603_00538_amd import ft

    tc, tconn = tmesh
    sc, sconn = smesh
    n, E = tc.shape[0], tconn.shape[0]
    N, F, dim = w.samples_per_elem, svals.shape[0], tc.shape[1]
    Q = T.query_count(N)
    pts = torch.empty((dim, Q), dtype=torch.float64, device="cuda")
    vals = torch.empty((1, Q), dtype=torch.float64, device="cuda")
    x = torch.empty((1, n), dtype=torch.float64, device="cuda")
    total = 0.0
    iters = []
    for f in range(F):
        S1 = ft.Source(sc, sconn, np.ascontiguousarray(svals[f:f + 1]), bins=w.bins if any(w.bins) else None)
        cfg = ft.SampleCfg(N, 1, w.alpha, w.philox_seed, 0, ft.FT_F64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        T.sample_points(cfg, out=pts)
        S1.eval_query_list(pts, n, out=vals)
        T.consume(cfg, vals)
        res = T.project(1, rtol=w.rtol, max_iter=1000, x=x)
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
        iters.append(res.reports[0]["iters"])
        S1.close()
        if f % 16 == 15:
            log(f"sequential FP64 transfers: {f + 1}/{F}")
    return {"transfers": F, "ms_total": total, "value": E / (total * 1e-3), "unit": "target elements/s (all fields)",
            "cg_iters_max": int(max(iters))}


def bench_batch(args):
    """The uneven batch: 256 built-in-source transfers (mixed 2D/3D, 1e3-5e5
    elements, N in {32..256}) per ft_batch_run, captured as one graph."""
    import numpy as np
    import torch

    from paper_2603_00538_amd import ft
    from workloads import configs

    items = configs.batch_items()
    log(f"batch256: building {len(items)} mesh pairs")
    t0 = time.perf_counter()
    host = []
    for it in items:
        tc, tconn = it.target.build()
        sc, sconn = it.source.build()
        host.append((tc, tconn, sc, sconn, np.ascontiguousarray(it.field(np, sc))))
    log(f"meshes built in {time.perf_counter() - t0:.1f} s")
    torch.cuda.set_device(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    targets = [ft.Target(tc, tconn) for tc, tconn, _, _, _ in host]
    sources = [ft.Source(sc, sconn, sv) for _, _, sc, sconn, sv in host]
    prec = ft.FT_F32 if args.precision == "f32" else ft.FT_F64
    if args.precision not in ("f64", "f32"):
        raise SystemExit("batch256 runs the f64 and f32 forms")
    cfgs = [ft.SampleCfg(it.samples_per_elem, 1, 1.0, configs.BATCH_PHILOX_SEED, it.stream_id, prec)
            for it in items]
    B = ft.Batch(targets, sources, cfgs, graph=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tune = None
    if args.autotune != "off":
        # element variants and bin grids timed per kind of transfer (cached in a
        # JSON file when --tune-cache names one)
        t0 = time.perf_counter()
        n_tuned = B.autotune(args.tune_cache or None)
        torch.cuda.synchronize()
        hist = {}
        for k in range(len(items)):
            g_, p_ = B.variant(k)
            hist[f"G{g_}xP{p_}"] = hist.get(f"G{g_}xP{p_}", 0) + 1
        tune = {"kinds_timed": n_tuned, "ms": (time.perf_counter() - t0) * 1e3, "variants": hist,
                "cache": args.tune_cache or None}
        log(f"batch autotune: {n_tuned} kinds timed in {tune['ms']:.0f} ms; variants {hist}")
    E_tot = int(sum(t.n_elems for t in targets))
    S_tot = int(sum(t.n_elems * it.samples_per_elem for t, it in zip(targets, items)))
    xs = [torch.empty(t.n_nodes, dtype=torch.float64, device="cuda") for t in targets]
    bs = [torch.empty(t.n_nodes, dtype=torch.float64, device="cuda") for t in targets]
    max_iter = 60
    for i in range(max(1, args.warmup)):
        B.run(rtol=1e-14, max_iter=max_iter, xs=xs, bs=bs)
        log(f"batch warmup {i + 1}")
    torch.cuda.synchronize()
    times = []
    reps = sts = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, reps, sts, st = B.run(rtol=1e-14, max_iter=max_iter, xs=xs, bs=bs)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    wall = time.perf_counter() - t0
    ms = wall * 1e3 / args.steps
    src_bytes = 0
    for S in sources:
        si = S.info
        src_bytes += source_mesh_bytes(si.dim, 1, {"E": si.n_elems, "n": si.n_nodes, "n_reg": si.n_registrations,
                                                   "nbins": int(np.prod([si.bins[c] for c in range(si.dim)]))})
    # per element: connectivity, vertex coordinates, control values, measure, beta
    elem_bytes = sum(t.n_elems * ((t.dim + 1) * 4 + (t.dim + 1) * t.dim * 8 + (t.dim + 1) * 8 + 8 + (t.dim + 1) * 8)
                     for t in targets)
    abytes = src_bytes + elem_bytes
    achieved = abytes / (float(np.mean(times)) * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": E_tot / (ms * 1e-3),
        "unit": "target elements/s (aggregate over the batch)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "batch256", "transfers": len(items), "target_elements": E_tot, "samples": S_tot,
                   "dims": {"2": sum(1 for it in items if it.dim == 2), "3": sum(1 for it in items if it.dim == 3)},
                   "samples_per_elem": "per transfer from {32, 64, 128, 256}", "alpha": 1.0, "rtol": 1e-14,
                   "cg_launches": max_iter, "graph": True},
        "queries_per_s": S_tot / (ms * 1e-3),
        "event_ms": float(np.mean(times)),
        "setup_ms": setup_s * 1e3,
        "autotune": tune,
        "cg_iters_max": int(max(r["iters"] for r in reps)),
        "cons_defect_max": float(max(r["cons_defect"] for r in reps)),
        "status": ft.STATUS_NAMES[st],
        "roofline": {"bound": "hbm", "kernel": "ft_batch_run (whole graph)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes": abytes, "avg_ms": float(np.mean(times))},
    }
    if args.sequential:
        out["sequential_f64"] = sequential_batch(targets, sources, cfgs, xs, max_iter)
        out["sequential_f64"]["speedup_of_batched"] = out["sequential_f64"]["ms_total"] / ms
    B.close()
    for t in targets:
        t.close()
    for s_ in sources:
        s_.close()
    print(json.dumps(out), flush=True)


def sequential_batch(targets, sources, cfgs, xs, max_iter):
    """The comparator of the batch: the same transfers one after another
    through the single-transfer calls (ft_transfer_p1, then ft_project, which
    returns its report to the host), one untimed pass, then one timed pass."""
    import torch

    total = 0.0
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for T, S, c, x in zip(targets, sources, cfgs, xs):
            T.transfer_from(S, c)
            T.project(1, rtol=1e-14, max_iter=max_iter, x=x.view(1, -1), want_b=False)
        torch.cuda.synchronize()
        total = (time.perf_counter() - t0) * 1e3
        log(f"sequential batch pass {rep + 1}: {total:.1f} ms")
    return {"transfers": len(targets), "ms_total": total,
            "value": sum(t.n_elems for t in targets) / (total * 1e-3), "unit": "target elements/s"}


# FETCH_SIZE / WRITE_SIZE (KiB per dispatch) scaled by what they read for a
# plain device copy of known size (see profiles/hbm_traffic.md)
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
RECORD_KERNELS = ["k_emit", "k_src_eval_many", "k_src_eval", "k_consume_mfma", "k_consume", "k_fused_p1"]


def counter_records(dirs, workload, precision):
    """Record lines for the records files from rocprofv3 --pmc CSV output
    (FETCH_SIZE, WRITE_SIZE, SQ_INSTS_VALU, SQ_WAVES): per kernel of the step,
    the counters averaged over its dispatches, with the digest of its current
    device sources and the average duration of its dispatches."""
    import csv
    import glob

    per = {}   # kernel -> dispatch id -> {counter: value, "ns": duration}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as fh:
                for row in csv.DictReader(fh):
                    name = row["Kernel_Name"]
                    k = next((k for k in RECORD_KERNELS if f"ft::{k}<" in name or name.startswith(f"ft::{k}(")
                              or name == f"ft::{k}"), None)
                    if k is None:
                        continue
                    disp = per.setdefault(k, {}).setdefault((path, row["Dispatch_Id"]), {})
                    disp[row["Counter_Name"]] = disp.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
                    disp["ns"] = float(row["End_Timestamp"]) - float(row["Start_Timestamp"])
                    disp["grid"] = int(row["Grid_Size"])
    lines = []
    for k, disps in per.items():
        # the step's own launch: the largest grid (smaller ones are tuning samples)
        gmax = max(x["grid"] for x in disps.values())
        disps = {key: x for key, x in disps.items() if x["grid"] == gmax}
        def mean(c):
            v = [x[c] for x in disps.values() if c in x]
            return sum(v) / len(v) if v else None
        rec = {"kernel": k, "workload": workload, "precision": precision, "dispatches": len(disps),
               "sources": sources_digest(k)}
        if mean("FETCH_SIZE") is not None or mean("WRITE_SIZE") is not None:
            rec.update(fetch_bytes=(mean("FETCH_SIZE") or 0.0) * 1024 * FETCH_SCALE,
                       write_bytes=(mean("WRITE_SIZE") or 0.0) * 1024 * WRITE_SCALE)
        if mean("SQ_INSTS_VALU") is not None:
            rec.update(valu_insts=mean("SQ_INSTS_VALU"), waves=mean("SQ_WAVES"))
        rec["avg_ms_profiled"] = mean("ns") * 1e-6
        lines.append("record " + json.dumps(rec))
    return lines


def calibrate_copy(nbytes):
    """A plain device copy of known size, for scaling rocprof FETCH_SIZE / WRITE_SIZE."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tri2d_1m")
    ap.add_argument("--precision", default="f64", choices=list(PRECISIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--counter-records", nargs="+", metavar="DIR",
                    help="print record lines for profiles/hbm_traffic.md and profiles/valu_counts.md from "
                         "rocprofv3 --pmc CSV output directories (with --workload and --precision)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES")
    ap.add_argument("--route", default="blackbox", choices=["blackbox", "fused"],
                    help="blackbox: sample -> source eval -> consume through the point-query list; "
                         "fused: ft_transfer_p1 (built-in source, no query list)")
    ap.add_argument("--no-fused", action="store_true", help="skip the extra fused-route and plan-route measurements")
    ap.add_argument("--layout", default="auto", choices=["auto", "field-major", "tiles"],
                    help="layout of the query values: field-major [F][Q] or element tiles (ft_source_eval_tiles); "
                         "auto: tiles for several fields")
    ap.add_argument("--bins", type=int, default=0, help="source bin cells per axis (0: the workload's choice)")
    ap.add_argument("--refine-steps", type=int, default=0,
                    help="mass solve: 0 = binary64 PCG; k > 0 = binary32 inner PCG with k binary64 refinement steps")
    ap.add_argument("--autotune", default="auto", choices=["auto", "on", "off"],
                    help="tune the source bin grid on a sample of the queries (auto: when the workload fixes none); "
                         "batch256: the element variants and bin grids per kind of transfer")
    ap.add_argument("--tune-cache", default="", help="batch256: JSON file of the batch autotuner's choices")
    ap.add_argument("--sequential", action="store_true",
                    help="multi-field workloads: also time F sequential one-field FP64 transfers; "
                         "batch256: also time the transfers one after another")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the transfer shards by target elements but the multi-GPU path is not built", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.cpu_baseline_child:
        cpu_baseline_child(args)
        return
    if args.counter_records:
        for line in counter_records(args.counter_records, args.workload, args.precision):
            print(line)
        return

    import numpy as np
    import torch

    from paper_2603_00538_amd import ft
    from workloads import configs, fields

    if args.workload == "batch256":
        bench_batch(args)
        return
    w = configs.WORKLOADS[args.workload]
    log(f"workload {w.name}: building meshes")
    tmesh = configs.target_mesh(w)
    analytic = w.source is None   # the field itself is the black box (no source mesh)
    if analytic and args.route != "blackbox":
        print(f"{w.name} has no source mesh: only the black-box route applies", file=sys.stderr)
        sys.exit(2)
    if not analytic:
        smesh = configs.build_mesh(w.source)
        svals = configs.source_nodal_values(w, smesh[0])
        sc, sconn = smesh
    tc, tconn = tmesh
    dim, E, n = w.dim, tconn.shape[0], tc.shape[0]
    N, F = w.samples_per_elem, w.n_fields
    prec = getattr(ft, PRECISIONS[args.precision])
    p = 8 if prec == ft.FT_F64 else 4
    dt_ = torch.float64 if prec == ft.FT_F64 else torch.float32
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    # ---- setup (once per mesh pair)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = ft.Target(tc, tconn, order=w.order)
    bins = (args.bins,) * 3 if args.bins else (w.bins if any(w.bins) else None)
    S = None if analytic else ft.Source(sc, sconn, svals, bins=bins)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s * 1e3:.1f} ms; nnz {T.info.nnz}")
    Q = T.query_count(N)
    tuned = None
    if not analytic and (args.autotune == "on" or (args.autotune == "auto" and bins is None)):
        # sample: about 4M queries of this transfer's query list, the samples of
        # 16 runs of consecutive elements spread evenly over the target (runs,
        # so that neighbouring waves share cached candidates as in a full
        # step).  The node block is left out: it is a small part of a step,
        # but in a structured node order its waves take the point-by-point
        # search, whose cost falls with finer bins.
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        full = torch.empty((dim, Q), dtype=dt_, device=dev)
        T.sample_points(ft.SampleCfg(N, F, w.alpha, w.philox_seed, 0, prec), out=full)
        E_ = T.n_elems
        run_len = max(1, min(E_, 4_000_000 // N) // 16)
        starts = torch.linspace(0, E_ - run_len, 16, device=dev).round().long()
        picked = (starts[:, None] + torch.arange(run_len, device=dev)[None, :]).reshape(-1).unique()
        qidx = (n + picked[:, None] * N + torch.arange(N, device=dev)[None, :]).reshape(-1)
        sample = full[:, qidx].contiguous()
        m = int(sample.shape[1])
        del full
        base = int(S.info.bins[0])
        cands = sorted({max(4, int(round(base * f))) for f in (0.75, 0.9, 1.0, 1.15, 1.3, 1.5, 1.7)})
        tuned = {"candidates": cands, "chosen": S.autotune(sample, 0, cands)[:dim],
                 "sample_queries": m, "ms": 0.0}
        del sample
        torch.cuda.synchronize()
        tuned["ms"] = (time.perf_counter() - t0) * 1e3
        log(f"autotuned bins {tuned['chosen']} from {cands} in {tuned['ms']:.0f} ms")
    cfg = ft.SampleCfg(N, F, w.alpha, w.philox_seed, 0, prec)
    tiles = args.layout == "tiles" or (args.layout == "auto" and F > 1)
    cfg.values_layout = ft.FT_VALUES_ELEMENT_TILES if tiles else ft.FT_VALUES_FIELD_MAJOR
    pts = torch.empty((dim, Q), dtype=dt_, device=dev)
    vals = torch.empty((F, Q), dtype=dt_, device=dev)
    x = torch.empty((F, n), dtype=torch.float64, device=dev)
    b = torch.empty((F, n), dtype=torch.float64, device=dev)

    phases = ["emit", "eval", "consume", "project"] if args.route == "blackbox" else ["fused", "project"]
    times = {k: [] for k in phases}
    reports = None
    status = None

    def step(record, route):
        nonlocal reports, status
        nev = 5 if route == "blackbox" else 3
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(nev)] if record else None
        if record:
            ev[0].record()
        if route == "blackbox":
            T.sample_points(cfg, out=pts)
            if record:
                ev[1].record()
            if analytic:
                vals.copy_(fields.evaluate(w.field, torch, pts.t()))
            elif tiles:
                S.eval_tiles(pts, n, E, N, out=vals.view(-1))
            else:
                S.eval_query_list(pts, n, out=vals)
            if record:
                ev[2].record()
            T.consume(cfg, vals)
        else:
            T.transfer_from(S, cfg)
        if record:
            ev[nev - 2].record()
        res = T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b, refine_steps=args.refine_steps)
        if record:
            ev[nev - 1].record()
        reports, status = res.reports, res.status
        return ev

    def timed(route, steps, warmup):
        names = ["emit", "eval", "consume", "project"] if route == "blackbox" else ["fused", "project"]
        tms = {k: [] for k in names}
        for i in range(warmup):
            step(False, route)
            log(f"{route} warmup {i + 1}/{warmup}")
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for i in range(steps):
            evs.append(step(True, route))
        torch.cuda.synchronize()
        wall_ = time.perf_counter() - t0
        for ev in evs:
            for k, name in enumerate(names):
                tms[name].append(ev[k].elapsed_time(ev[k + 1]))
        log(f"{route}: timed {steps} steps in {wall_:.3f} s")
        return wall_, {k: float(np.mean(v)) for k, v in tms.items()}

    wall, phase_ms = timed(args.route, args.steps, args.warmup)
    ms_step = wall * 1e3 / args.steps
    extra_route = None
    if args.route == "blackbox" and not args.no_fused and F <= 4 and prec == ft.FT_F64 and not analytic:
        fw, fph = timed("fused", args.steps, 1)
        extra_route = {"route": "fused (ft_transfer_p1, no query list)", "ms_per_step": fw * 1e3 / args.steps,
                       "value": E / (fw / args.steps), "phases_ms": fph}

    plan_route = None
    if args.route == "blackbox" and not args.no_fused and F <= 4 and prec == ft.FT_F64 and w.order == 1 \
            and not analytic:
        # setup/online split: localization cached once, then online transfers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = ft.Plan(T, S, ft.SampleCfg(N, F, w.alpha, w.philox_seed, 0, ft.FT_F64))
        torch.cuda.synchronize()
        plan_setup = time.perf_counter() - t0
        for _ in range(1):
            plan.transfer()
            T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
        ms = []
        for _ in range(args.steps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            plan.transfer()
            e1.record()
            T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
            e2.record()
            torch.cuda.synchronize()
            ms.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
        on = float(np.mean([a + c for a, c in ms]))
        plan_route = {"route": "plan (localization cached at setup; online transfer + project)",
                      "setup_ms": plan_setup * 1e3, "online_ms": on, "value": E / (on * 1e-3),
                      "phases_ms": {"online": float(np.mean([a for a, _ in ms])),
                                    "project": float(np.mean([c for _, c in ms]))}}
        plan.close()

    supermesh_route = None
    if args.route == "blackbox" and not args.no_fused and F <= 4 and w.order == 1 and not analytic:
        # the exact load vector by mesh intersection (the paper's comparator):
        # its time, and the Monte Carlo load vector's distance from it
        b_mc = b.clone()
        T.transfer_supermesh(S)
        T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
        ms = []
        for _ in range(args.steps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            T.transfer_supermesh(S)
            e1.record()
            T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
            e2.record()
            torch.cuda.synchronize()
            ms.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
        on = float(np.mean([a_ + c_ for a_, c_ in ms]))
        err = float(torch.linalg.norm(b_mc - b) / torch.linalg.norm(b))
        supermesh_route = {"route": "mesh intersection (ft_transfer_supermesh, exact b) + project",
                           "ms_per_step": on, "value": E / (on * 1e-3),
                           "phases_ms": {"intersect": float(np.mean([a_ for a_, _ in ms])),
                                         "project": float(np.mean([c_ for _, c_ in ms]))},
                           "mc_load_vector_rel_l2_error": err}
        # the variance variants on the same workload: their load vectors' distance
        # from the exact one (one realization each) and their step times
        exact = b.clone()
        variants = {"plain": {"rel_l2_error": err}}
        for name, strat, own in (("stratified", True, False), ("own_alpha", False, True),
                                 ("stratified_own_alpha", True, True)):
            c_ = ft.SampleCfg(N, F, w.alpha, w.philox_seed, 0, prec)
            c_.sampling = ft.FT_SAMPLING_STRATIFIED if strat else ft.FT_SAMPLING_PLAIN
            c_.alpha_mode = ft.FT_ALPHA_ELEMENT if own else ft.FT_ALPHA_FIXED
            tms = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                T.sample_points(c_, out=pts)
                S.eval_query_list(pts, n, out=vals)
                T.consume(c_, vals)
                T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
                e1.record()
                torch.cuda.synchronize()
                tms.append(e0.elapsed_time(e1))
            variants[name] = {"rel_l2_error": float(torch.linalg.norm(b - exact) / torch.linalg.norm(exact)),
                              "ms_per_step": float(np.median(tms))}
        if prec in (ft.FT_F64, ft.FT_F32):
            # variance-driven counts: a pilot of N/4 samples per element (fused
            # route, its own stream) gives the element variances; the counts
            # for N per element on average follow them (field 0)
            n0 = max(2, N // 4)
            pc = ft.SampleCfg(n0, F, w.alpha, w.philox_seed, 1 << 20, prec)
            ac = ft.SampleCfg(0, F, w.alpha, w.philox_seed, 0, prec)
            tp, tal, tms, tfu = [], [], [], []
            for _ in range(3):
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                e0.record()
                T.transfer_from(S, pc)
                T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
                e1.record()
                offs, al = T.allocate_samples(N * E, n_min=2)
                e2.record()
                pa = torch.empty((dim, n + al.total), dtype=dt_, device=dev)
                va = torch.empty((F, n + al.total), dtype=dt_, device=dev)
                torch.cuda.synchronize()
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
                ev[0].record()
                T.sample_points_adaptive(ac, offs, al.total, out=pa)
                ev[1].record()
                S.eval_query_list(pa, n, out=va)
                ev[2].record()
                T.consume_adaptive(ac, offs, al.total, va)
                ev[3].record()
                ra = T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
                ev[4].record()
                torch.cuda.synchronize()
                del pa, va
                ef = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                ef[0].record()
                T.transfer_from_adaptive(S, ac, offs, al.total)
                ef[1].record()
                rf = T.project(F, rtol=w.rtol, max_iter=1000, x=x, b=b)
                ef[2].record()
                torch.cuda.synchronize()
                tp.append(e0.elapsed_time(e1))
                tal.append(e1.elapsed_time(e2))
                tms.append([ev[k].elapsed_time(ev[k + 1]) for k in range(4)])
                tfu.append([ef[0].elapsed_time(ef[1]), ef[1].elapsed_time(ef[2])])
            cnt = torch.diff(offs)
            ph = np.median(np.array(tms), axis=0)
            variants["neyman_counts"] = {
                "rel_l2_error": float(torch.linalg.norm(b - exact) / torch.linalg.norm(exact)),
                "ms_per_step": float(ph.sum()), "phases_ms": dict(zip(("emit", "eval", "consume", "project"),
                                                                      map(float, ph))),
                "counts_min_max": [int(cnt.min()), int(cnt.max())], "pilot_ms": float(np.median(tp)),
                "allocate_ms": float(np.median(tal)), "pilot_samples_per_elem": n0,
                "total_samples": int(al.total), "sum_b_stderr": ra.reports[0]["sum_b_stderr"],
                "predicted_stderr": al.predicted_stderr,
                "uniform_sum_b_stderr": reports[0]["sum_b_stderr"],
                "fused_route": {"ms_per_step": float(np.median(np.array(tfu).sum(axis=1))),
                                "phases_ms": dict(zip(("fused", "project"), map(float, np.median(np.array(tfu), axis=0)))),
                                "sum_b_stderr": rf.reports[0]["sum_b_stderr"]}}
        supermesh_route["variance_variants"] = variants
        del b_mc, exact

    if analytic:
        src_info = None
    else:
        si = S.info
        src_info = {"E": sconn.shape[0], "n": sc.shape[0], "n_reg": int(si.n_registrations),
                    "nbins": int(np.prod([si.bins[c] for c in range(dim)]))}
    # (an analytic black box is the caller's work, not a kernel of the library)
    cand = [k for k in ("emit", "eval", "consume", "fused") if k in phase_ms and not (analytic and k == "eval")]
    dom = max(cand, key=lambda k: phase_ms[k])
    split = prec in (ft.FT_SPLIT_F16, ft.FT_SPLIT_BF16) and N <= 256 and F <= 64
    kernel_names = {"emit": "k_emit", "eval": "k_src_eval_many" if F > 1 else "k_src_eval",
                    "consume": "k_consume_mfma" if split else "k_consume", "fused": "k_fused_p1"}
    roof = kernel_roofline(kernel_names[dom], w.name, args.precision,
                           algorithmic_bytes(dom, dim, E, n, N, F, p, src_info), phase_ms[dom])
    method = None
    if "emit" in phase_ms and "consume" in phase_ms:
        # the method's own stream around a black box: emission writes the
        # points, consumption reads the values (plus element and node data)
        per = {}
        for ph in ("emit", "consume"):
            per[kernel_names[ph]] = kernel_roofline(kernel_names[ph], w.name, args.precision,
                                                    algorithmic_bytes(ph, dim, E, n, N, F, p, src_info),
                                                    phase_ms[ph])
        mb = sum(r["algorithmic_bytes"] if r["bound"] == "hbm" else r["hbm"]["algorithmic_bytes"]
                 for r in per.values())
        mt = phase_ms["emit"] + phase_ms["consume"]
        tr = [r["traffic"] for r in per.values()]
        method = {"bound": "hbm", "kernels": "k_emit + k_consume (+ node assembly)", "achieved": mb / (mt * 1e-3) / 1e9,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mb / (mt * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "traffic": sum(tr) if all(t is not None for t in tr) else None, "algorithmic_bytes": mb,
                  "ms": mt, "per_kernel": per}
    # conservation against the exact integral of the source field (sec. 2 Eq.
    # conservation; the relative conservation error of sec. 5.1)
    ints = S.integral() if not analytic else [configs.field_integral(w)] * F
    cons = []
    for f_, rep_ in enumerate(reports):
        I = ints[f_]
        cons.append({"int_source": I, "int_x": rep_["int_x"], "sum_b": rep_["sum_b"],
                     "E_mass": abs(rep_["int_x"] - I) / abs(I) if I != 0 else None,
                     "discrete_defect": rep_["cons_defect"]})
    out = {
        "metric": METRIC,
        "value": E / (ms_step * 1e-3),
        "unit": "target elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "route": args.route, "dim": dim, "target_elements": E, "target_nodes": n,
                   "source_elements": None if analytic else int(sconn.shape[0]),
                   "black_box": f"analytic {w.field}" if analytic else "P1 source mesh (ft_source_eval)",
                   "samples_per_elem": N, "n_fields": F,
                   "queries": Q, "alpha": w.alpha, "rtol": w.rtol,
                   "bins": list(w.bins[:dim]) if any(w.bins) else "default", "precision": args.precision,
                   "values_layout": "element tiles" if tiles else "field-major",
                   "solve": "binary64 PCG" if args.refine_steps == 0 else
                            f"binary32 PCG + {args.refine_steps} binary64 refinement steps"},
        "queries_per_s": Q / (ms_step * 1e-3),
        "phases_ms": phase_ms,
        "setup_ms": setup_s * 1e3,
        "cg_iters": reports[0]["iters"],
        "cons_defect": reports[0]["cons_defect"],
        "rel_resid": reports[0]["rel_resid"],
        "status": ft.STATUS_NAMES[status],
        "roofline": roof,
        "conservation": cons[0] if F == 1 else {
            "fields": F, "E_mass_max": max(c_["E_mass"] for c_ in cons if c_["E_mass"] is not None),
            "discrete_defect_max": max(c_["discrete_defect"] for c_ in cons)},
    }
    if method is not None:
        out["method_roofline"] = method
    if extra_route is not None:
        out["fused_route"] = extra_route
    if plan_route is not None:
        out["plan_route"] = plan_route
    if supermesh_route is not None:
        out["supermesh_route"] = supermesh_route
    if tuned is not None:
        out["bin_autotune"] = tuned
    if not analytic:
        out["config"]["bins"] = [int(si.bins[c]) for c in range(dim)]
        out["config"]["bin_registrations"] = int(si.n_registrations)
        S.close()
    else:
        out["config"]["bins"] = None
    del pts, vals
    torch.cuda.empty_cache()
    if args.sequential and F > 1:
        out["sequential_f64"] = sequential_f64(T, w, tmesh, smesh, svals)
        out["sequential_f64"]["speedup_of_batched"] = out["sequential_f64"]["ms_total"] / ms_step
    T.close()
    if not args.no_cpu_baseline and w.order == 1 and not analytic:
        log("cpu baseline (the oracle on the host cores, bounded samples, child process)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
