#!/usr/bin/env python3
"""Throughput of the free-flight expansion (prescription (FF), section 5.2) on one MI355X.

A step is one whole expansion of the workload: every q-term of (FFpsi)
(premultiply, forward transform, chirp, pruned inverse, twiddle-gather-
accumulate) and the density |Psibar|^2 of every field, with the inputs already
resident in device memory. The default workload is the ragged ensemble of 768
3-D realizations (256 each of 32x32x256, 48x48x384 and 64x64x512, magnification
40 per axis, 64000 terms each), expanded by one HIP graph launch per step, in
the FP32 form (FP32 data, FP64-built phase tables: the headline value) and in
plain FP64 on the same ensemble; --config selects the single-field workloads.

Prints one JSON line with the throughput in output lattice points per second,
the FP64 line and the speedup between the two, the roofline of the dominant
kernel (its launches timed with HIP events on the stream they run on), the
relative L2 error of one realization per shape class against the oracle, and
the CPU oracle timed on the host as a baseline.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
ADJOINT_SLOT0 = 32  # first pass-timing slot of the adjoint schedule (FX_ADJOINT_SLOT0 in include/fx.h)


def pass_cost(p: dict, csize: int, outer_chunks: int = 1):
    """Algorithmic flops and unique bytes of one launch of a pass (the roofline model).

    Counting convention: complex multiply 6 flops, complex add 2, complex
    multiply-add 8, a length-N transform 5 N log2 N. Per line and magnification index:
      transform form of E:  6M (premultiply) + 5M log2 M + 6M (chirp) + 2(M - P) (fold)
                            + 5P log2 P (pruned inverse) + 2P
      register form of E:   6M (premultiply) + 5M log2 P (g transforms of P points) + 6M (folded
                            chirp table) + 2M (sum over the g subsequences) + 5P log2 P (inverse)
      EA adds 8M (the twiddle multiply-accumulate of every output point), or with the structured
      accumulate (EA with "eas") 8P (one twiddle product per pruned output) per line and term plus
      a g-point inverse transform (5 g log2 g) per output group (P groups per line).
    A: 8 flops per output and term; AA (two fused accumulates) and its adjoint AAH: 16 per
    term sample plus a g_u x g_v transform per output group.
    """
    kind, M, P, lam = p["kind"], p["M"], p["P"], p["lam"]
    qn = p.get("qn", lam)
    lines = p["Qin"] * p["A"] * p["S"]
    lg = lambda n: math.log2(n) if n > 1 else 0.0
    if p.get("reg") and kind in ("E", "EA", "EH"):
        e_line = 6 * M + 5 * M * lg(P) + 6 * M + 2 * M + 5 * P * lg(P)
    else:
        e_line = 6 * M + 5 * M * lg(M) + 6 * M + 2 * (M - P) + 5 * P * lg(P) + 2 * P
    if kind in ("E", "EH"):
        flops = lines * qn * e_line
        byts = (lines * M + lines * qn * P) * csize
    elif kind in ("EA", "EAH"):
        if p.get("eas"):
            g = M // P
            flops = lines * qn * (e_line + 8 * P) + lines * P * 5 * g * lg(g)
        else:
            flops = lines * qn * (e_line + 8 * M) + lines * M * 2
        byts = 2 * lines * M * csize
    elif kind in ("AA", "AAH"):
        nin = p["O"] * p["qn2"] * qn * p["X"] * P * p["Y"] * p["P2"] * p["Z"]
        nout = p["O"] * p["X"] * M * p["Y"] * p["M2"] * p["Z"]
        flops = nin * 16 + nout * 5 * lg(p["g"] * p["g2"])
        byts = (nin + nout) * csize
    else:  # A, AH
        outs = p["Qin"] * p["A"] * M * p["S"]
        flops = outs * 8 * qn
        byts = (outs + p["Qin"] * qn * p["A"] * P * p["S"]) * csize
    return flops, byts


def kernels_hash() -> str:
    from paper_1602_03395_amd.profiling import kernels_hash as kh
    return kh()


def load_traffic_entry(tag: str, kernel_key: str):
    """The committed counter summary of one pass (dict), or None when it was taken on other kernel
    sources or another workload."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernels_hash") != kernels_hash():
        return None
    return d.get("workloads", {}).get(tag, {}).get("passes", {}).get(kernel_key)


def load_traffic(tag: str, kernel_key: str):
    """HBM bytes per launch of one pass from the committed counter summary, or None when it
    was taken on other kernel sources or another workload."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernels_hash") != kernels_hash():
        return None
    ent = d.get("workloads", {}).get(tag, {}).get("passes", {}).get(kernel_key)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def cpu_baseline(wl, field, lam, dx, t):
    import numpy as np

    import oracle
    from oracle import propagator as OP
    OP._axis_matrix_cached.cache_clear()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = min(threads, os.cpu_count() or threads)
    t0 = time.perf_counter()
    ref = oracle.expand(field.astype(np.complex128), dx, wl.m_over_hbar, t, lam)
    rho = oracle.density(ref)
    dt = time.perf_counter() - t0
    return ref, rho, {"value": field.size / dt, "unit": "output lattice pts/s", "cores": threads,
                      "kind": "oracle", "seconds": dt,
                      "sample": f"one full field of the workload ({field.size} output points): per-axis "
                                f"long-double kernel tables + FP64 per-axis contraction"}


def _time_batch(b, psis, outs, rhos, steps, warmup, stream):
    """Warmup, then EXACTLY `steps` graph launches bracketed by synchronisations; returns ms per step."""
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            b.run(psis, psi_outs=outs, rho_outs=rhos)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            b.run(psis, psi_outs=outs, rho_outs=rhos)
        ev1.record(stream)
        torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / max(steps, 1)


def _batch_pass_rows(b, psis, outs, rhos, stream, csize):
    """Per-pass kernel durations of one ensemble run, per class: HIP events the library records on
    the stream every launch goes to (the class's lane) while timing is on (the run is then issued
    eagerly, launch by launch, in the configuration the graph holds). Flops of a pass over the whole
    class: the per-launch count of one work item (G realizations, one q-block) times the items."""
    import torch
    classes = b.classes()
    for c in classes:
        c["plan"].set_timing(True)
        c["plan"].pass_times()
    with torch.cuda.stream(stream):
        b.run(psis, psi_outs=outs, rho_outs=rhos)
    torch.cuda.synchronize()
    rows = []
    for c in classes:
        plan = c["plan"]
        times = plan.pass_times()
        plan.set_timing(False)
        desc = json.loads(plan.describe())
        G = desc["slices"]
        nmem = len(c["members"])
        seen = {}
        for i, (n_launch, tot_ms) in enumerate(times):
            if n_launch == 0 or i >= len(desc["passes"]):
                continue
            pdesc = desc["passes"][i]
            key = f'{pdesc["kind"]}#{seen.get(pdesc["kind"], 0)}'
            seen[pdesc["kind"]] = seen.get(pdesc["kind"], 0) + 1
            f_launch, b_launch = pass_cost(pdesc, csize)
            # every pass is linear in the slices (G realizations) and in the q-block of the outer
            # index: scale one item's count to the whole class
            lam_outer = desc["passes"][0]["lam"]
            scale = (nmem / G) * (lam_outer / desc["outer_block"])
            rows.append({"class": "x".join(str(x) for x in plan.shape), "pass": f'{pdesc["kind"]}(axis{pdesc["axis"]})',
                         "key": key, "kernel": pdesc.get("kernel", "?"), "launches": n_launch, "ms": tot_ms,
                         "flops": f_launch * scale, "bytes": b_launch * scale,
                         "group": G, "q_block": desc["outer_block"], "lane": c["lane"]})
    # replicas of a class (same shape, items split over two lanes) add up into one row per pass
    merged = {}
    for r in rows:
        m = merged.get((r["class"], r["key"]))
        if m is None:
            merged[(r["class"], r["key"])] = dict(r)
        else:
            for f in ("launches", "ms", "flops", "bytes"):
                m[f] += r[f]
    rows = list(merged.values())
    for r in rows:
        r["avg_ms"] = r["ms"] / r["launches"]
        r["tflops"] = r["flops"] / (r["ms"] * 1e-3) / 1e12
        r["gbs"] = r["bytes"] / (r["ms"] * 1e-3) / 1e9
    return classes, rows


def _calibration_copy(mib, dev):
    """A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the traffic
    figures of the profiled kernels."""
    import torch
    nb = mib << 20
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    # two strided gathers of the same source (rows of 512 bytes, the first 256 / 64 bytes of each): they
    # check the copy's scale factors on partial-line reads like those of the strided line passes
    rows = src.view(-1, 128)
    half = rows[:, :64].contiguous()
    eighth = rows[:, :16].contiguous()
    torch.cuda.synchronize()
    del src, dst, half, eighth


def bench_c4(args, fields):
    """The ragged ensemble: every realization expanded by one graph launch per step, FP32 form
    (headline) and plain FP64 on the same ensemble."""
    import numpy as np
    import torch

    import paper_1602_03395_amd as fx
    import workloads

    dev = torch.device("cuda:0")
    if args.calibrate_copy_mb > 0:
        _calibration_copy(args.calibrate_copy_mb, dev)
    n = len(fields)
    lam, t, dx = (40, 40, 40), 400.0, (1.0, 1.0, 1.0)
    specs = [dict(shape=tuple(f.shape), dx=dx, lam=lam, t=t) for f in fields]
    npts = sum(int(f.size) for f in fields)
    stream = torch.cuda.Stream()
    result = {
        "metric": "expanded lattice pts/s + HBM roofline %, FP32/FP64-phase vs FP64 at 1e-5 err",
        "unit": "output lattice pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_ragged_ensemble", "members": n,
                   "shapes": [list(s) for s in workloads.C4_SHAPES], "lam": list(lam), "t": t, "dx": list(dx),
                   "terms_per_member": 64000, "schedule": args.schedule, "precision": "c64_phase64",
                   "launch": "one HIP graph launch per ensemble"},
    }
    # parity members: the first realization of every shape class
    par_idx = sorted({min(i for i in range(n) if fields[i].shape == shp) for shp in {f.shape for f in fields}})

    # ---- FP32 data, FP64-built phase tables (the headline) ----
    psis = [torch.from_numpy(f).to(dev) for f in fields]
    outs = [torch.empty_like(x) for x in psis]
    rhos = [torch.empty(x.shape, dtype=torch.float32, device=dev) for x in psis]
    tc = time.perf_counter()
    b = fx.Batch(specs, dtype=torch.complex64, schedule=args.schedule)
    create32 = time.perf_counter() - tc
    w0 = time.perf_counter()
    ms32 = _time_batch(b, psis, outs, rhos, args.steps, args.warmup, stream)
    wall32 = time.perf_counter() - w0
    result.update({"value": npts / (ms32 * 1e-3), "ms_per_step": ms32,
                   "q_term_pts_per_s": npts * 64000 / (ms32 * 1e-3)})
    got32 = {i: (rhos[i].cpu().numpy().astype(np.float64), outs[i].cpu().numpy().astype(np.complex128))
             for i in par_idx}
    classes, rows, rows_alone = ([], [], [])
    if not args.no_pass_timing:
        classes, rows = _batch_pass_rows(b, psis, outs, rhos, stream, 8)
        # the same passes one kernel at a time (every class on one stream): each kernel alone on the device
        b.set_lanes(1)
        _, rows_alone = _batch_pass_rows(b, psis, outs, rhos, stream, 8)
        b.set_lanes(0)
    cls_info = [{"shape": list(c["plan"].shape), "members": len(c["members"]), "group": c["group"],
                 "lane": c["lane"], "passes": [{"kind": p["kind"], "axis": p["axis"], "kernel": p.get("kernel"),
                                               "qn": p["qn"]} for p in json.loads(c["plan"].describe())["passes"]]}
                for c in (classes or b.classes())]
    result["config"]["classes"] = cls_info
    roofline = None
    if rows:
        dom = max(rows, key=lambda r: r["ms"])
        roofline = {"bound": "alu", "achieved": dom["tflops"], "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": dom["tflops"] / PEAK_FP32_TFLOPS, "traffic": None,
                    "kernel": f'{dom["kernel"]} ({dom["pass"]}, class {dom["class"]})',
                    "launches_per_step": dom["launches"], "avg_launch_ms": dom["avg_ms"],
                    "flops_per_launch": dom["flops"] / dom["launches"],
                    "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"]}
        alone = [r for r in rows_alone if r["class"] == dom["class"] and r["key"] == dom["key"]]
        if alone:
            a = alone[0]
            roofline["alone"] = {"achieved": a["tflops"], "frac": a["tflops"] / PEAK_FP32_TFLOPS,
                                 "avg_launch_ms": a["avg_ms"],
                                 "note": "the same launches with the classes one after the other on one stream"}
        ai = dom["flops"] / max(dom["bytes"], 1)
        if ai < PEAK_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
            roofline.update({"bound": "hbm", "achieved": dom["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": dom["gbs"] / PEAK_HBM_GBS})
        # measured HBM bytes per launch of that kernel (copy-calibrated FETCH_SIZE + WRITE_SIZE), while
        # the committed counters match the kernel sources
        ent = load_traffic_entry(f"c4_ragged_ensemble/c64/{args.schedule}", f'{dom["class"]}/{dom["key"]}')
        if ent:
            alg = roofline["algorithmic_bytes_per_launch"]
            if ent.get("group") == dom["group"] and ent.get("q_block") == dom["q_block"]:
                roofline["traffic"] = ent["hbm_bytes_per_launch"]
            elif ent.get("traffic_over_algorithmic"):
                # the tuner chose another item shape than the profiled run: the counters' ratio of
                # measured to algorithmic bytes, applied to this launch's algorithmic bytes
                roofline["traffic"] = ent["traffic_over_algorithmic"] * alg
                roofline["traffic_note"] = (f'scaled from the profiled launch (items of {ent.get("group")} '
                                            f'realizations, q-block {ent.get("q_block")})')
        result["passes"] = rows
    result["roofline"] = roofline
    del b, psis, outs, rhos
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # ---- plain FP64 on the same ensemble (inputs upcast exactly) ----
    fp64 = None
    got64 = {}
    if not args.no_fp64:
        psis = [torch.from_numpy(f).to(dev).to(torch.complex128) for f in fields]
        outs = [torch.empty_like(x) for x in psis]
        rhos = [torch.empty(x.shape, dtype=torch.float64, device=dev) for x in psis]
        tc = time.perf_counter()
        b = fx.Batch(specs, dtype=torch.complex128, schedule=args.schedule)
        create64 = time.perf_counter() - tc
        steps64 = args.fp64_steps if args.fp64_steps is not None else args.steps
        warm64 = min(args.warmup, 2)
        ms64 = _time_batch(b, psis, outs, rhos, steps64, warm64, stream)
        got64 = {i: (rhos[i].cpu().numpy(), outs[i].cpu().numpy()) for i in par_idx}
        fp64 = {"ms_per_step": ms64, "value": npts / (ms64 * 1e-3), "steps": steps64, "warmup": warm64,
                "batch_create_s": create64}
        del b, psis, outs, rhos
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    result["fp64"] = fp64
    result["speedup_fp32_vs_fp64"] = (fp64["ms_per_step"] / ms32) if fp64 else None
    result["batch_create_s"] = create32
    result["wall_s_timed_fp32"] = wall32

    # ---- the oracle on one realization per class: CPU baseline and parity of the batched outputs ----
    cpu = None
    parity = {}
    if not args.no_cpu_baseline:
        import oracle
        from oracle import propagator as OP
        threads = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1)
        secs = 0.0
        pts = 0
        for i in par_idx:
            OP._axis_matrix_cached.cache_clear()
            f = fields[i].astype(np.complex128)
            tc = time.perf_counter()
            ref = oracle.expand(f, dx, 1.0, t, lam)
            secs += time.perf_counter() - tc
            pts += f.size
            rr = oracle.density(ref)
            name = "x".join(str(x) for x in f.shape)
            ent = {"member": i, "fp32_rho_rel_l2": float(np.linalg.norm(got32[i][0] - rr) / np.linalg.norm(rr)),
                   "fp32_psi_rel_l2": float(np.linalg.norm(got32[i][1] - ref) / np.linalg.norm(ref))}
            if i in got64:
                ent["fp64_rho_rel_l2"] = float(np.linalg.norm(got64[i][0] - rr) / np.linalg.norm(rr))
                ent["fp64_psi_rel_l2"] = float(np.linalg.norm(got64[i][1] - ref) / np.linalg.norm(ref))
            parity[name] = ent
        cpu = {"value": pts / secs, "unit": "output lattice pts/s", "cores": threads, "kind": "oracle",
               "seconds": secs,
               "sample": f"the first realization of each of the {len(par_idx)} shape classes ({pts} output points), "
                         "full oracle solves: per-axis long-double kernel tables + FP64 per-axis contraction"}
    result["cpu_baseline"] = cpu
    result["speedup_gpu_vs_cpu_oracle"] = (result["value"] / cpu["value"]) if cpu else None
    result["parity_vs_oracle"] = parity or None
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c4", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="c4 ensemble: timed steps of the plain FP64 run (default: --steps)")
    ap.add_argument("--no-fp64", action="store_true", help="c4 ensemble: skip the plain FP64 run")
    ap.add_argument("--members", type=int, default=768, help="c4 only: number of realizations")
    ap.add_argument("--member", type=int, default=None,
                    help="c4 only: expand this single realization through one plan (per-pass timing)")
    ap.add_argument("--dtype", default=None, choices=[None, "c64", "c128"])
    ap.add_argument("--schedule", default="paper", choices=["paper", "axis_factorised"])
    ap.add_argument("--variant", default=None, choices=["free", "spectrum", "pair", "far_field", "brute_force", "grad"],
                    help="free: free flight (the paper's case); spectrum: a tabulated non-quadratic "
                         "axis-additive spectrum of the same size; pair: positive-P pair psi, psi^+; "
                         "far_field: the far-field estimate (comparator) on the same output lattice; "
                         "brute_force: the padded-lattice propagation (comparator), same result; "
                         "grad: expansion plus the gradient of the density fit loss (adjoint); "
                         "default: grad for the fitting workload (c5), free otherwise")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pass-timing", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.variant is None:
        args.variant = "grad" if args.config == "c5" else "free"
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(sharding the magnification terms over GPUs is not implemented)"}), flush=True)
        sys.exit(2)

    import numpy as np

    import workloads

    c4_fields = None
    if args.config == "c4" and args.member is None:
        # host generation in forked workers, before this process touches the GPU
        workers = max(1, min(16, os.cpu_count() or 1))
        c4_fields = workloads.c4_fields_c64(range(args.members), workers=workers)

    import torch

    import paper_1602_03395_amd as fx

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(3)

    if c4_fields is not None:
        return bench_c4(args, c4_fields)

    if args.config == "c4":
        wl = workloads.make_c4(members=[args.member])
    else:
        wl = workloads.make_workload(args.config)
    dtype_name = args.dtype or wl.dtype
    dtype = torch.complex64 if dtype_name == "c64" else torch.complex128
    npdt = np.complex64 if dtype_name == "c64" else np.complex128
    field = wl.fields[0].astype(npdt)
    dx, lam, t = wl.dx, wl.lam, wl.t
    # the fitting workload is a stack of fields expanded (and differentiated) in one call
    stacked = args.config == "c5"
    if stacked and args.variant not in ("free", "grad"):
        print(json.dumps({"error": "the stacked fitting workload runs the free or grad variant only"}), flush=True)
        sys.exit(2)

    dev = torch.device("cuda:0")
    if args.calibrate_copy_mb > 0:
        _calibration_copy(args.calibrate_copy_mb, dev)
    psi = torch.from_numpy(field).to(dev)
    stack = torch.from_numpy(np.stack([f.astype(npdt) for f in wl.fields])).to(dev) if stacked else None
    spectrum = None
    if args.variant == "spectrum":
        # per-axis Bogoliubov-like spectrum omega = sqrt(eps (eps + 2 mu)), eps = k^2 / 2m
        mu = 0.1
        spectrum = []
        for j in range(len(lam)):
            k = fx.fine_wavenumbers(psi.shape[j], lam[j], dx[j])
            eps = k * k / (2.0 * wl.m_over_hbar)
            spectrum.append(t * np.sqrt(eps * (eps + 2.0 * mu)))
    plan = fx.Plan(psi.shape, dx, wl.m_over_hbar, t, lam, dtype=dtype, schedule=args.schedule, spectrum=spectrum)
    out = torch.empty_like(psi)
    rho = torch.empty(psi.shape, dtype=torch.float32 if dtype == torch.complex64 else torch.float64, device=dev)
    if args.variant == "pair":
        rng = np.random.default_rng(np.random.SeedSequence(11))
        noise = 0.05 * (rng.standard_normal(field.shape) + 1j * rng.standard_normal(field.shape))
        psi_plus = torch.from_numpy((field.conj() + noise).astype(field.dtype)).to(dev)

        def step():
            return plan.expand_pair(psi, psi_plus)
    elif args.variant == "far_field":
        def step():
            return plan.far_field(psi)
    elif args.variant == "brute_force":
        def step():
            return plan.brute_force(psi)
    elif stacked:
        # the whole stack per step: its expansion, and with the grad variant the gradient of the
        # fitting loss L = sum (rho - tau)^2 of every field (tau: fixed synthetic images, here the
        # densities of the hidden fields on the input lattice; the timing does not depend on them)
        sout = torch.empty_like(stack)
        srho = torch.empty(stack.shape, dtype=rho.dtype, device=dev)
        tau = torch.from_numpy(np.stack([np.abs(h) ** 2 for h in wl.extra["hidden"]])).to(dev, rho.dtype)
        sgrad_rho = torch.empty_like(srho)
        sgrad = torch.empty_like(stack)

        def step():
            plan.expand_many(stack, psi_out=sout, rho_out=srho)
            if args.variant == "grad":
                torch.sub(srho, tau, out=sgrad_rho).mul_(2.0)
                plan.density_adjoint_many(sout, sgrad_rho, grad_in=sgrad)
    elif args.variant == "grad":
        # one forward + backward of the fitting loss L = sum (rho - tau)^2 (tau: a fixed synthetic image)
        tau = torch.full(psi.shape, 1e-6, dtype=rho.dtype, device=dev)
        grad_rho = torch.empty_like(rho)
        grad = torch.empty_like(psi)

        def step():
            plan.expand(psi, psi_out=out, rho_out=rho)
            torch.sub(rho, tau, out=grad_rho).mul_(2.0)
            return plan.density_adjoint(out, grad_rho, grad_in=grad)
    else:
        def step():
            return plan.expand(psi, psi_out=out, rho_out=rho)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    desc = json.loads(plan.describe())

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = ev0.elapsed_time(ev1)

    # Per-pass kernel durations: HIP events recorded by the library on the launch stream around
    # every pass, over a second run of the same K steps (the events add gaps between passes, so
    # they stay out of the headline loop above).
    timing = not args.no_pass_timing
    passes = []
    if timing:
        plan.set_timing(True)
        plan.pass_times()  # clear
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        passes = plan.pass_times()
        plan.set_timing(False)

    if stacked:
        desc = json.loads(plan.describe())  # the pass layout of the stacked call (fields as slices)
    ms_per_step = gpu_ms / args.steps
    npts = int(np.prod(psi.shape)) * (int(stack.shape[0]) if stacked else 1)
    value = npts / (ms_per_step * 1e-3)
    terms = plan.num_terms()

    csize = 8 if dtype == torch.complex64 else 16
    peak_alu = PEAK_FP32_TFLOPS if dtype == torch.complex64 else PEAK_FP64_TFLOPS
    ridge = peak_alu * 1e12 / (PEAK_HBM_GBS * 1e9)
    pass_rows = []
    seen = {}
    for i, (n_launch, tot_ms) in enumerate(passes):
        if n_launch == 0:
            continue
        # slots from ADJOINT_SLOT0 on time the passes of the adjoint schedule (gradient variant)
        lst, j = (desc["passes"], i) if i < ADJOINT_SLOT0 else (desc.get("adjoint_passes", []), i - ADJOINT_SLOT0)
        p = dict(lst[j]) if j < len(lst) else {"kind": "?"}
        key = f'{p["kind"]}#{seen.get(p["kind"], 0)}'
        seen[p["kind"]] = seen.get(p["kind"], 0) + 1
        avg_ms = tot_ms / max(n_launch, 1)
        flops, byts = pass_cost(p, csize)
        pass_rows.append({"pass": f'{p["kind"]}(axis{p.get("axis")})', "key": key,
                          "launches_per_step": n_launch / args.steps,
                          "avg_ms": avg_ms, "flops": flops, "bytes": byts,
                          "tflops": flops / (avg_ms * 1e-3) / 1e12, "gbs": byts / (avg_ms * 1e-3) / 1e9})
    roofline = None
    if pass_rows:
        dom = max(pass_rows, key=lambda r: r["avg_ms"] * r["launches_per_step"])
        ai = dom["flops"] / max(dom["bytes"], 1)
        if ai >= ridge:
            roofline = {"bound": "alu", "achieved": dom["tflops"], "peak": peak_alu, "unit": "TFLOP/s",
                        "frac": dom["tflops"] / peak_alu}
        else:
            roofline = {"bound": "hbm", "achieved": dom["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": dom["gbs"] / PEAK_HBM_GBS}
        roofline["kernel"] = dom["pass"]
        tag = f"{wl.name}/{dtype_name}/{args.schedule}" + ("" if args.variant == "free" else f"/{args.variant}")
        roofline["traffic"] = load_traffic(tag, dom["key"])

    # Whole-step HBM view: measured bytes (copy-calibrated counters of every pass, while they match
    # the kernel sources) over the step time, as a fraction of the HBM peak.
    step_s = ms_per_step * 1e-3
    hbm = {"peak_GBs": PEAK_HBM_GBS}
    measured = [load_traffic(tag, r["key"]) for r in pass_rows] if pass_rows else []
    if measured and all(m is not None for m in measured):
        tot = sum(m * r["launches_per_step"] for m, r in zip(measured, pass_rows))
        hbm["measured_bytes_per_step"] = tot
        hbm["measured_GBs"] = tot / step_s / 1e9
        hbm["measured_frac"] = hbm["measured_GBs"] / PEAK_HBM_GBS
    else:
        hbm["measured_bytes_per_step"] = None

    result = {
        "metric": "expanded lattice pts/s + HBM roofline %, FP32/FP64-phase vs FP64 at 1e-5 err",
        "value": value,
        "unit": "output lattice pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == torch.complex64 else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "shape": list(psi.shape), "fields": int(stack.shape[0]) if stacked else 1,
                   "lam": list(lam), "dx": list(dx), "t": t,
                   "terms": terms, "schedule": args.schedule, "variant": args.variant,
                   "precision": "c64_phase64" if dtype == torch.complex64 else "c128",
                   "outer_block": desc["outer_block"]},
        "q_term_pts_per_s": npts * terms / (ms_per_step * 1e-3),
        "roofline": roofline,
        "hbm": hbm,
        "passes": pass_rows,
    }

    if not args.no_cpu_baseline and args.variant == "free":
        ref, ref_rho, cb = cpu_baseline(wl, field, lam, dx, t)
        result["cpu_baseline"] = cb
        got = (srho[0] if stacked else rho).cpu().numpy().astype(np.float64)
        if stacked:
            out = sout[0]
        result["rel_l2_rho_vs_oracle"] = float(np.linalg.norm(got - ref_rho) / np.linalg.norm(ref_rho))
        result["rel_l2_psi_vs_oracle"] = float(np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref))
    elif not args.no_cpu_baseline and stacked and args.variant == "grad":
        # the oracle's loss and gradient of the first field (same target image), timed on the host
        import oracle
        from oracle import propagator as OP
        OP._axis_matrix_cached.cache_clear()
        threads = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1)
        tau0 = tau[0].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        _, g_ref = oracle.loss_and_grad(field.astype(np.complex128), tau0, dx, wl.m_over_hbar, t, lam)
        secs = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": field.size / secs, "unit": "output lattice pts/s (expansion + gradient)",
                                  "cores": threads, "kind": "oracle", "seconds": secs,
                                  "sample": f"the loss and gradient of the first field ({field.size} points): "
                                            "per-axis long-double kernel tables + FP64 per-axis contractions"}
        g_gpu = sgrad[0].cpu().numpy().astype(np.complex128)
        result["rel_l2_grad_vs_oracle"] = float(np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref))
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
