#!/usr/bin/env python3
"""Benchmark of the damage-diffusion hot path on one MI355X.

Workload: the arrival query (Eq. 6 evaluated at every probe visit at the
moment it starts) of a 512x512 probe grid scanned in a seeded random order,
pitch 1 nm, sigma 0.4 nm, dwell 0.5 us, D = 1e-12 m^2/s, in mixed precision:
262144 visits, 3.436e10 causal pair terms per step.  One step is one full
query (near band, far region, fixed-order reduction) with the scan's probe
and lag-row tables resident in HBM (the first query builds them).  Prints
one JSON line.

The dominant kernel (far region) is timed with HIP events on the stream it
runs on; its FLOPs per launch are the causal pairs of the launch times the
FLOPs per pair of the committed counter record (rocprofv3 instruction
counters), or the library's plan while no record matches the sources.  The
CPU oracle, on its own visit list, is timed on a seeded sample of the same
visits on one core and on every core of the host, and its values are the
accuracy check of the GPU result.  The learned surrogate is measured
against the exact batched kernel on 2000 held-out 64x64 scans (speedup at its
relative L2 error, with its exact judge and fallback), the batched
configuration (256 scans in one call) and the time-sampled simulation (maps
every half dwell over a whole 64x64 scan) and the streaming query (the last
1024 visits of the scan) are reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair E1-terms/s at oracle-matched accuracy; surrogate speedup @≤1% L2 err"
# HBM bytes of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
# valid only while the device sources hash to the recorded value.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_arrival_far_512x512_random_record.txt")
DEVICE_SOURCES = ("dd_device.h", "dd_internal.h", "dd_items.h", "dd_kernels.hip", "dd_queries.cpp",
                  "dd_host.cpp")
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}  # MI355X FP32 / FP64 vector peaks
FP32_NONPACKED_TFLOPS = 78.6  # FP32 vector peak without packed instructions
VALU_ISSUE_PEAK = 256 * 64 * 2.4e9  # lane-instructions/s: one VALU op per lane per clock


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def device_source_hash():
    import hashlib

    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_00294_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record(side):
    """The committed counter record of the far kernels on the 512x512 arrival
    query (HBM bytes of the mixed kernel, VALU lane-instructions per pair of
    both), or None when the kernel sources changed since the counters were
    taken or the workload is not the recorded one."""
    if side != 512 or not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = {}
    with open(TRAFFIC_RECORD) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    if rec.get("source_sha256") != device_source_hash():
        return None
    return rec


def recorded_traffic(precision, side):
    """Bytes per launch of the mixed far kernel from the committed counter
    record, or None."""
    rec = counter_record(side) if precision == "mixed" else None
    return None if rec is None else float(rec["fetch_bytes"]) + float(rec["write_bytes"])


def far_roofline(prec, kern, side):
    """Roofline of the far-region kernel: FLOPs per launch = its causal pairs
    times the FLOPs per pair of the counter record (or of the plan while no
    record matches the sources), over its live HIP-event time; the VALU
    issue rate from the recorded instructions per pair (rocprofv3
    SQ_INSTS_VALU) times the live pair rate."""
    far = kern["arrival_far"]
    far_ms = far["ms"] / max(far["launches"], 1)
    pairs_l = far["pairs"] / max(far["launches"], 1)
    plan_flops = far["flops"] / max(far["launches"], 1)
    rec = counter_record(side)
    tag = "" if prec == "mixed" else "fp64_"
    if rec is not None and tag + "flops_per_pair" in rec:
        far_flops, source = pairs_l * float(rec[tag + "flops_per_pair"]), "counters"
    else:
        far_flops, source = plan_flops, "plan"
    achieved = far_flops / (far_ms * 1e-3) / 1e12
    roofline = {
        "bound": "alu", "kernel": "k_arrival_far32" if prec == "mixed" else "k_arrival_far64",
        "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_TFLOPS[prec], 4),
        "traffic": recorded_traffic(prec, side),
        "avg_launch_ms": round(far_ms, 4),
        "rocprof_avg_launch_ms": float(rec[tag + "rocprof_avg_launch_ms"])
        if rec is not None and tag + "rocprof_avg_launch_ms" in rec else None,
        "pairs_per_launch": pairs_l,
        "flops_per_launch": far_flops,
        "flops_per_pair": far_flops / max(pairs_l, 1.0),
        "flops_source": source,
        "plan_flops_per_pair": plan_flops / max(pairs_l, 1.0),
    }
    if prec == "mixed":
        # the kernels are compiled without packed FP32, so 78.6 TFLOP/s is the FLOP ceiling
        roofline["frac_of_fp32_nonpacked"] = round(achieved / FP32_NONPACKED_TFLOPS, 4)
    rec = counter_record(side)
    key = "valu_lane_instructions_per_pair" if prec == "mixed" else \
        "fp64_valu_lane_instructions_per_pair"
    if rec is not None and key in rec:
        ipp = float(rec[key])
        rate = roofline["pairs_per_launch"] / (far_ms * 1e-3) * ipp
        roofline["valu_issue"] = {"lane_instructions_per_pair": ipp, "achieved": rate,
                                  "peak": VALU_ISSUE_PEAK, "unit": "lane-instructions/s",
                                  "frac": round(rate / VALU_ISSUE_PEAK, 4)}
    return roofline


def time_query(scan, prec, out, steps, warmup, dd, torch):
    for _ in range(warmup):
        scan.arrival(prec, out=out)
    torch.cuda.synchronize()
    for k in ("arrival_far", "arrival_near", "lag_rows", "reduce"):
        dd.profile_read(k, reset=True)
    dd.profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        scan.arrival(prec, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dd.profiling(False)
    kern = {k: dd.profile_read(k, reset=True)
            for k in ("arrival_far", "arrival_near", "lag_rows", "reduce")}
    return (t1 - t0) / steps, kern


def host_cpu():
    """(logical CPUs of the host, CPUs this process may run on, CPU model)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return os.cpu_count() or 1, usable, model


def cpu_baseline(spec, result, floor, seconds, wl):
    """The oracle on its own visit list of the benchmark scan, timed on a
    seeded sample of visits: on one thread (about seconds / 5) and on every
    CPU this process may use (about `seconds`).  Returns the record and the
    largest relative error of the GPU result on the sampled visits."""
    import numpy as np

    import oracle

    oracle.build()
    nproc, usable, model = host_cpu()
    ids = oracle.visits(oracle.RANDOM, spec.nx, spec.ny, seed=spec.seed)
    ora = oracle.Scan(spec.nx, spec.ny, ids, spec.pitch_m, spec.tau_v, spec.sigma_m, spec.D_m2s,
                      spec.Q0_us)
    V = ids.size

    def timed(n_vis, seed, threads):
        idx = wl.sampled_visits(V, n_vis, seed=seed)
        t0 = time.perf_counter()
        ref = ora.psi_arrival(idx, nthreads=threads)
        return idx, ref, time.perf_counter() - t0

    # calibrate on one thread, then size both samples to their targets
    idx, _, dt = timed(8, 101, 1)
    rate1 = max(float(idx.sum()), 1.0) / max(dt, 1e-6)
    n1 = int(max(8, min(V, seconds / 5 * rate1 / (V / 2))))
    idx1, _, dt1 = timed(n1, 5, 1)
    per_core = float(idx1.sum()) / dt1
    n_all = int(max(32, min(V, seconds * per_core * usable / (V / 2))))
    idx, ref, dt = timed(n_all, 7, usable)
    s_pairs = float(idx.sum())
    err = np.abs(result[idx] - ref) / np.maximum(np.abs(ref), floor)
    cpu = {"value": s_pairs / dt, "unit": "pair-terms/s", "cores": usable, "kind": "oracle",
           "per_core": per_core, "nproc": nproc, "cpu_model": model,
           "sample": f"arrival at {idx.size} seeded visits of the same scan ({s_pairs:.3e} pairs, "
                     f"{dt:.1f} s on {usable} threads; one thread: {idx1.size} visits, "
                     f"{float(idx1.sum()):.3e} pairs, {dt1:.1f} s), long double, the oracle's "
                     f"own visit list"}
    return cpu, float(err.max())


def run_oracle_full(j0, j1):
    """The benchmark scan's arrival on the GPU (both precisions) against the
    oracle at every visit j0 <= j < j1 (its own visit list, every host CPU),
    in batches of about 5e8 pairs with a progress line each; one JSON line
    with the largest relative errors.  Two ranges cover the whole scan."""
    import numpy as np
    import torch

    import oracle
    import paper_2507_00294_amd as dd
    from paper_2507_00294_amd import workloads as wl

    oracle.build()
    torch.cuda.set_device(0)
    dd.load_library()
    spec = wl.large_random()
    scan = dd.Scan(**spec.kwargs())
    got = {p: scan.arrival(p).cpu().numpy() for p in ("mixed", "fp64")}
    ids = oracle.visits(oracle.RANDOM, spec.nx, spec.ny, seed=spec.seed)
    assert np.array_equal(ids, scan.visits()), "visit lists differ"
    ora = oracle.Scan(spec.nx, spec.ny, ids, spec.pitch_m, spec.tau_v, spec.sigma_m, spec.D_m2s,
                      spec.Q0_us)
    V = ids.size
    j0, j1 = max(0, j0), min(V, j1)
    _, usable, model = host_cpu()
    pref = spec.Q0_us / (4 * np.pi * spec.D_m2s)
    floors = {"mixed": 1e-30 * pref, "fp64": 1e-250 * pref}
    worst = {p: (0.0, -1) for p in got}
    t_all, j, pairs = 0.0, j0, 0.0
    while j < j1:
        # visits j .. e-1 hold about 5e8 pairs (visit k has k of them)
        e = int(min(j1, max(j + 64, np.sqrt(float(j) * j + 1e9))))
        idx = np.arange(j, e, dtype=np.int64)
        t0 = time.perf_counter()
        ref = ora.psi_arrival(idx, nthreads=usable)
        t_all += time.perf_counter() - t0
        pairs += float(idx.sum())
        for p, g in got.items():
            err = np.abs(g[idx] - ref) / np.maximum(np.abs(ref), floors[p])
            k = int(err.argmax())
            if err[k] > worst[p][0]:
                worst[p] = (float(err[k]), int(idx[k]))
        log(f"[oracle-full] visits {j}..{e - 1} done, {t_all:.0f} s; max rel err mixed "
            f"{worst['mixed'][0]:.3e}, fp64 {worst['fp64'][0]:.3e}")
        j = e
    print(json.dumps({"workload": "arrival query, 512x512 random-order scan (seed 3), every visit "
                                  "in the range against the oracle",
                      "visits": [j0, j1], "pairs": pairs, "oracle_s": t_all, "threads": usable,
                      "cpu_model": model,
                      "max_rel_err": {p: w[0] for p, w in worst.items()},
                      "at_visit": {p: w[1] for p, w in worst.items()}}), flush=True)


def _gpu_time(fn, torch, reps=10):
    import numpy as np

    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def run_configs():
    """The plain FP64 configurations in full and the batched one on sampled
    scans, each against the oracle (own visit lists, every host CPU): GPU
    time, largest relative error, oracle time."""
    import numpy as np
    import torch

    import oracle
    import paper_2507_00294_amd as dd
    from paper_2507_00294_amd import workloads as wl

    oracle.build()
    torch.cuda.set_device(0)
    dd.load_library()
    nproc, usable, model = host_cpu()
    codes = {"raster": oracle.RASTER, "interleaved": oracle.INTERLEAVED,
             "random": oracle.RANDOM, "multiframe": oracle.MULTIFRAME}

    def ora_scan(sp):
        ids = oracle.visits(codes[sp.order], sp.nx, sp.ny, stride=sp.stride, frames=sp.frames,
                            seed=sp.seed)
        return oracle.Scan(sp.nx, sp.ny, ids, sp.pitch_m, sp.tau_v, sp.sigma_m, sp.D_m2s,
                           sp.Q0_us)

    def rel(g, r, sp, fl):
        return float(np.max(np.abs(g - r) / np.maximum(np.abs(r), fl * sp.Q0_us /
                                                       (4 * math.pi * sp.D_m2s))))

    out = {"host": {"nproc": nproc, "threads": usable, "cpu_model": model}}
    # small: 8x8 raster, 64 maps of 32x32 at the end of every dwell
    sp = wl.small_raster()
    sc = dd.Scan(**sp.kwargs())
    m = wl.small_raster_maps(sp)
    args = (m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w, m.h, m.times_s)
    res = {}
    for pr in ("fp64", "mixed"):
        g = sc.damage_map(*args, pr).cpu().numpy()
        res[pr] = (g, _gpu_time(lambda: sc.damage_map(*args, pr), torch))
    t0 = time.perf_counter()
    ref = ora_scan(sp).psi_map(*args, nthreads=usable)
    t_o = time.perf_counter() - t0
    pairs = float(sum(m.w * m.h * min(k, sp.n_visits) for k in range(1, sp.n_visits + 1)))
    out["small"] = {"pairs": pairs, "oracle_s": t_o,
                    **{pr: {"gpu_ms": t * 1e3, "max_rel_err": rel(g, ref, sp, 1e-250 if pr == "fp64"
                                                                   else 1e-30)}
                       for pr, (g, t) in res.items()}}
    log(f"[configs] small: {out['small']}")
    # medium: 16 scans of 32x32 (raster, interleaved s = 2), arrival + 128x128 final map
    specs = wl.medium_scans()
    tg = {"fp64": 0.0, "mixed": 0.0}
    err = {"fp64": 0.0, "mixed": 0.0}
    t_o, pairs = 0.0, 0.0
    for sp in specs:
        sc = dd.Scan(**sp.kwargs())
        fm = wl.medium_final_map(sp)
        margs = (fm.x0_m, fm.y0_m, fm.dx_m, fm.dy_m, fm.w, fm.h, fm.times_s)
        o = ora_scan(sp)
        t0 = time.perf_counter()
        ra = o.psi_arrival(nthreads=usable)
        rm = o.psi_map(*margs, nthreads=usable)
        t_o += time.perf_counter() - t0
        pairs += wl.causal_arrival_pairs(sp.n_visits) + fm.w * fm.h * sp.n_visits
        for pr in ("fp64", "mixed"):
            def both():
                sc.arrival(pr)
                sc.damage_map(*margs, pr)
            tg[pr] += _gpu_time(both, torch, 5)
            fl = 1e-250 if pr == "fp64" else 1e-30
            err[pr] = max(err[pr], rel(sc.arrival(pr).cpu().numpy(), ra, sp, fl),
                          rel(sc.damage_map(*margs, pr).cpu().numpy(), rm, sp, fl))
        sc.close()
    out["medium"] = {"scans": len(specs), "pairs": pairs, "oracle_s": t_o,
                     **{pr: {"gpu_ms": tg[pr] * 1e3, "max_rel_err": err[pr]} for pr in tg}}
    log(f"[configs] medium: {out['medium']}")
    # batched: 256 scans in one call; 16 of them against the oracle on sampled
    # visits (64) and final-map pixels (64)
    specs = wl.batch_scans()
    scans = [dd.Scan(**sp.kwargs()) for sp in specs]
    mask = dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES
    rng = np.random.default_rng(17)
    pick = rng.choice(len(specs), size=16, replace=False)
    bres = {}
    t_o, s_pairs = 0.0, 0.0
    refs = {}
    for k in pick:
        sp = specs[k]
        o = ora_scan(sp)
        idx = wl.sampled_visits(sp.n_visits, 64, seed=int(k))
        pix = rng.choice(sp.nx * sp.ny, size=64, replace=False)
        x, y = (pix % sp.nx) * sp.pitch_m, (pix // sp.nx) * sp.pitch_m
        t = np.full(pix.size, sp.n_visits * sp.tau_v)
        t0 = time.perf_counter()
        refs[k] = (idx, o.psi_arrival(idx, nthreads=usable), pix,
                   o.psi_points(x, y, t, nthreads=usable))
        t_o += time.perf_counter() - t0
        s_pairs += float(idx.sum()) + 64.0 * sp.n_visits
    for pr in ("mixed", "fp64"):
        outs = dd.batch_solve(scans, mask, pr)
        e = 0.0
        for k in pick:
            idx, ra, pix, rf = refs[k]
            o_ = outs[k].cpu().numpy()
            fl = 1e-250 if pr == "fp64" else 1e-30
            e = max(e, rel(o_[idx], ra, specs[k], fl),
                    rel(o_[specs[k].n_visits + pix], rf, specs[k], fl))
        t = _gpu_time(lambda: dd.batch_solve(scans, mask, pr), torch, 3)
        bres[pr] = {"gpu_ms": t * 1e3, "max_rel_err_sampled": e}
    pairs = float(sum(wl.causal_arrival_pairs(s.num_visits) + sp.nx * sp.ny * s.num_visits
                      for s, sp in zip(scans, specs)))
    out["batched"] = {"scans": len(specs), "pairs": pairs, "oracle_sample_pairs": s_pairs,
                      "oracle_sample_s": t_o, **bres}
    log(f"[configs] batched: {out['batched']}")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--side", type=int, default=512)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-versus-exact measurement")
    ap.add_argument("--surrogate-maps", type=int, default=2000)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-configuration measurement")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the time-sampled simulation measurement")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streaming (visit range) measurement")
    ap.add_argument("--no-visits", action="store_true",
                    help="skip the general visit list measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes three times "
                         "(reference for the HBM byte counters) and exit")
    ap.add_argument("--configs", action="store_true",
                    help="only measure the small, medium and batched configurations against "
                         "the oracle (GPU time, error, oracle time) and print one JSON line")
    ap.add_argument("--oracle-full", type=int, nargs=2, metavar=("J0", "J1"),
                    help="only compare the benchmark scan's arrival (both precisions) with the "
                         "oracle at every visit J0 <= j < J1 and print one JSON line")
    args = ap.parse_args()
    if args.oracle_full:
        run_oracle_full(*args.oracle_full)
        return
    if args.configs:
        run_configs()
        return
    if args.copy_calibration:
        import torch

        n = args.copy_calibration // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"[bench] copied {4 * n} bytes three times")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_00294_amd as dd
    from paper_2507_00294_amd import workloads as wl

    torch.cuda.set_device(0)
    dd.load_library()
    spec = wl.large_random(args.side)
    scan = dd.Scan(**spec.kwargs())
    V = scan.num_visits
    pairs = wl.causal_arrival_pairs(V)
    out = torch.empty(V, dtype=torch.float64, device="cuda")
    prec = args.precision
    log(f"[bench] {args.side}x{args.side} random scan, V={V}, pairs={pairs:.4e}, {prec}")

    sec, kern = time_query(scan, prec, out, args.steps, args.warmup, dd, torch)
    value = pairs / sec
    log(f"[bench] {prec}: {sec * 1e3:.3f} ms/step, {value:.4e} pairs/s")
    roofline = far_roofline(prec, kern, args.side)
    result = out.cpu().numpy()
    # Streaming: psi at the last 1024 visits of the scan (the visits just made,
    # the most expensive 1024 of the scan), latency of one call.
    stream = None
    if not args.no_stream:
        j0 = V - 1024
        tail = torch.empty(V - j0, dtype=torch.float64, device="cuda")
        scan.arrival_range(j0, V, prec, out=tail)
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            t0 = time.perf_counter()
            scan.arrival_range(j0, V, prec, out=tail)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t_st = float(np.median(ts))
        pairs_st = float(sum(range(j0, V)))
        dev = float(np.max(np.abs(tail.cpu().numpy() - result[j0:]) / np.abs(result[j0:])))
        stream = {"ms_per_call": t_st * 1e3, "visits": V - j0, "pairs_per_call": pairs_st,
                  "value": pairs_st / t_st, "unit": "pair-terms/s",
                  "max_rel_diff_vs_full_query": dev,
                  "workload": "arrival at the last 1024 visits of the same scan, one call "
                              "(host to host latency with the scan tables resident)"}
        log(f"[bench] streaming: last {V - j0} visits in {t_st * 1e3:.3f} ms")

    # The other precision on the same workload, for context.
    other = "fp64" if prec == "mixed" else "mixed"
    sec_o, kern_o = time_query(scan, other, out, max(2, args.steps // 4), 1, dd, torch)
    other_res = out.cpu().numpy()
    floor = 1e-30 * spec.Q0_us / (4 * math.pi * spec.D_m2s)
    diff = np.abs(result - other_res) / np.maximum(np.abs(other_res if other == "fp64" else result),
                                                  floor)
    log(f"[bench] {other}: {sec_o * 1e3:.3f} ms/step; max rel diff mixed vs fp64 {diff.max():.3e}")

    # Batched configuration: 256 scans of uneven size, order and physics in one
    # call (arrival at every visit and the final map at the probes).
    bat = None
    if not args.no_batched:
        specs_b = wl.batch_scans()
        scans_b = [dd.Scan(**sp.kwargs()) for sp in specs_b]
        mask = dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES
        dd.batch_solve(scans_b, mask, prec)  # builds the scans' device tables
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            dd.batch_solve(scans_b, mask, prec)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t_b = float(np.median(ts))
        vs = [sb.num_visits for sb in scans_b]
        pairs_b = float(sum(wl.causal_arrival_pairs(v) + sp.nx * sp.ny * v
                            for v, sp in zip(vs, specs_b)))
        bat = {"value": pairs_b / t_b, "unit": "pair-terms/s", "ms_per_call": t_b * 1e3,
               "pairs_per_call": pairs_b, "precision": prec, "scans": len(scans_b),
               "workload": "256 scans (seed 4): side U{16..256}, order uniform over raster / "
                           "interleaved / random / 4-frame, dwell 10^U(-7,-5) s, D 10^U(-15,-11) "
                           "m^2/s, sigma U[0.2,1] nm; arrival at every visit + final map at the "
                           "probes, one call"}
        log(f"[bench] batched: {t_b * 1e3:.1f} ms/call, {bat['value']:.4e} pairs/s")
        for sb in scans_b:
            sb.close()

    # Time-sampled simulation (the paper's workload of maps every time step on
    # a sampling grid): a 64x64 raster scan, maps of 128x128 pixels at half
    # the pitch every half dwell over the whole scan (8192 maps).
    swp = None
    if not args.no_sweep:
        sp = wl.ScanSpec(64, 64, "raster", 1e-9, 1e-6, 0.5e-9, 2.5e-13, 1.0)
        sc = dd.Scan(**sp.kwargs())
        n_t, w = 2 * sp.n_visits, 128
        dt = sp.tau_v / 2
        out = torch.empty((n_t, w, w), dtype=torch.float64, device="cuda")
        sc.damage_sweep(0.0, 0.0, 0.5e-9, 0.5e-9, w, w, 0.0, dt, n_t, prec, out=out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            sc.damage_sweep(0.0, 0.0, 0.5e-9, 0.5e-9, w, w, 0.0, dt, n_t, prec, out=out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t_s = float(np.median(ts))
        # visits started before t = k dt: ceil(k / 2), at most V
        started = np.minimum((np.arange(n_t) + 1) // 2, sp.n_visits)
        pairs_s = float(w * w * started.sum())
        swp = {"value": pairs_s / t_s, "unit": "pair-terms/s", "ms_per_call": t_s * 1e3,
               "pairs_per_call": pairs_s, "maps": n_t, "precision": prec,
               "workload": "time-sampled simulation: 64x64 raster scan (pitch 1 nm, sigma 0.5 nm, "
                           "dwell 1 us, D 2.5e-13 m^2/s), 128x128 maps at 0.5 nm every half "
                           "dwell from t = 0 to the end of the scan, one call"}
        log(f"[bench] sweep: {n_t} maps in {t_s * 1e3:.1f} ms, {swp['value']:.4e} pairs/s")
        # Visualisation of the sweep: every frame to an RGB image (automatic
        # log range per frame, iso-lines per decade), one call.
        rgb = torch.empty((n_t, w, w, 3), dtype=torch.uint8, device="cuda")
        dd.render_maps(out, decades=6.0, levels=6, out=rgb)
        torch.cuda.synchronize()
        tr = []
        for _ in range(5):
            t0 = time.perf_counter()
            dd.render_maps(out, decades=6.0, levels=6, out=rgb)
            torch.cuda.synchronize()
            tr.append(time.perf_counter() - t0)
        t_r = float(np.median(tr))
        px = float(n_t * w * w)
        swp["render"] = {"ms_per_call": t_r * 1e3, "frames": n_t, "pixels": px,
                         "bytes_per_call": px * 11.0, "achieved_GBs": px * 11.0 / t_r / 1e9,
                         "peak_GBs": 8000.0, "frac": px * 11.0 / t_r / 8e12,
                         "workload": "the sweep's 8192 frames of 128x128 to 8-bit RGB: per pixel "
                                     "8 bytes of psi read, 3 written (automatic log range over 6 "
                                     "decades per frame, iso-line per decade)"}
        log(f"[bench] render: {n_t} frames in {t_r * 1e3:.2f} ms")
        del rgb
        del out
        sc.close()

    # General visit list: a 256x256 raster with per-visit dwell jitter and a
    # flyback dead time after every line; psi at every visit when it starts
    # and the final map at the probes, one call each, in FP64 and mixed.
    gvl = None
    if not args.no_visits:
        vl = wl.visit_list("flyback", 256, 256, seed=21)
        gv = dd.Visits(vl.x_m, vl.y_m, vl.t0_s, vl.dwell_s, **vl.kwargs())
        arr = torch.empty(vl.n_visits, dtype=torch.float64, device="cuda")
        fin = torch.empty((1, 256, 256), dtype=torch.float64, device="cuda")
        margs = (0.0, 0.0, 1e-9, 1e-9, 256, 256, [vl.t_end])
        pa = float(wl.causal_arrival_pairs(vl.n_visits))
        pm = float(vl.n_visits) * 256 * 256
        res = {}
        for pr in ("fp64", "mixed"):
            gv.arrival(pr, out=arr)
            gv.damage_map(*margs, pr, out=fin)
            torch.cuda.synchronize()
            ta, tm = [], []
            for _ in range(3):
                t0 = time.perf_counter()
                gv.arrival(pr, out=arr)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                gv.damage_map(*margs, pr, out=fin)
                torch.cuda.synchronize()
                ta.append(t1 - t0)
                tm.append(time.perf_counter() - t1)
            t_a, t_m = float(np.median(ta)), float(np.median(tm))
            res[pr] = {"value": (pa + pm) / (t_a + t_m), "ms_per_call": (t_a + t_m) * 1e3,
                       "arrival_ms": t_a * 1e3, "map_ms": t_m * 1e3}
            log(f"[bench] visit list {pr}: arrival {t_a * 1e3:.1f} ms, final map "
                f"{t_m * 1e3:.1f} ms, {res[pr]['value']:.4e} pairs/s")
        gvl = dict(res["fp64"], unit="pair-terms/s", pairs_per_call=pa + pm, precision="fp64",
                   mixed=res["mixed"],
                   workload="general visit list: 256x256 raster (pitch 1 nm, sigma 0.5 nm, "
                            "D 2.5e-13 m^2/s), dwell 1 us x U(0.5, 1.5) per visit, 64 us "
                            "flyback after every line (seed 21); arrival at every visit + "
                            "final map at the probes")
        gv.close()
        # Many small lists in one call: 512 sparse lists (a random quarter of a
        # 32x32 lattice each, D 10^U(-14,-11) m^2/s), arrival at every visit,
        # against the same lists one call each.
        rng = np.random.Generator(np.random.PCG64(27))
        vls = [wl.visit_list("sparse", 32, 32, seed=100 + k,
                             D_m2s=float(10.0 ** rng.uniform(-14, -11))) for k in range(512)]
        lists = [dd.Visits(v.x_m, v.y_m, v.t0_s, v.dwell_s, **v.kwargs()) for v in vls]
        flat = torch.empty(sum(v.n_visits for v in vls), dtype=torch.float64, device="cuda")
        dd.visits_batch_arrival(lists, "mixed", out=flat)
        for g_ in lists:
            g_.arrival("mixed")
        torch.cuda.synchronize()
        tb, tl = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            dd.visits_batch_arrival(lists, "mixed", out=flat)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for g_ in lists:
                g_.arrival("mixed")
            torch.cuda.synchronize()
            tb.append(t1 - t0)
            tl.append(time.perf_counter() - t1)
        pb = float(sum(wl.causal_arrival_pairs(v.n_visits) for v in vls))
        gvl["batched_lists"] = {
            "lists": len(vls), "precision": "mixed", "pairs_per_call": pb,
            "ms_per_call": float(np.median(tb)) * 1e3,
            "ms_one_call_per_list": float(np.median(tl)) * 1e3,
            "value": pb / float(np.median(tb)), "unit": "pair-terms/s",
            "workload": "512 sparse visit lists (a random quarter of a 32x32 lattice each, seeds "
                        "100..611, D 10^U(-14,-11) m^2/s), arrival at every visit, one call"}
        log(f"[bench] 512 visit lists: {np.median(tb) * 1e3:.2f} ms in one call vs "
            f"{np.median(tl) * 1e3:.2f} ms one call per list")
        for g_ in lists:
            g_.close()

    # Learned surrogate against the exact batched kernel on the held-out 64x64
    # test scans (both timed end to end, scans' device tables built first).
    sur = None
    if not args.no_surrogate:
        from paper_2507_00294_amd import surrogate as sg

        if os.path.exists(sg.DEFAULT_WEIGHTS):
            net = dd.UNet(0)
            sg.load_weights(net)
            res = sg.evaluate(net, wl.surrogate_scans(args.surrogate_maps, seed=6), 0.02, "mixed",
                              repeats=3, extra_tols=(0.01,))
            net.close()
            sur = {"metric": "surrogate speedup over the exact batched kernel at <= 1% mean "
                             "relative L2 error", "speedup": res["speedup"],
                   "rel_l2_mean": res["rel_l2_mean"], "rel_l2_p95": res["rel_l2_p95"],
                   "rel_l2_max": res["rel_l2_max"], "fallback_rate": res["fallback_rate"],
                   "exact_ms": res["exact_s"] * 1e3, "surrogate_ms": res["surrogate_s"] * 1e3,
                   "network_only_ms": res["network_only_s"] * 1e3,
                   "network_only_rel_l2_mean": res["network_only_rel_l2_mean"],
                   "maps": res["maps"], "spot_tol": res["spot_tol"],
                   "judge": "exact values on the 8x8 probe sub-grid of stride 9 per map; "
                            "rel_l2_max is the worst accepted map (rejected maps are exact)",
                   "at_spot_tol_0.01": res["at_spot_tol"][0.01],
                   "workload": "final damage maps of 64x64 scans, batched-config sampling "
                               "(seed 6), mixed precision exact path"}
            log(f"[bench] surrogate: x{sur['speedup']:.2f} at rel L2 {sur['rel_l2_mean']:.4f} "
                f"(fallback {sur['fallback_rate']:.3f})")
        else:
            log("[bench] surrogate weights missing; surrogate measurement skipped")

    cpu = None
    max_err = None
    if not args.no_cpu_baseline:
        cpu, max_err = cpu_baseline(spec, result, floor, args.cpu_seconds, wl)
        log(f"[bench] oracle: {cpu['value']:.3e} pairs/s on {cpu['cores']} threads "
            f"({cpu['per_core']:.3e} on one); max rel err GPU vs oracle {max_err:.3e}")

    line = {
        "metric": METRIC, "value": value, "unit": "pair-terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"arrival query, {args.side}x{args.side} random-order scan "
                               f"(seed 3), pitch 1 nm, sigma 0.4 nm, dwell 0.5 us, D 1e-12 m^2/s",
                   "visits": V, "pairs_per_step": pairs, "precision": prec},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": max_err,
        "other_precision": {"precision": other, "ms_per_step": sec_o * 1e3,
                            "value": pairs / sec_o, "max_rel_diff_mixed_vs_fp64": float(diff.max()),
                            "roofline": far_roofline(other, kern_o, args.side)},
        "kernels_ms_per_step": {k: v["ms"] / max(v["launches"], 1) for k, v in kern.items()},
        "batched": bat,
        "sweep": swp,
        "visit_list": gvl,
        "streaming": stream,
        "surrogate": sur,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
