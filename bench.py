#!/usr/bin/env python3
"""Benchmark of the hot path: a batched wavelength sweep of the quasistatic LSPR BEM.

Workload (default): silver sphere R = 10 nm with 32768 panels, 64 wavelengths 350-420 nm
(Drude silver, water), treecode theta = 0.5, P = 8, K = 4, K_fine = 19, N_k = 9, FP32 far-field
kernels, FP64 GMRES (tol 1e-5).  One step = the whole path on one batch: geometry set-up
(panels, Morton sort, octree, lists, near-singular table, right-hand side) from meshes already
in device memory, the batched GMRES over all 64 wavelengths, dipole moments and extinction
cross-sections.

Printed: one JSON line with the throughput in wavelength-solves per second (wavelengths whose
C_ext is within 1e-4 of the FP64 reference, per second), the roofline position of the dominant
kernel (measured with HIP events on its launch stream during the timed steps) and the oracle's
CPU throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("treecode matvec Gpair/s; wavelength-solves/s at 1e-4 rel err vs FP64; p50/p99")
PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X datasheet, dense FP32 matrix cores (measured sustained: 155)
PEAK_FP64_MFMA_TFLOPS = 78.6    # MI355X datasheet, dense FP64 matrix cores
PEAK_FP32_VALU_TFLOPS = 157.3   # MI355X datasheet, FP32 vector (packed); 78.6 unpacked
PEAK_HBM_GBS = 8000.0
WIDTH_BINS = ((1, 8), (9, 16), (17, 32), (33, 64))  # wavelengths per far-field launch


def precomputed_flops(info, op):
    """Geometry-only work the matrix-core path does once per geometry instead of per launch:
    far-rule kernel values (15 flops per node, 9 per pair) and Taylor coefficients (about 10
    flops per term)."""
    return (float(info["p2p_pairs"]) * (15.0 * op["k_far"] + 9.0)
            + float(info["m2p_pairs"]) * 10.0 * info["n_terms"])


def width_rows(lspr, name, peak_tflops, timed):
    """Roofline position of the far-field launches by width.  Arithmetic intensity = executed
    flops / algorithmic bytes (the tile store read once, densities, moments, sums); below the
    ridge (peak flop/s over 8 TB/s) a launch is bound by HBM and its fraction is GB/s over
    8 TB/s, above it by the matrix cores and its fraction is TFLOP/s over the peak."""
    rows = []
    ridge = peak_tflops * 1e12 / (PEAK_HBM_GBS * 1e9)
    for lo, hi in WIDTH_BINS:
        q = timed[(name, lo, hi)]
        if q["launches"] == 0 or q["total_ms"] <= 0:
            continue
        t = q["total_ms"] * 1e-3
        tf, gbs = q["flops"] / t / 1e12, q["bytes"] / t / 1e9
        hbm = q["flops"] / max(q["bytes"], 1.0) < ridge
        rows.append({"wavelengths": f"{lo}-{hi}", "launches": q["launches"],
                     "avg_launch_ms": q["total_ms"] / q["launches"],
                     "tflops": tf, "gbs": gbs, "flop_per_byte": q["flops"] / max(q["bytes"], 1.0),
                     "bound": "hbm" if hbm else "mfma",
                     "frac": gbs / PEAK_HBM_GBS if hbm else tf / peak_tflops})
    return rows


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, n_rows=768, seed=0, iters_full=None):
    """The oracle (numpy FP64 dense BEM, unchanged) timed on a bounded sample of this workload.

    Sample: `n_rows` random target rows of the dense single/double-layer matrices at full size
    (all 4N far-rule nodes, near-singular and singular terms) and one dense complex product of
    those rows of the system matrix.  Extrapolated per wavelength-solve:
    (row assembly x N / n_rows) / n_lambda + (iterations + 1) x (row product x 2N / n_rows),
    with the iteration count of this system itself (`iters_full`: the mean of the GPU's FP64
    solves of the same workload at the same tolerance, one wavelength per solve); without it,
    the oracle's own GMRES count on the same sphere coarsened to 512 panels.
    """
    import oracle
    from threadpoolctl import threadpool_info
    from lspr_inputs import octasphere

    v, t = w.surfaces[0]
    N = len(t)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(N, n_rows, replace=False))
    op = w.op
    t0 = time.perf_counter()
    V, K = oracle.operator_rows(v, t, rows, op["k_far"], op["k_fine"], op["n_k"], op["threshold"])
    t_rows = time.perf_counter() - t0
    # one block of system rows [n_rows, 2N] times a vector, as the oracle's GMRES does
    A_rows = np.concatenate([0.5 * (np.arange(N)[None, :] == rows[:, None]) - K,
                             V * (w.eps_surface[0, 0] / w.eps_medium[0])], 1)
    x = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    t0 = time.perf_counter()
    for _ in range(3):
        A_rows @ x
    t_mv = (time.perf_counter() - t0) / 3
    if iters_full is not None:
        iters = float(iters_full)
        how = (f"the {N}-panel system's own GMRES iteration count ({iters:.1f}, mean of the "
               f"GPU's FP64 treecode solves of this workload at tol {w.gmres['tol']:g}, one "
               f"wavelength per solve)")
    else:
        vs, ts = octasphere(8, 10.0)
        mid = len(w.lambdas) // 2
        t0 = time.perf_counter()
        r = oracle.solve(vs, ts, np.zeros(len(ts), int), w.lambdas[mid:mid + 1],
                         w.eps_medium[mid:mid + 1], w.eps_surface[mid:mid + 1], w.e_field,
                         op["k_far"], op["k_fine"], op["n_k"], op["threshold"], method="gmres",
                         tol=w.gmres["tol"], restart=w.gmres["restart"],
                         max_iter=w.gmres["max_iter"])
        iters = float(r["iters"][0])
        how = (f"the oracle's unpreconditioned GMRES iteration count ({iters:.0f}) on the "
               f"512-panel sphere at {w.lambdas[mid]:.1f} nm "
               f"({time.perf_counter() - t0:.1f} s)")
    per_solve = (t_rows * N / n_rows) / len(w.lambdas) + (iters + 1) * t_mv * (2 * N / n_rows)
    blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {
        "value": 1.0 / per_solve, "unit": "wavelength-solves/s", "cores": int(blas_threads),
        "kind": "oracle",
        "sample": (f"{n_rows} of {N} target rows of the dense V,K matrices ({t_rows:.1f} s) and "
                   f"one product of those system rows ({t_mv * 1e3:.1f} ms), extrapolated to one "
                   f"wavelength-solve with {how}; row assembly single-threaded numpy, products "
                   f"use {blas_threads} BLAS threads"),
        "seconds_per_solve": per_solve,
    }


def _build_request(args):
    from lspr_inputs import serving_request
    return serving_request(*args)


def serving_requests(n_requests, seed=5, workers=12):
    """The first n_requests of the seeded Poisson stream (arrival offsets, workloads); meshes are
    built in a process pool (each request has its own generator, so the stream is unchanged)."""
    from lspr_inputs import serving_stream_params
    params = list(serving_stream_params(seed=seed, n_requests=n_requests))
    arrivals = np.array([p[0] for p in params])
    jobs = [(seed,) + tuple(p[1:]) for p in params]
    if n_requests <= 16 or workers <= 1:
        reqs = [_build_request(j) for j in jobs]
    else:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            reqs = pool.map(_build_request, jobs, chunksize=1)
    return arrivals, reqs


def serving_leg(lspr, n_requests, seed=5, max_slots=4, load=0.8, n_burst=None):
    """Request-serving leg: the first n_requests of the seeded Poisson stream (spheres of
    2048-131072 panels with 0-4 analytes at 0.5-3 nm, 1-64 wavelengths each) through the
    request server.  A burst of the first n_burst requests (all submitted at once; default all
    of them) gives the saturated throughput; then all n_requests arrive with the stream's own
    exponential gaps rescaled to `load` times that rate, and the latency (completion - arrival)
    of each is recorded: p50 and p99 are over those n_requests samples."""
    arrivals, reqs = serving_requests(n_requests, seed)
    n_burst = len(reqs) if n_burst is None else min(n_burst, len(reqs))
    gaps = np.diff(arrivals, prepend=0.0)
    sv = lspr.Server(max_slots=max_slots)

    def submit(w):
        return sv.submit(w.surfaces, w.lambdas, w.eps_medium, w.eps_surface, w.e_field,
                         op=lspr.op_params(**w.op), gmres=lspr.gmres_params(**w.gmres))

    try:
        t0 = time.perf_counter()
        burst = [sv.poll(t, wait=True) for t in [submit(w) for w in reqs[:n_burst]]]
        burst_s = time.perf_counter() - t0
        burst_stats = sv.stats()
        rate = load * n_burst / burst_s
        log(f"[bench] serving burst: {n_burst} requests in {burst_s:.1f} s; pacing "
            f"{len(reqs)} requests at {rate:.3f} req/s")
        arrive = np.cumsum(gaps) - gaps[0]
        arrive *= (1.0 / rate) / max(np.mean(gaps), 1e-12)
        start = time.perf_counter()
        tickets = []
        for k, w in enumerate(reqs):
            while time.perf_counter() - start < arrive[k]:
                time.sleep(0.0005)
            tickets.append(submit(w))
            if (k + 1) % 25 == 0:
                log(f"[bench] serving: {k + 1}/{len(reqs)} submitted")
        paced = [sv.poll(t, wait=True) for t in tickets]
        paced_s = time.perf_counter() - start
        paced_stats = sv.stats()
    finally:
        sv.close()
    lat = np.array([r["latency_s"] for r in paced])
    ok_b = [r["status"] == lspr.LSPR_OK for r in burst]
    ok_p = [r["status"] == lspr.LSPR_OK for r in paced]
    n_ok_lambda = int(sum(r["n_lambda"] for r, good in zip(burst, ok_b) if good))
    return {
        "requests": len(reqs), "burst_requests": n_burst, "max_slots": max_slots,
        "panels": {"min": int(min(r["n_panels"] for r in paced)),
                   "max": int(max(r["n_panels"] for r in paced))},
        "wavelengths": int(sum(r["n_lambda"] for r in paced)),
        "converged": int(sum(ok_p)),
        "burst_s": burst_s, "burst_requests_per_s": n_burst / burst_s,
        "burst_wavelength_solves_per_s": n_ok_lambda / burst_s,
        "max_concurrent": int(max(burst_stats["max_active"], paced_stats["max_active"])),
        "paced_rate_requests_per_s": rate,
        "paced_s": paced_s,
        "paced_wavelength_solves_per_s": int(sum(r["n_lambda"] for r, g in zip(paced, ok_p)
                                                 if g)) / paced_s,
        "latency_samples": int(len(lat)),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
        "estimate_violations": int(paced_stats["estimate_violations"]),
        "precision": reqs[0].op["precision"],
    }


def serving_main(args):
    """--serving-only: the request stream alone (metric: served wavelength-solves/s at the paced
    rate, with p50/p99 latency over every paced request)."""
    import torch
    from paper_1812_10722_amd import lspr
    torch.cuda.set_device(0)
    n = 200 if args.serving_requests is None else args.serving_requests
    n_burst = 32 if args.serving_burst is None else args.serving_burst
    log(f"[bench] serving stream: {n} requests, burst of {n_burst} ...")
    srv = serving_leg(lspr, n, n_burst=n_burst)
    line = {"metric": "served wavelength-solves/s at 0.8 of the saturated request rate; p50/p99 "
                      "request latency", "value": srv["paced_wavelength_solves_per_s"],
            "unit": "wavelength-solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "fp32+fp64", "data": "synthetic (seeded Poisson request stream)",
            "config": {"workload": f"serving_stream_seed5_first{n}", "requests": n,
                       "max_slots": srv["max_slots"], "parallelism": "single GPU"},
            "latency_p50_s": srv["latency_p50_s"], "latency_p99_s": srv["latency_p99_s"],
            "serving": srv}
    log(f"[bench] serving: burst {srv['burst_requests_per_s']:.3f} req/s; {n} paced at "
        f"{srv['paced_rate_requests_per_s']:.3f} req/s: p50 {srv['latency_p50_s']:.2f} s, p99 "
        f"{srv['latency_p99_s']:.2f} s")
    print(json.dumps(line), flush=True)


def traffic_entry(kernel_file, name):
    """HBM bytes per launch from rocprofv3 counter runs, valid only for the same kernel source."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")  # written from rocprofv3 --pmc runs
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(kernel_file, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec


def record_traffic(fetch_csv, write_csv, kernel_file, name, workload):
    """Turn two rocprofv3 counter passes (FETCH_SIZE, then WRITE_SIZE, each over a run with
    --copy-calibration) into the traffic record of the far-field kernel.  The counters are in KiB
    per dispatch; each is scaled by what it reads for a kernel of known traffic in the same run
    (the 256 MiB fill writes 256 MiB; the 256 MiB elementwise multiply reads 256 MiB)."""
    import collections
    import csv
    import re

    def load(path, counter):
        rows = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                rows[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return rows

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    known_kib = 256.0 * 1024.0

    def only(rows, tag):
        hits = [v for k, v in rows.items() if tag in k]
        if len(hits) != 1 or len(hits[0]) != 1:
            raise SystemExit(f"calibration kernel {tag!r} not found exactly once")
        return hits[0][0]

    fetch_scale = known_kib / only(fetch, "AUnaryFunctor")
    write_scale = known_kib / only(write, "FillFunctor")
    per, total_b, total_n = {}, 0.0, 0
    for k in sorted(fetch):
        # the FP32 instances (wide launches run k_far_wide): the kernel the roofline times
        if "k_far_tiles_op<float" not in k and "k_far_wide<" not in k:
            continue
        f, wr = fetch[k], write.get(k, [])
        if len(f) != len(wr):
            raise SystemExit(f"dispatch counts differ between the passes for {k}")
        b = [fv * 1024 * fetch_scale + wv * 1024 * write_scale for fv, wv in zip(f, wr)]
        m = re.search(r"(k_\w+(?:<[^()]*>)?)\(", k)
        short = m.group(1) if m else k
        per[short] = {"dispatches": len(f), "fetch_kib_raw_mean": float(np.mean(f)),
                      "write_kib_raw_mean": float(np.mean(wr)),
                      "bytes_scaled_mean": float(np.mean(b))}
        total_b += sum(b)
        total_n += len(b)
    if not total_n:
        raise SystemExit("no far-field dispatches in the counter files")
    rec = {"kernel": "k_far_wide + k_far_tiles_op<float>", "workload": workload,
           "source_sha256": hashlib.sha256(open(kernel_file, "rb").read()).hexdigest(),
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "bytes_per_launch": total_b / total_n, "per_instance": per}
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"FETCH_SIZE x {fetch_scale:.3f}, WRITE_SIZE x {write_scale:.3f}")
    print("| instance | dispatches | FETCH_SIZE KiB (raw mean) | WRITE_SIZE KiB (raw mean) | "
          "scaled bytes per launch |")
    print("|---|---:|---:|---:|---:|")
    for k, v in per.items():
        print(f"| `{k}` | {v['dispatches']} | {v['fetch_kib_raw_mean']:.0f} | "
              f"{v['write_kib_raw_mean']:.0f} | {v['bytes_scaled_mean'] / 1e9:.3f} GB |")
    print(f"Average over all far-field launches: {rec['bytes_per_launch'] / 1e9:.3f} GB; "
          f"written {path}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_32k_sweep")
    ap.add_argument("--precision", choices=("fp32", "fp64", "fp32_refine64", "fp32_lead64"),
                    help="override the workload's product precision")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="inner tolerance of fp32_refine64, or the FP64-to-FP32 switch level of "
                         "fp32_lead64 (default: the library's)")
    ap.add_argument("--tol", type=float, default=None, help="override the GMRES tolerance")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run a workload's fixed treecode settings instead of the autotuner's")
    ap.add_argument("--op", action="append", default=[], metavar="KEY=VALUE",
                    help="override an operator parameter of the workload (p, theta, ncrit, "
                         "m2p_min_panels, stream_narrow, pair_operators, pair_narrow, ...); "
                         "implies --no-autotune")
    ap.add_argument("--serving-requests", type=int, default=None,
                    help="requests of the serving leg (default 16, or 200 with --serving-only; "
                         "0 skips it)")
    ap.add_argument("--serving-burst", type=int, default=None,
                    help="requests of the burst that measures the saturated rate (default: all "
                         "of them, or 32 with --serving-only)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving stream: a burst prefix measures the saturated rate, "
                         "then the requests arrive paced at 0.8 of it; one JSON line with p50/p99 "
                         "latency over all of them")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the FP64 reference solve and the one-at-a-time FP64 comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device-to-device copy of 256 MiB (a kernel of known "
                         "traffic, used to scale hardware byte counters)")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: write the far-field traffic record from two rocprofv3 "
                         "counter files (FETCH_SIZE, WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.traffic_record:
        from lspr_inputs import workload
        record_traffic(*args.traffic_record,
                       os.path.join(ROOT, "paper_1812_10722_amd", "csrc", "operator.hip"), "far",
                       workload(args.workload).name)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the library targets "
              "a single MI355X; a split of the wavelengths over several GPUs is designed but "
              "not built.", file=sys.stderr)
        sys.exit(2)
    if args.serving_only:
        return serving_main(args)

    import torch
    from lspr_inputs import workload
    from paper_1812_10722_amd import lspr

    torch.cuda.set_device(0)
    w = workload(args.workload)
    op = dict(w.op)
    gm = dict(w.gmres)
    if args.precision:
        op["precision"] = args.precision
    for kv in args.op:
        k, v = kv.split("=", 1)
        op[k] = (v.lower() == "true") if v.lower() in ("true", "false") else \
            (int(v) if v.lstrip("-").isdigit() else (float(v) if k == "theta" else v))
        args.no_autotune = True
    if args.inner_tol is not None:
        gm["inner_tol"] = args.inner_tol
    if args.tol is not None:
        gm["tol"] = args.tol
    lam, em, es, ef = w.lambdas, w.eps_medium, w.eps_surface, w.e_field
    dev = [(torch.as_tensor(v).cuda(), torch.as_tensor(t).cuda()) for v, t in w.surfaces]
    stream = torch.cuda.current_stream()
    tuned = None
    if w.tune and not args.no_autotune:
        # untimed: the library's autotuner picks P, theta, N_crit and the kernel schedule under
        # the workload's bound, at the middle wavelength's permittivities
        mid = len(lam) // 2
        t0 = time.perf_counter()
        top, entries, ok = lspr.lspr_autotune(dev, w.tune["n_cols"], em[mid], es[mid],
                                              max_rel_err=w.tune["max_rel_err"],
                                              op=lspr.op_params(**op))
        tuned = {"seconds": time.perf_counter() - t0, "met_bound": bool(ok),
                 "max_rel_err": w.tune["max_rel_err"], "n_cols": w.tune["n_cols"],
                 "p": top.p, "theta": top.theta, "ncrit": top.ncrit,
                 "m2p_min_panels": top.m2p_min_panels, "flags": top.flags,
                 "candidates": len(entries),
                 "chosen": next((e for e in entries if e["p"] == top.p and e["ncrit"] == top.ncrit
                                 and abs(e["theta"] - top.theta) < 1e-12
                                 and e["m2p_min_panels"] == top.m2p_min_panels
                                 and e["flags"] == top.flags), None)}
        op.update(p=top.p, theta=top.theta, ncrit=top.ncrit, m2p_min_panels=top.m2p_min_panels,
                  stream_narrow=bool(top.flags & lspr.LSPR_STREAM_NARROW),
                  pair_operators=bool(top.flags & lspr.LSPR_PAIR_OPERATORS))
        log(f"[bench] autotune: P={top.p} theta={top.theta} ncrit={top.ncrit} "
            f"m2p_min_panels={top.m2p_min_panels} flags={top.flags} ({tuned['seconds']:.1f} s, "
            f"{len(entries)} candidates)")

    def step(op_kw, lam_, em_, es_, gm_kw):
        g = lspr.Geometry(dev, validate=False, **op_kw)
        out = g.solve(lam_, em_, es_, ef, allow_noconv=True, **gm_kw)
        info = g.info()
        g.close()
        return out, info

    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)  # elementwise kernel: reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del a, b
    assert lspr.lspr_mesh_validate(w.surfaces) == lspr.LSPR_OK
    log(f"[bench] workload {w.name}: N={w.n_panels}, {len(lam)} wavelengths")
    for k in range(args.warmup):
        out, info = step(op, lam, em, es, gm)
        log(f"[bench] warmup {k}: iters {out['iters'].min()}-{out['iters'].max()}")
    # the timed steps record HIP events around the far-field launches only (the roofline);
    # the breakdown of a step by phase comes from one more, untimed step with every scope
    lspr.lspr_profile_reset()
    lspr.lspr_profile_enable(2)
    times = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        out, info = step(op, lam, em, es, gm)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[bench] step {k}: {times[-1] * 1e3:.1f} ms, iters {out['iters'].min()}-"
            f"{out['iters'].max()}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    lspr.lspr_profile_enable(False)
    far_timed = lspr.lspr_profile_query("far")
    width_timed = {(name, lo, hi): lspr.lspr_profile_query_width(name, lo, hi)
                   for name in ("far", "far64") for lo, hi in WIDTH_BINS}
    lspr.lspr_profile_reset()
    lspr.lspr_profile_enable(1)
    step(op, lam, em, es, gm)
    torch.cuda.synchronize()
    lspr.lspr_profile_enable(False)
    prof = {n: lspr.lspr_profile_query(n)
            for n in ("far", "far64", "p2m", "p2m64", "near", "matvec", "arnoldi", "setup")}
    n_matvec = prof["matvec"]["launches"]

    # accuracy against the FP64 reference (dense direct FP64 on the GPU, validated against the
    # oracle by the parity tests), and the plain FP64 one-wavelength-at-a-time form
    accuracy = None
    fp64_b1 = None
    if not args.no_reference:
        ref_op = dict(op, method="dense", precision="fp64")
        ref, _ = step(ref_op, lam, em, es, dict(gm, tol=1e-10, restart=100, max_iter=2000))
        rel = np.abs(out["cext_sensor"] / ref["cext_sensor"] - 1)
        accuracy = {"reference": "GPU dense direct FP64, GMRES tol 1e-10",
                    "max_rel_err": float(rel.max()), "median_rel_err": float(np.median(rel)),
                    "within_1e-4": int((rel <= 1e-4).sum()), "n_lambda": int(len(lam))}
        log(f"[bench] accuracy vs FP64: max {rel.max():.2e}, {accuracy['within_1e-4']}/{len(lam)}")
        sel = np.linspace(0, len(lam) - 1, 4).round().astype(int)
        g64 = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g64 = lspr.Geometry(dev, validate=False, **dict(op, precision="fp64"))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        it64 = []
        for k in sel:
            it64.append(int(g64.solve(lam[k:k + 1], em[k:k + 1], es[k:k + 1], ef,
                                      **gm)["iters"][0]))
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        g64.close()
        fp64_b1 = {"form": "treecode FP64 kernels, one wavelength per solve",
                   "wavelengths": int(len(sel)), "iters": it64,
                   "solves_per_s_incl_setup": len(sel) / (t_setup + t_solve),
                   "solves_per_s_steady": len(sel) / t_solve}
        log(f"[bench] FP64 one-at-a-time: {fp64_b1['solves_per_s_steady']:.2f} solves/s")

    # wavelengths within 1e-4 of the FP64 reference; without the reference nothing is credited
    value = accuracy["within_1e-4"] * args.steps / total if accuracy else None
    far = far_timed
    achieved = far["flops"] / (far["total_ms"] * 1e-3) / 1e12 if far["total_ms"] > 0 else 0.0
    mfma = op.get("matrix_cores", True) and info["n_tiles"] > 0
    # without tiles the far field is FP32 vector arithmetic: 256 CUs x 64 lanes x 2 flops (FMA)
    # x 2 (packed FP32) x 2.4 GHz
    peak = PEAK_FP32_MFMA_TFLOPS if mfma else PEAK_FP32_VALU_TFLOPS
    trec = traffic_entry(os.path.join(ROOT, "paper_1812_10722_amd", "csrc", "operator.hip"),
                         "far") if mfma else None
    roofline = {"kernel": "k_far_wide (above 32 wavelengths) and k_far_tiles_op (FP32 "
                          "matrix-core far field: expansion and direct far-rule tiles)" if mfma else
                          "k_far (FP32 vector-ALU far field, no tiles kept)",
                "bound": "mfma" if mfma else "alu",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak,
                "traffic": (trec["bytes_per_launch"] if trec else None),
                "launches": far["launches"],
                "avg_launch_ms": far["total_ms"] / max(far["launches"], 1),
                # executed: 4 flops per used real column and direct pair, 4 (P+1)^2 per column
                # and expansion pair (the tile contraction); the kernel values and Taylor
                # coefficients are precomputed once per geometry (precomputed_flops)
                "flops_per_launch": far["flops"] / max(far["launches"], 1),
                "precomputed_flops": precomputed_flops(info, op),
                "by_width": width_rows(lspr, "far", PEAK_FP32_MFMA_TFLOPS, width_timed),
                "fp64_by_width": width_rows(lspr, "far64", PEAK_FP64_MFMA_TFLOPS, width_timed)}
    times_s = np.array(times)
    line = {
        "metric": METRIC, "value": value, "unit": "wavelength-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "fp32", "fp64": "fp64"}.get(op["precision"], "fp32+fp64"),
        "data": "synthetic (seed-free octahedral sphere mesh, Drude silver in water)",
        "config": {"workload": w.name, "panels": w.n_panels, "wavelengths": int(len(lam)),
                   "method": op["method"], "p": op["p"], "theta": op["theta"],
                   "k_far": op["k_far"], "k_fine": op["k_fine"], "n_k": op["n_k"],
                   "threshold": op["threshold"], "kernels": op["precision"], "gmres": "fp64",
                   "gmres_tol": gm["tol"], "parallelism": "single GPU"},
        # (direct target-NODE pairs + expansion target-box pairs) x wavelengths per second of
        # the FP32 far-field launches; the panel form counts direct target-PANEL pairs (the
        # entries of the operator matrices the launch applies, K = 4 times fewer)
        "matvec_gpair_per_s": far["items"] / (far["total_ms"] * 1e-3) / 1e9
        if far["total_ms"] > 0 else None,
        "matvec_gpair_definition": "(target-node + target-box) pairs x wavelengths / s",
        "matvec_panel_gpair_per_s": (far["items"] / (far["total_ms"] * 1e-3) / 1e9
                                     * (info["p2p_pairs"] + info["m2p_pairs"])
                                     / (info["p2p_pairs"] * op["k_far"] + info["m2p_pairs"]))
        if far["total_ms"] > 0 else None,
        "matvec_launches_per_step": n_matvec,
        "step_latency_p50_s": float(np.percentile(times_s, 50)),
        "step_latency_p99_s": float(np.percentile(times_s, 99)),
        "latency_p50_s": None, "latency_p99_s": None, "serving": None,
        "roofline": roofline,
        "cpu_baseline": None,
        "accuracy": accuracy,
        "fp64_one_at_a_time": fp64_b1,
        "gmres_iters": {"min": int(out["iters"].min()), "max": int(out["iters"].max()),
                        "mean": float(out["iters"].mean()),
                        "converged": bool(out["converged"]),
                        "max_rel_resid": float(out["rel_resid"].max())},
        # one extra step after the timed ones, with events around every phase
        "kernel_ms_per_step": {n: p["total_ms"] for n, p in prof.items()},
        # algorithmic bytes / event time of the HBM-bound passes (Arnoldi: the basis vectors,
        # p and w read, q and the next vector written; near: table, densities and sums)
        "hbm_passes": {n: {"GB/s": prof[n]["bytes"] / (prof[n]["total_ms"] * 1e-3) / 1e9,
                           "frac": prof[n]["bytes"] / (prof[n]["total_ms"] * 1e-3) / 1e9
                           / PEAK_HBM_GBS}
                       for n in ("arnoldi", "near") if prof[n]["total_ms"] > 0},
        "lists": {k: int(info[k]) for k in ("n_boxes", "n_m2p", "n_p2p_ranges", "p2p_pairs",
                                            "m2p_pairs", "n_near", "n_terms", "ncrit")},
        "autotune": tuned,
    }
    n_srv = 16 if args.serving_requests is None else args.serving_requests
    if n_srv > 0:
        log(f"[bench] serving leg: {n_srv} requests ...")
        srv = serving_leg(lspr, n_srv, n_burst=args.serving_burst)
        line["serving"] = srv
        line["latency_p50_s"] = srv["latency_p50_s"]
        line["latency_p99_s"] = srv["latency_p99_s"]
        log(f"[bench] serving: burst {srv['burst_requests_per_s']:.2f} req/s, p50 "
            f"{srv['latency_p50_s']:.2f} s, p99 {srv['latency_p99_s']:.2f} s at "
            f"{srv['paced_rate_requests_per_s']:.2f} req/s")
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline on a bounded sample ...")
        line["cpu_baseline"] = cpu_baseline(
            w, iters_full=float(np.mean(fp64_b1["iters"])) if fp64_b1 else None)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
