"""Benchmark: galaxy-centres per second of the shear 4PCF multipole estimator
on one MI355X (the 600'x600' GRF catalogue, N = 1e6, 12 log bins over
1-100', nmax = 10), mixed-precision path timed; the FP64 GPU path, the
mixed-vs-FP64 error per correlator, the stage roofline and the FP64 CPU
oracle baseline are reported on the same JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp16|bf16|fp64]

Inputs are generated on the host, copied to HBM before the timed region;
each step is one full estimate_4pcf_multipoles call over every centre
(cell list, stage (a), stage (b), corrections, FP64 tail).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "galaxy-centers/sec for Υ (mixed vs FP64 GPU) + mock p50/p99 latency"
PEAK_FP32_VALU = 157.3e12     # published vector fp32 peak (packed FMA)
PEAK_FP64_VALU = 78.6e12      # published vector fp64 peak
PEAK_F16_MFMA = 2.5e15        # published dense fp16 / bf16 matrix peak
PEAK_FP64_MFMA = 78.6e12      # published fp64 matrix peak
STAGE_A_SRC = os.path.join(ROOT, "paper_2509_07974_amd", "csrc", "stage_a.hip")
STAGE_A_INPUT_SRCS = [os.path.join(ROOT, "paper_2509_07974_amd", "csrc", f)
                      for f in ("api.hip", "cells.hip", "sort.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_a_grf1m_traffic.txt")


def stage_a_flops_per_pair(nmax: int) -> float:
    """Algorithmic flops of stage (a) per in-bin (centre, neighbour) pair:
    2 (52 nmax + 72), i.e. one complex multiply-add chain per accumulated
    block order (G, Q: 4(4n+3) each; W: 2(2n+1); A: 2(2n+2); V: 2(2n+1);
    the triple blocks: 17) plus the power chain z^k (about 4(2n+6))."""
    return 2.0 * (52 * nmax + 72)


def stage_a_flops_executed_per_pair(nmax: int) -> float:
    """Flops the kernel actually issues per pair: one real-weight x power
    multiply-add (2 flops) per accumulated real unit (28 nmax + 56 units,
    orders k >= 0 only) plus one complex multiply (6 flops) per power of the
    chain."""
    units = 28 * nmax + 56
    powers = max(2 * nmax + 5, nmax + 6)
    return 2.0 * units + 6.0 * powers


def kernel_source_hash() -> str:
    import hashlib
    with open(STAGE_A_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def input_source_hash() -> str:
    """sha256 over the sources that decide what stage (a) reads: the planner
    (cell grid), the cell-list build and its sort."""
    import hashlib
    h = hashlib.sha256()
    for src in STAGE_A_INPUT_SRCS:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stage_a_traffic():
    """HBM bytes per stage (a) launch from the committed rocprofv3 counter
    summary, or None if it is missing or was taken on another kernel, planner
    or cell-list source."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != kernel_source_hash():
            return None
        if kv.get("input_source_sha256") != input_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(nbytes: int):
    """One plain device-to-device copy of nbytes (the reference kernel for
    scaling the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}))


def cpu_baseline(cat, edges, nmax, seconds_target=15.0):
    import oracle
    procs = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(2024)
    # calibrate on one centre, then size the sample for ~seconds_target of CPU work
    t = time.perf_counter()
    oracle.upsilon(*cat.arrays(), edges, nmax, centers=rng.choice(cat.n, 1, replace=False))
    per = time.perf_counter() - t
    nsample = int(max(procs, min(procs * 8, seconds_target * procs / max(per, 1e-3))))
    nsample = max(procs, (nsample // procs) * procs)
    idx = rng.choice(cat.n, nsample, replace=False)
    t = time.perf_counter()
    oracle.upsilon_parallel(*cat.arrays(), edges, nmax, centers=idx, processes=procs)
    wall = time.perf_counter() - t
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": nsample / wall, "unit": "centres/s", "cores": procs, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"{nsample} seeded centres of the same catalogue (all 1e6 galaxies as neighbours), "
                      f"FP64 NumPy oracle in {procs} processes, {wall:.1f} s wall"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Request stream for the latency report: the first SERVE_REQUESTS requests of
# the seeded serving stream at their full size (N log-uniform in [1e5, 2e6]
# galaxies, square patches of 4-100 deg^2, the grf-1m GRF recipe on a 4096^2
# grid with each request's own seed, 8-16 log bins over 1-100', nmax 8),
# arriving Poisson at a fixed rate.  The rate was calibrated once as 0.7 of
# the alone service rate of these requests (mean alone service time 1.268 s
# on one MI355X, `--serving-only --serve-alone`) and is frozen here so that
# latencies stay comparable between builds.
SERVE_REQUESTS = 32
SERVE_N_SCALE = 1.0
SERVE_NGRID = 4096
SERVE_SEED = 77
SERVE_LAMBDA = 0.55      # requests/s


def _make_catalogues(reqs):
    """The request catalogues, drawn in a process pool over the host's share
    of cores (each request's GRF needs a 4096^2 FFT)."""
    import multiprocessing as mp
    import synth
    procs = max(1, min(16, os.cpu_count() or 1, len(reqs)))
    if procs == 1:
        return [synth.make_request_catalogue(r) for r in reqs]
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(synth.make_request_catalogue, reqs)


def serving_report(precision: str, nreq: int = SERVE_REQUESTS, n_scale: float = SERVE_N_SCALE,
                   lam_fixed=SERVE_LAMBDA, alone: bool = False, ngrid: int = SERVE_NGRID):
    """Latency of the request stream served with continuous batching.  With
    `alone`, every request is first served by itself (the calibration of the
    arrival rate, and the check that each result in the mix equals its result
    alone, which the serving tests also assert)."""
    import paper_2509_07974_amd as fp  # noqa: F401
    from paper_2509_07974_amd.serve import Job, Server, latency_stats
    import synth
    t = time.perf_counter()
    reqs = synth.serving_requests(nreq, n_scale=n_scale, ngrid=ngrid)
    cats = _make_catalogues(reqs)
    log(f"serving: generated {len(reqs)} request catalogues in {time.perf_counter() - t:.1f} s")

    def jobs():
        return [Job(r["rid"], *c.arrays(), synth.log_edges(1.0, 100.0, r["nbins"]), r["nmax"],
                    precision=precision) for r, c in zip(reqs, cats)]

    service = []
    if alone:
        single = jobs()
        for k, j in enumerate(single):
            srv = Server()
            t = time.perf_counter()
            srv.submit(j)
            srv.drain()
            service.append(time.perf_counter() - t)
            if (k + 1) % 8 == 0:
                log(f"serving: alone pass {k + 1}/{len(single)} requests, {sum(service):.1f} s")
    lam = lam_fixed if lam_fixed else 0.7 / float(np.mean(service))
    rng = np.random.default_rng(SERVE_SEED)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
    arrivals -= arrivals[0]
    mix = jobs()
    for j, a in zip(mix, arrivals):
        j.arrival = float(a)
    srv = Server()
    t = time.perf_counter()
    # Server.run, with a progress line every 30 s
    todo = sorted(mix, key=lambda j: j.arrival)
    srv.t0 = srv.clock()
    k, last = 0, time.perf_counter()
    while k < len(todo) or not srv.idle():
        now = srv.now()
        while k < len(todo) and todo[k].arrival <= now:
            srv.submit(todo[k])
            k += 1
        if not srv.poll():
            time.sleep(2e-4)
        if time.perf_counter() - last > 30.0:
            last = time.perf_counter()
            log(f"serving: mix pass {len(srv.finished)}/{len(mix)} finished")
    wall = time.perf_counter() - t
    stats = latency_stats(mix)
    centres = sum(j.n for j in mix if j.state == "done")
    log(f"serving: mix pass {wall:.1f} s, p50 {stats['p50_s']:.3f} s, p99 {stats['p99_s']:.3f} s")
    rep = {"requests": len(mix), "precision": precision, "lambda_per_s": lam,
           "lambda_source": "fixed (0.7 / mean alone service time, calibrated once)" if lam_fixed
           else "0.7 / mean alone service time of this run",
           "p50_latency_s": stats["p50_s"], "p99_latency_s": stats["p99_s"],
           "mean_latency_s": stats["mean_s"], "max_latency_s": stats["max_s"],
           "wall_s": wall, "centres_per_s": centres / wall, "galaxies": int(sum(r["n"] for r in reqs)),
           "all_done": all(j.state == "done" for j in mix),
           "hbm_budget_bytes": srv.budget, "peak_admitted_bytes": srv.peak_used,
           "stream": f"seeded requests 0..{len(mix) - 1} (seeds 1000+r) at N x {n_scale:g}, GRF on a "
                     f"{ngrid}^2 grid, Poisson arrivals seed {SERVE_SEED}"}
    if alone:
        rep.update({"service_alone_p50_s": float(np.median(service)),
                    "service_alone_mean_s": float(np.mean(service)),
                    "mix_equals_alone": bool(all(m.state == "done" and a.state == "done"
                                                 and np.array_equal(m.result, a.result)
                                                 for m, a in zip(mix, single)))})
    return rep


def c4_report(precision: str):
    """One timed estimate of the largest workload: 2400'x2400', 1e7 galaxies
    on a lognormal density, 16 log bins 0.5-200', nmax 15, centre tiles
    chosen by the planner (catalogue already on the device)."""
    import torch
    import paper_2509_07974_amd as fp
    import synth
    t = time.perf_counter()
    cat, edges, nmax, desc = synth.workload("lognormal-10m")
    gen = time.perf_counter() - t
    log(f"lognormal-10m: generated in {gen:.1f} s")
    dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
    torch.cuda.synchronize()
    fp.profile_enable(True)
    t = time.perf_counter()
    out = fp.estimate_4pcf_multipoles(*dev, edges, nmax, precision=precision)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    prof = fp.profile_read()
    fp.profile_enable(False)
    del out, dev
    log(f"lognormal-10m: {dt:.2f} s per estimate")
    return {"workload": "lognormal-10m", "description": desc, "precision": precision, "value": cat.n / dt,
            "unit": "centres/s", "seconds": dt, "tiles": prof["steps"],
            "stage_ms": {k: prof[k + "_ms"] for k in ("stage_a", "relayout", "stage_b", "corr")},
            "generation_s": gen}


def stage_b_roofline(ncent, nb, nmax, precision, ms, issued, useful):
    """MFMA roofline of the contraction over the measured stage time: useful
    flops (8 per complex multiply-add of the distinct block products the
    library formed: each product of three blocks once, over all bin
    triples), the matrix-core flops it issued (padding, surplus tiles and
    the three hi/lo products of the 16-bit paths included), and the rate of
    one dense contraction per (mu, n2, n3) giving the same outputs in the
    same time (8 flop x 9 nb^3 (2nmax+1)^2 per centre)."""
    nn = 2 * nmax + 1
    dense = 8.0 * 9 * nb ** 3 * nn * nn * ncent
    peak = PEAK_FP64_MFMA if precision == "fp64" else PEAK_F16_MFMA
    t = ms * 1e-3
    return {"bound": "mfma", "useful_tflops": useful / t / 1e12, "issued_tflops": issued / t / 1e12,
            "dense_equivalent_tflops": dense / t / 1e12,
            "peak": peak / 1e12, "unit": "TFLOP/s", "frac_issued": issued / t / peak,
            "frac_useful": useful / t / peak, "stage_ms": ms}


TREE = (0.5, 3, 40.0)   # grids of 0.5', 1', 2' and r_min = 40 (the paper's setting)


def tree_report(fp, dev, n, edges, nmax, precision, exact_out, exact_dt):
    """The same estimate with the tree approximation: time per step and the
    deviation from the discrete result per correlator."""
    import torch

    def run():
        return fp.estimate_4pcf_multipoles(*dev, edges, nmax, precision=precision, tree=TREE)

    run()
    torch.cuda.synchronize()
    fp.profile_enable(True)
    t = time.perf_counter()
    for _ in range(2):
        res = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 2
    prof = fp.profile_read()
    fp.profile_enable(False)
    a, b = res.cpu().numpy(), exact_out.cpu().numpy()
    dev_mu = [float(np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m])) for m in range(9)]
    c = nmax
    lo = (Ellipsis, slice(c - 2, c + 3), slice(c - 2, c + 3))   # |n2|, |n3| <= 2
    dev_lo = [float(np.linalg.norm(a[m][lo] - b[m][lo]) / np.linalg.norm(b[m][lo])) for m in range(9)]
    log(f"tree: {dt:.3f} s/step")
    return {"delta1": TREE[0], "levels": TREE[1], "rmin": TREE[2], "value": n / dt, "unit": "centres/s",
            "ms_per_step": dt * 1e3, "speedup_vs_discrete": exact_dt / dt,
            "stage_a_ms_per_step": prof["stage_a_ms"] / 2,
            "deviation_from_discrete_per_mu": dev_mu,
            "deviation_from_discrete_per_mu_n_le_2": dev_lo}


NATURAL_NPHI = 129   # angular bins per axis of the natural components (the paper's choice)


def natural_report(fp, ups_dev, nphi, block=256):
    """Natural components of every radial-bin triplet of the result, streamed
    in blocks on the device (nothing of size nbins^3 nphi^2 is kept)."""
    import torch
    nb = ups_dev.shape[1]
    for _ in fp.natural_blocks(ups_dev, nphi, block=block):   # warm-up pass
        break
    torch.cuda.synchronize()
    t = time.perf_counter()
    n = 0
    for trip, gam, nrm in fp.natural_blocks(ups_dev, nphi, block=block):
        n += len(trip)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    log(f"natural components: {n} triplets x {nphi}^2 angles in {dt:.3f} s")
    return {"nphi": nphi, "triplets": n, "block": block, "seconds": dt,
            "values_per_s": 9 * n * nphi * nphi / dt,
            "streamed_bytes": 8 * n * nphi * nphi * 16 + n * nphi * nphi * 8}


THREEPCF_NMAX = 10   # 3PCF multipoles |n| <= 10 (stage (a) records of order 5)


BASETREE = (0.5, 3, 40.0)    # base grids 0.5', 1', 2'; a bin uses the coarsest with edge / grid >= 40


def grid_levels(edges, delta1, nlevels, rmin):
    """Grid of each radial bin: the coarsest d with edges[b] / (delta1 2^(d-1)) >= rmin, 0 if none."""
    out = []
    for e in edges[:-1]:
        ok = [d for d in range(1, nlevels + 1) if e / (delta1 * 2.0 ** (d - 1)) >= rmin]
        out.append(max(ok) if ok else 0)
    return out


def threepcf_report(fp, dev, n, edges, precision, no_fp64):
    """The shear 3PCF on the same catalogue: one warmup and two timed
    estimates (per-stage times from the library's events), and the FP64 path
    for the error per component."""
    import torch

    def run(prec):
        return fp.estimate_3pcf_multipoles(*dev, edges, THREEPCF_NMAX, precision=prec)

    run(precision)
    torch.cuda.synchronize()
    fp.profile_enable(True)
    t = time.perf_counter()
    for _ in range(2):
        out = run(precision)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 2
    prof = fp.profile_read()
    fp.profile_enable(False)
    rep = {"nmax": THREEPCF_NMAX, "record_order": (THREEPCF_NMAX + 1) // 2, "precision": precision,
           "value": n / dt, "unit": "centres/s", "ms_per_step": dt * 1e3,
           "stage_ms_per_step": {"stage_a": prof["stage_a_ms"] / 2, "relayout": prof["relayout_ms"] / 2,
                                 "contraction_and_same_neighbour": prof["stage_b_ms"] / 2}}
    log(f"3pcf: {dt:.3f} s/step")
    if precision != "fp64":
        # BaseTree (base points on grids of 0.5', 1', 2', r_min 40, the tree
        # setting of the paper's survey measurement) and DoubleTree (the
        # neighbours on the same grids as well)
        for key, kw in (("basetree", {"base": BASETREE}), ("doubletree", {"base": BASETREE, "tree": BASETREE})):
            def run_bt():
                return fp.estimate_3pcf_multipoles(*dev, edges, THREEPCF_NMAX, precision=precision, **kw)
            run_bt()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(2):
                bto = run_bt()
            torch.cuda.synchronize()
            dbt = (time.perf_counter() - t) / 2
            a, b = bto.cpu().numpy(), out.cpu().numpy()
            rep[key] = {
                "delta1": BASETREE[0], "levels": BASETREE[1], "rmin": BASETREE[2],
                "bin_grids": grid_levels(edges, *BASETREE),
                "ms_per_step": dbt * 1e3, "value": n / dbt, "unit": "centres/s",
                "speedup_vs_discrete": dt / dbt,
                "deviation_from_discrete_per_mu": [float(np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m]))
                                                   for m in range(5)]}
            log(f"3pcf {key}: {dbt:.3f} s/step ({dt / dbt:.2f}x)")
    if not no_fp64 and precision != "fp64":
        run("fp64")
        torch.cuda.synchronize()
        t = time.perf_counter()
        ref = run("fp64")
        torch.cuda.synchronize()
        rep["fp64_ms_per_step"] = (time.perf_counter() - t) * 1e3
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        rep["mixed_vs_fp64_rel_err_per_mu"] = [float(np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m]))
                                               for m in range(5)]
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16")
    ap.add_argument("--workload", default="grf-1m")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the mock request-stream latency report")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 mixed-path run")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the request-stream report (with --serve-requests / --serve-n-scale)")
    ap.add_argument("--serve-requests", type=int, default=SERVE_REQUESTS)
    ap.add_argument("--serve-n-scale", type=float, default=SERVE_N_SCALE)
    ap.add_argument("--serve-lambda", type=float, default=SERVE_LAMBDA or 0.0,
                    help="arrival rate (requests/s); 0 = 0.7 / mean alone service time")
    ap.add_argument("--serve-alone", action="store_true",
                    help="serve every request alone first (calibrates the rate, checks mix == alone)")
    ap.add_argument("--no-c4", action="store_true", help="skip the timed lognormal-10m estimate")
    ap.add_argument("--no-3pcf", action="store_true", help="skip the 3PCF run on the same catalogue")
    ap.add_argument("--no-tree", action="store_true", help="skip the tree-approximation run")
    ap.add_argument("--no-natural", action="store_true",
                    help="skip the blockwise natural-component conversion of the result")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; the multi-GPU path "
                          "(centre sharding + one all-reduce of Upsilon) is not built"}))
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.serving_only:
        rep = serving_report(args.precision, args.serve_requests, args.serve_n_scale, args.serve_lambda or None,
                             alone=args.serve_alone)
        print(json.dumps({"serving": rep}))
        return

    import torch
    import paper_2509_07974_amd as fp
    import synth

    t0 = time.perf_counter()
    cat, edges, nmax, desc = synth.workload(args.workload)
    gen_s = time.perf_counter() - t0
    dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
    torch.cuda.synchronize()

    def run(prec):
        return fp.estimate_4pcf_multipoles(*dev, edges, nmax, precision=prec)

    log(f"generated {args.workload} in {gen_s:.1f} s")
    for i in range(args.warmup):
        t = time.perf_counter()
        run(args.precision)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t:.3f} s")
    fp.profile_enable(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        out = run(args.precision)
        if i == 0 or i + 1 == args.steps:
            log(f"step {i} issued")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    prof = fp.profile_read()
    fp.profile_enable(False)
    value = cat.n / dt

    steps = args.steps
    launches = max(prof["stage_a_launches"], 1)
    pairs_per_launch = prof["pairs"] / launches
    a_ms = prof["stage_a_ms"] / launches
    peak = PEAK_FP64_VALU if args.precision == "fp64" else PEAK_FP32_VALU
    achieved = pairs_per_launch * stage_a_flops_per_pair(nmax) / (a_ms * 1e-3)
    executed = pairs_per_launch * stage_a_flops_executed_per_pair(nmax) / (a_ms * 1e-3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak,
            # the committed counters cover the binary32 kernel on grf-1m only
            "traffic": stage_a_traffic() if args.workload == "grf-1m" and args.precision != "fp64" else None,
            "kernel": "stage_a_kernel (pair multipoles)",
            "avg_launch_ms": a_ms, "launches_per_step": launches / steps,
            "pairs_per_launch": pairs_per_launch,
            "flops_per_pair": stage_a_flops_per_pair(nmax),
            "executed_flops_per_pair": stage_a_flops_executed_per_pair(nmax),
            "achieved_executed": executed / 1e12}

    extra = {"stage_ms_per_step": {k: prof[k + "_ms"] / steps for k in ("stage_a", "relayout", "stage_b", "corr")},
             "generation_s": gen_s,
             "roofline_stage_b": stage_b_roofline(cat.n, len(edges) - 1, nmax, args.precision,
                                                  prof["stage_b_ms"] / steps,
                                                  prof["stage_b_mfma_flops"] / steps,
                                                  prof["stage_b_useful_flops"] / steps)}
    log(f"timed {args.steps} steps: {dt:.3f} s/step")
    if not args.no_fp64 and args.precision != "fp64":
        ref = run("fp64")
        torch.cuda.synchronize()
        log("fp64 warmup done")
        # the FP64 path is timed over up to three estimates (about 2.6 s each at grf-1m)
        k64 = max(1, min(args.steps, 3))
        fp.profile_enable(True)
        t = time.perf_counter()
        for _ in range(k64):
            ref = run("fp64")
        torch.cuda.synchronize()
        dt64 = (time.perf_counter() - t) / k64
        p64 = fp.profile_read()
        fp.profile_enable(False)
        a = out.cpu().numpy()
        b = ref.cpu().numpy()
        err = [float(np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m])) for m in range(9)]
        extra.update({"fp64_value": cat.n / dt64, "fp64_ms_per_step": dt64 * 1e3,
                      "fp64_steps": k64,
                      "fp64_stage_ms_per_step": {k: p64[k + "_ms"] / k64 for k in ("stage_a", "relayout", "stage_b", "corr")},
                      "mixed_vs_fp64_rel_err_per_mu": err,
                      # largest element error per mu, relative to that mu's largest |value|
                      "mixed_vs_fp64_max_abs_err_per_mu": [float(np.abs(a[m] - b[m]).max() / np.abs(b[m]).max())
                                                           for m in range(9)],
                      "mixed_speedup_vs_fp64": dt64 / dt})
        if not args.no_bf16 and args.precision != "bf16":
            run("bf16")
            torch.cuda.synchronize()
            t = time.perf_counter()
            o16 = run("bf16")
            torch.cuda.synchronize()
            dtb = time.perf_counter() - t
            c = o16.cpu().numpy()
            extra.update({"bf16_value": cat.n / dtb, "bf16_ms_per_step": dtb * 1e3,
                          "bf16_vs_fp64_rel_err_per_mu":
                              [float(np.linalg.norm(c[m] - b[m]) / np.linalg.norm(b[m])) for m in range(9)]})
            log(f"bf16: {dtb:.3f} s/step")
        del ref
    if not args.no_tree and args.precision != "fp64":
        extra["tree"] = tree_report(fp, dev, cat.n, edges, nmax, args.precision, out, dt)
    if not args.no_natural:
        extra["natural_blocks"] = natural_report(fp, out, NATURAL_NPHI)
    if not args.no_3pcf:
        extra["threepcf"] = threepcf_report(fp, dev, cat.n, edges, args.precision, args.no_fp64)
    line = {"metric": METRIC, "value": value, "unit": "centres/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp16": "f32+f16x2+f64", "bf16": "f32+bf16x2+f64", "fp64": "f64"}[args.precision],
            "data": "synthetic",
            "config": {"workload": args.workload, "description": desc, "n_galaxies": cat.n,
                       "nbins": len(edges) - 1, "nmax": nmax, "precision": args.precision},
            "roofline": roof}
    if not args.no_serving:
        sv = serving_report(args.precision, args.serve_requests, args.serve_n_scale,
                            args.serve_lambda or None, alone=args.serve_alone)
        extra["serving"] = sv
        line["latency"] = {"p50_s": sv["p50_latency_s"], "p99_s": sv["p99_latency_s"],
                           "workload": f"first {sv['requests']} requests of the seeded serving stream at "
                                       f"full N ({sv['galaxies']} galaxies in all, 1e5-2e6 each, GRF on a "
                                       f"{SERVE_NGRID}^2 grid, 8-16 bins, nmax 8), Poisson arrivals at "
                                       f"{sv['lambda_per_s']:g}/s"}
    if not args.no_c4:
        extra["lognormal_10m"] = c4_report(args.precision)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(cat, edges, nmax)
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()
