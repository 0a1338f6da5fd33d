#!/usr/bin/env python
"""Benchmark of the periodic Stokes mobility solve on one MI355X.

Workload: 200 random ellipses at area fraction 0.4, 256 nodes each (N = 51,200),
seed 2 (the large-cell configuration on which node-pair evaluations per second are
quoted). One step = one complete mobility solve from a zero initial guess to an FP64
relative residual of 1e-10 (matvecs + GMRES + readout of v, omega, mu_eff), then
mu_eff once more by contour deformation (valid with particles across the wall D), with
the geometry already resident in HBM. Default solver: FP32 near sums inside FP64
iterative refinement with the right block preconditioner (the fastest variant at this
residual); --precision and --precond choose others, and the untimed comparison solves
report plain FP64 GMRES, the other mixed forms and the FMM near sum beside it.

value = node-image pair evaluations (9 N^2 per matvec, all matvecs of the step) per
second of wall time over the timed steps.

roofline: the near-sum kernel (the dominant kernel), timed live with HIP events
recorded on the library's stream around every launch inside the timed region;
algorithmic work 19 flop per pair (r: 2, |r|^2: 3, r.n: 3, r.f: 3, 1/|r|^2: 1,
square: 1, coefficient: 2, accumulate: 4).

cpu_baseline: the FP64 CPU oracle's near-image traction sum (plain C, OpenMP) on a
bounded sample of targets of the same workload, in pair evaluations per second.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 19
PEAK = {"fp32": 157.3, "fp64": 78.6}   # MI355X vector ALU peaks, TFLOP/s
COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "near_sum_fp32_ellipses200_N51200_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_04501_amd", "csrc", f) for f in ("k_near.hip", "spm_internal.h")]


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the FP32 near sum from the committed counter summary, or
    None when that summary is missing or was taken on different kernel sources."""
    import re
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cells, target_seconds=10.0):
    """The oracle's near-image traction sum timed on the host: a prefix of the targets
    when one sweep of every cell would take longer than target_seconds, otherwise whole
    sweeps over every cell, repeated until about target_seconds have passed."""
    import numpy as np

    from oracle import _clib, geometry
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    prep = []
    for wl in cells:
        g = geometry.build_geometry(wl)
        sig = np.random.default_rng(7).standard_normal((g.N, 2))
        prep.append((g, g.w[:, None] * sig, g.shifts(1)))

    def run(g, f, sh, nt):
        t0 = time.perf_counter()
        _clib.near_traction(g.x[:nt], g.n[:nt], g.x, f, sh, np.arange(nt))
        return time.perf_counter() - t0

    g, f, sh = max(prep, key=lambda p: p[0].N)
    n0 = min(g.N, 1024)
    run(g, f, sh, min(g.N, 64))
    rate = n0 * g.N * 9 / run(g, f, sh, n0)
    sweep_pairs = sum(p[0].N * p[0].N * 9 for p in prep)
    Ntot = sum(p[0].N for p in prep)
    if sweep_pairs / rate > target_seconds:   # a prefix of the largest cell's targets
        nt = int(min(g.N, max(n0, rate * target_seconds / (g.N * 9))))
        t = run(g, f, sh, nt)
        pairs = nt * g.N * 9
        what = f"{nt} of the {g.N} targets against all {g.N} sources x 9 images"
    else:                                     # whole sweeps until target_seconds have passed
        reps, t = 0, 0.0
        while t < target_seconds:
            for p in prep:
                t += run(*p, p[0].N)
            reps += 1
        pairs = reps * sweep_pairs
        what = (f"{reps} full sweep(s) of all {Ntot} targets against their own cell's sources x 9 images"
                + (f" over {len(prep)} cells" if len(prep) > 1 else ""))
    return {"value": pairs / t, "unit": "pair-evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"FP64 oracle near-image traction sum (plain C, OpenMP): {what} ({pairs:.3e} pairs, {t:.1f} s)"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_solve_times(with_c2=False):
    """The oracle's complete FP64 mobility solves (set-up + MGS GMRES to 1e-10 from zero) of
    the single ellipse (N = 128) and the 25-ellipse cell (N = 5,112), and the dense LU solve of
    the single ellipse (the matrix assembled column by column from operator products); with
    with_c2 also the 200-ellipse cell (N = 51,200; minutes on the host's cores)."""
    from oracle import operator as op
    from paper_1912_04501_amd import workloads as W
    out = {}
    cases = [("single_ellipse_N128", W.single_ellipse()), ("ellipses25_N5112", W.ellipses_25())]
    if with_c2:
        cases.append(("ellipses200_N51200", W.ellipses_200()))
    for name, wl in cases:
        t0 = time.perf_counter()
        prob = op.make_problem(wl)
        count = [0]

        def product(v, prob=prob, count=count, name=name):
            count[0] += 1
            if count[0] % 10 == 0:
                log(f"[bench] oracle solve {name}: {count[0]} operator products, {time.perf_counter() - t0:.0f}s")
            return op.apply(prob, v)
        x, info = op.gmres(product, op.rhs(prob), tol=1e-10)
        out[f"gmres_s_{name}"] = time.perf_counter() - t0
        out[f"gmres_its_{name}"] = info["iterations"]
        if name == "single_ellipse_N128":
            t0 = time.perf_counter()
            op.solve(prob, method="lu")
            out[f"dense_lu_s_{name}"] = time.perf_counter() - t0
    return out


def gpu_small_solve_times():
    """The same two solves on the GPU (FP64 GMRES to 1e-10, geometry resident, second solve timed)."""
    import torch

    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W
    out = {}
    for name, wl in (("single_ellipse_N128", W.single_ellipse()), ("ellipses25_N5112", W.ellipses_25())):
        s = spm.Solver("cuda:0")
        s.set_workload(wl)
        s.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        out[f"gpu_fp64_s_{name}"] = time.perf_counter() - t0
        out[f"gpu_fp64_its_{name}"] = r["info"]["iterations"]
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32_ir", "fp32_relaxed", "fp64"], default=None,
                    help="solver precision (default: fp32_ir for the 200-ellipse cell, fp32_relaxed for the "
                         "ensemble)")
    ap.add_argument("--precond", choices=["none", "block"], default=None,
                    help="ellipses200 and ensemble64: right block preconditioner (default: block)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the untimed FP64-vs-FP32+IR comparison solves")
    ap.add_argument("--oracle-c2", action="store_true",
                    help="cpu_baseline also times the oracle's whole solve of the 200-ellipse cell (minutes)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (reuse launch shapes across runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy three times (HBM counter calibration)")
    ap.add_argument("--workload", choices=["ellipses200", "ensemble64", "learned", "stepping", "jamming", "islands"],
                    default="ellipses200",
                    help="ellipses200: the 200-ellipse cell (default); ensemble64: 64 independent cells in one "
                         "launch; learned: time stepping with the trained warm-start network; stepping: the same held-out "
                         "trajectory steps without the network; jamming: two "
                         "star-shaped particles sheared into contact (Sec. 8 Examples 4 and 5); islands: K random "
                         "star-shaped islands of 350 nodes (Sec. 8 Example 2 scale) with the FMM near sum")
    ap.add_argument("--islands", default="100,250,500,1000", help="islands: the island counts K")
    ap.add_argument("--direct-max", type=int, default=250,
                    help="islands: largest K also solved with the direct FP32 near sum")
    ap.add_argument("--example", type=int, choices=[4, 5], default=4, help="jamming: which of the two runs")
    ap.add_argument("--nodes", type=int, default=2500, help="jamming: nodes per star")
    ap.add_argument("--omega", type=int, default=4, help="jamming: arms of each star, r = s (1 + cos(omega t)/2)")
    ap.add_argument("--full-series", action="store_true", help="jamming: every step of mu_eff(t) in the JSON line")
    ap.add_argument("--no-tune", action="store_true", help="jamming: keep the heuristic near-sum launch shapes")
    ap.add_argument("--jam-tol", type=float, default=None,
                    help="jamming: GMRES tolerance (default 1e-9 for Example 4, 1e-8 for Example 5: near contact "
                         "the FP64 residual floor of the operator reaches 2e-10 at mu_eff ~ 1e5 and 1e-9 at gaps "
                         "~ 1e-4)")
    ap.add_argument("--dt", type=float, default=5e-4, help="jamming: forward Euler step")
    ap.add_argument("--t-end", type=float, default=None, help="jamming: last time (default 0.46 / 0.475)")
    ap.add_argument("--window", type=float, nargs=2, default=None,
                    help="jamming: fit window (default: the example's, and the same width before the run's end)")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = "fp32_ir"
    if args.precond is None:
        args.precond = "block" if args.workload in ("ensemble64", "ellipses200") else "none"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver runs on a single GPU",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x {COPY_BYTES} bytes read and written")
    if args.workload == "ensemble64":
        return bench_ensemble(args)
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "jamming":
        return bench_jamming(args)
    if args.workload == "stepping":
        return bench_stepping(args)
    if args.workload == "islands":
        return bench_islands(args)
    t0 = time.perf_counter()
    wl = W.ellipses_200()
    log(f"[bench] workload {wl['name']} generated in {time.perf_counter() - t0:.1f}s")
    prec = {"fp32_relaxed": spm.SPM_FP32_RELAXED, "fp32_ir": spm.SPM_FP32_IR, "fp64": spm.SPM_FP64}[args.precision]
    s = spm.Solver("cuda:0", precision=prec,
                   precond=spm.SPM_PRECOND_BLOCK if args.precond == "block" else spm.SPM_PRECOND_NONE)
    s.set_workload(wl)
    N = s.N
    pairs_per_matvec = 9.0 * N * N
    log(f"[bench] N={N} particles={s.No} close pairs={len(s.close_pairs())}")
    t0 = time.perf_counter()
    tune = s.autotune(args.tune_cache)
    log(f"[bench] autotune {time.perf_counter() - t0:.1f}s: {tune}")

    for k in range(args.warmup):
        r = s.solve()
        s.effective_viscosity_contour(r["sigma"])
        log(f"[bench] warmup {k}: {r['info']}")
    torch.cuda.synchronize()
    # timed region: the production path (each GMRES iteration replayed as a captured HIP graph,
    # no timing events)
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        r = s.solve()
        mu_c = s.effective_viscosity_contour(r["sigma"])
        infos.append(r["info"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for k, i in enumerate(infos):
        log(f"[bench] step {k}: {i}")
    matvecs = sum(i["fp64_matvecs"] + i["fp32_matvecs"] for i in infos)
    value = matvecs * pairs_per_matvec / elapsed
    # the same steps again with HIP events recorded on the library's stream around every
    # near-sum launch (events are not captured into graphs, so these iterations run unreplayed)
    s.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        rp = s.solve()
        s.effective_viscosity_contour(rp["sigma"])
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    profs = [s.profile_read(0), s.profile_read(1)]
    s.profile(False)

    def roof(kern):
        prof = profs[kern]
        avg_ms = prof["ms"] / max(prof["launches"], 1)
        achieved = FLOP_PER_PAIR * pairs_per_matvec / (avg_ms * 1e-3) / 1e12
        dt = "fp32" if kern == 1 else "fp64"
        return {"bound": "alu", "achieved": achieved, "peak": PEAK[dt], "unit": "TFLOP/s",
                "frac": achieved / PEAK[dt], "traffic": measured_traffic() if kern == 1 else None,
                "kernel": f"k_near<{'float' if kern else 'double'}> (near-image traction sum, {dt})",
                "avg_launch_ms": avg_ms, "launches": prof["launches"], "total_ms": prof["ms"],
                "pairs_per_launch": pairs_per_matvec, "launch_shape": tune["fp32" if kern else "fp64"]}

    # the dominant kernel is the near sum of the precision that took the most time
    kern = 0 if profs[0]["ms"] >= profs[1]["ms"] else 1
    roofline = roof(kern)
    other = roof(1 - kern) if profs[1 - kern]["launches"] > 0 else None

    extra = {}
    if not args.no_compare:
        # the paper's own near set (four images of every wrapped node, 4 N^2 pairs per matvec)
        # with 64 proxies on the dilated cell's walls, at two pseudo-inverse cutoffs
        dil = dict(near_set=spm.SPM_NEAR_SET_DILATED, M=64, m_wall=24)
        for name, cfg in (("fp64", dict(precision=spm.SPM_FP64)), ("fp32_ir", dict(precision=spm.SPM_FP32_IR)),
                          ("fp32_relaxed", dict(precision=spm.SPM_FP32_RELAXED)),
                          ("fp64_precond", dict(precision=spm.SPM_FP64, precond=1)),
                          ("fp32_ir_precond", dict(precision=spm.SPM_FP32_IR, precond=1)),
                          ("fp32_relaxed_precond", dict(precision=spm.SPM_FP32_RELAXED, precond=1)),
                          ("fmm_fp64_precond", dict(precision=spm.SPM_FP64, precond=1, near_method=spm.SPM_NEAR_FMM)),
                          ("dilated_fp64_precond", dict(precision=spm.SPM_FP64, precond=1, rcond=1e-8, **dil)),
                          ("dilated_fp32_ir_precond", dict(precision=spm.SPM_FP32_IR, precond=1, rcond=1e-8, **dil)),
                          ("dilated_fp32_ir_precond_rcond1e-10",
                           dict(precision=spm.SPM_FP32_IR, precond=1, rcond=1e-10, **dil))):
            c = spm.Solver("cuda:0", **cfg)
            c.set_workload(wl)
            if name.startswith("dilated"):   # a kernel of its own: its own launch shapes
                extra[f"launch_{name}"] = c.autotune(args.tune_cache)
            else:
                for pr, key in ((spm.SPM_FP64, "fp64"), (spm.SPM_FP32, "fp32")):
                    c.set_launch(pr, **tune[key])
            c.solve()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rr = c.solve()
            torch.cuda.synchronize()
            extra[f"solve_s_{name}"] = time.perf_counter() - t1
            extra[f"solve_info_{name}"] = {k: rr["info"][k] for k in ("iterations", "fp64_matvecs", "fp32_matvecs",
                                                                       "refinements", "rel_residual")}
            extra[f"mu_eff_{name}"] = float(rr["mu_eff"].item())
            if name.startswith("dilated"):
                extra[f"pairs_per_matvec_{name}"] = 4.0 * N * N
            c.close()
        log(f"[bench] comparison {extra}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample ...")
        cpu = cpu_baseline([wl])
        cpu["solves"] = {**oracle_solve_times(args.oracle_c2), **gpu_small_solve_times()}
        log(f"[bench] cpu baseline {cpu}")

    out = {"metric": "Stokes matvec pair-evals/s (whole mobility solve to 1e-10 FP64 residual)",
           "value": value, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prec == spm.SPM_FP64 else "f32+f64", "data": "synthetic",
           "config": {"workload": wl["name"], "N": N, "particles": s.No, "nodes_per_particle": 256,
                      "precision": args.precision, "precond": args.precond, "tol": 1e-10, "images": "3x3",
                      "proxies": 32,
                      "wall_points": 24, "close_factor": 10},
           "ms_per_step_profiled": 1e3 * elapsed_prof / args.steps,
           "roofline": roofline, "roofline_other_precision": other, "cpu_baseline": cpu,
           "mu_eff": {"stresslet": float(r["mu_eff"][0]), "contour": float(mu_c[0])}, **extra}
    print(json.dumps(out), flush=True)


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def bench_ensemble(args):
    """64 independent cells (seeds 1000..1063, 4-50 ellipses each) solved together in
    one persistent near-sum launch per matvec (FP32 + FP64 iterative refinement with the
    block preconditioner by default, --precision and --precond choose the solver), autotuned
    launch shape, every GMRES iteration replayed as a captured HIP graph. One step = one
    batched solve of every cell to 1e-10; value = cell solves per second; per-cell latency
    (device wall clock from the solve start to the cell's convergence) as p50 / p99 over the
    timed steps. Untimed comparisons: the other FP32 form, and the same solver without
    graph replay."""
    import numpy as np
    import torch

    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W
    t0 = time.perf_counter()
    cells = W.ensemble_cells(64)
    Ns = np.array([int(np.sum(c["n_nodes"])) for c in cells])
    log(f"[bench] 64 cells generated in {time.perf_counter() - t0:.1f}s: N_c {Ns.min()}..{Ns.max()}, "
        f"total {Ns.sum()}, particles {sum(len(c['theta']) for c in cells)}")
    precs = {"fp32_ir": spm.SPM_FP32_IR, "fp32_relaxed": spm.SPM_FP32_RELAXED, "fp64": spm.SPM_FP64}
    pc = spm.SPM_PRECOND_BLOCK if args.precond == "block" else spm.SPM_PRECOND_NONE
    s = spm.Solver("cuda:0", precision=precs[args.precision], precond=pc)
    s.set_cells(cells)
    tune = s.autotune(args.tune_cache)
    log(f"[bench] autotune: {tune}")
    for k in range(args.warmup):
        r = s.solve_cells()
        log(f"[bench] warmup {k}: its {[i['iterations'] for i in r['infos']][:8]} ...")
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()   # timed region: every iteration replayed as a captured HIP graph
    for k in range(args.steps):
        r = s.solve_cells()
        lat.extend(r["latency_s"].tolist())
        infos.extend(r["infos"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    compare = {}
    if not args.no_compare:
        # the same batch with the other FP32 form, and without graph replay (untimed region)
        others = [(n, p, 1) for n, p in precs.items() if n != args.precision and n != "fp64"]
        others.append((args.precision + "_no_graph", precs[args.precision], 0))
        for name, p, graph in others:
            c = spm.Solver("cuda:0", precision=p, precond=pc, use_graph=graph)
            c.set_cells(cells)
            for pr, key in ((spm.SPM_FP64, "fp64"), (spm.SPM_FP32, "fp32")):
                c.set_launch(pr, **tune[key])
            c.solve_cells()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rr = c.solve_cells()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            compare[name] = {"solves_per_s": 64 / dt, "latency_p50_ms": 1e3 * percentile(rr["latency_s"], 50),
                             "latency_p99_ms": 1e3 * percentile(rr["latency_s"], 99),
                             "max_rel_residual": max(i["rel_residual"] for i in rr["infos"])}
            c.close()
        log(f"[bench] ensemble comparison {compare}")
    assert max(i["rel_residual"] for i in infos) <= 1e-10
    pairs = float(9.0 * (Ns.astype(np.float64) ** 2).sum())
    # roofline of the near-sum launch over all 64 cells (inside a solve, launches skip the
    # cells that have converged): FP32 operator applications, HIP events on the stream
    x = torch.randn(2 * s.N, dtype=torch.float64, device="cuda:0")
    s.apply(x, precision=spm.SPM_FP32)
    torch.cuda.synchronize()
    s.profile(True)
    for _ in range(10):
        s.apply(x, precision=spm.SPM_FP32)
    torch.cuda.synchronize()
    prof = s.profile_read(1)
    s.profile(False)
    avg_ms = prof["ms"] / max(prof["launches"], 1)
    pairs_per_launch = prof["pairs"] / max(prof["launches"], 1)
    achieved = FLOP_PER_PAIR * pairs_per_launch / (avg_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cells)
        # in the metric's unit: the matvecs each cell took on the GPU, at the oracle's pair
        # rate, near sums only (so an upper bound on what the oracle's whole solve reaches)
        mv = np.array([i["fp64_matvecs"] + i["fp32_matvecs"] for i in infos[:len(cells)]], dtype=np.float64)
        cpu["solves_per_s_near_only"] = len(cells) / float((9.0 * Ns.astype(np.float64) ** 2 * mv).sum()
                                                           / cpu["value"])
    out = {"metric": f"ensemble cell solves/s (64 independent cells, {args.precision}"
                     f"{' + block preconditioner' if args.precond == 'block' else ''} to 1e-10 FP64 residual)",
           "value": 64 * args.steps / elapsed, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "ensemble_64_cells_phi0.3", "cells": 64, "nodes_total": int(Ns.sum()),
                      "nodes_min": int(Ns.min()), "nodes_max": int(Ns.max()), "pairs_per_matvec": pairs,
                      "precision": args.precision, "precond": args.precond, "tol": 1e-10},
           "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99),
                          "max": 1e3 * max(lat)},
           "iterations": {"p50": percentile([i["iterations"] for i in infos], 50),
                          "max": max(i["iterations"] for i in infos)},
           "compare": compare,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                        "frac": achieved / PEAK["fp32"], "traffic": None,
                        "kernel": "k_near<float> (near-image traction sum over all active cells, fp32)",
                        "avg_launch_ms": avg_ms, "launches": prof["launches"], "pairs_per_launch": pairs_per_launch,
                        "launch_shape": tune["fp32"]},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def bench_islands(args):
    """Random star-shaped islands at the scale of Sec. 8 Example 2 (K islands of 350 nodes,
    N = 350 K, area fraction 0.2, seed 1): complete FP64 mobility solves to 1e-10 with the FMM
    near sum (40 terms) and the block preconditioner. One step = one solve of the largest K;
    value = solves per second. Every K also reports the FMM near-sum kernels (HIP events) and
    one launch of the direct FP32 and FP64 near sums, a 100 x 100 field grid and five forward-Euler
    steps (dt 1e-3; each re-sets the geometry and solves to 1e-10 from a zero guess); K <=
    --direct-max also the best direct solve (FP32 + iterative refinement with the block
    preconditioner)."""
    import numpy as np
    import torch

    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W
    Ks = [int(k) for k in args.islands.split(",")]
    series = []
    last = None
    for K in Ks:
        wl = W.random_stars(K, 0.2, 1)
        N = int(np.sum(wl["n_nodes"]))
        s = spm.Solver("cuda:0", precision=spm.SPM_FP64, precond=spm.SPM_PRECOND_BLOCK, near_method=spm.SPM_NEAR_FMM)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_workload(wl)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        st = s.fmm_stats()
        log(f"[islands] K {K} N {N}: geometry set-up {setup_s:.3f}s, FMM {st}")
        for _ in range(args.warmup):
            r = s.solve()
        torch.cuda.synchronize()
        s.profile(True)
        t1 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            r = s.solve()
            infos.append(r["info"])
        torch.cuda.synchronize()
        solve_s = (time.perf_counter() - t1) / args.steps
        ev = {k: s.profile_read(k) for k in (2, 3)}
        s.profile(False)
        assert max(i["rel_residual"] for i in infos) <= 1e-10, infos
        # one FMM near sum in isolation (all of its kernels, CUDA events on torch's stream)
        x = torch.randn(2 * N, dtype=torch.float64, device="cuda:0")
        s.near_traction(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            s.near_traction(x)
        e1.record()
        torch.cuda.synchronize()
        fmm_ms = e0.elapsed_time(e1) / 5
        mu_c = float(s.effective_viscosity_contour(r["sigma"])[0])
        # flow field on a 100 x 100 grid over the cell (velocity and pressure)
        g1 = np.linspace(-0.5, 0.5, 100, endpoint=False) + 0.005
        grid = np.stack(np.meshgrid(g1, g1), axis=-1).reshape(-1, 2)
        s.eval_field(r["sigma"], grid)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.eval_field(r["sigma"], grid)
        torch.cuda.synchronize()
        field_s = time.perf_counter() - t1
        # forward Euler (Sec. 7) with the FMM: every step re-sets the geometry (nodes, proxy
        # pseudo-inverse, close pairs, quadtree) and solves to 1e-10
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        so = s.step(1e-3, 5, 0.0, wl["centers"], wl["theta"])
        torch.cuda.synchronize()
        step_ms = 1e3 * (time.perf_counter() - t1) / 5
        assert max(i["rel_residual"] for i in so["infos"]) <= 1e-10
        entry = {"K": K, "N": N, "setup_s": setup_s, "step_ms": step_ms, "fmm_levels": st["levels"], "fmm_order": st["order"],
                 "fmm_direct_pairs": st["p2p_pairs"], "fmm_m2l": st["m2l"], "solve_s": solve_s,
                 "iterations": infos[-1]["iterations"], "rel_residual": infos[-1]["rel_residual"],
                 "mu_eff": float(r["mu_eff"][0]), "mu_eff_contour": mu_c,
                 "fmm_near_sum_ms": fmm_ms,
                 "fmm_eval_kernel_ms": ev[2]["ms"] / max(ev[2]["launches"], 1),
                 "fmm_m2l_kernel_ms": ev[3]["ms"] / max(ev[3]["launches"], 1),
                 "field_grid_100x100_s": field_s}
        s.close()
        d = spm.Solver("cuda:0", precision=spm.SPM_FP32_IR, precond=spm.SPM_PRECOND_BLOCK)
        d.set_workload(wl)
        d.profile(True)
        for pr in (spm.SPM_FP32, spm.SPM_FP64):
            d.near_traction(x, precision=pr)
        torch.cuda.synchronize()
        entry["direct_fp32_near_sum_ms"] = d.profile_read(1)["ms"]
        entry["direct_fp64_near_sum_ms"] = d.profile_read(0)["ms"]
        d.profile(False)
        if K <= args.direct_max:
            d.solve()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rd = d.solve()
            torch.cuda.synchronize()
            entry["direct_fp32_ir_precond_solve_s"] = time.perf_counter() - t1
            entry["direct_iterations"] = rd["info"]["iterations"]
            entry["direct_mu_eff"] = float(rd["mu_eff"][0])
            d.eval_field(rd["sigma"], grid)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            d.eval_field(rd["sigma"], grid)
            torch.cuda.synchronize()
            entry["direct_field_grid_100x100_s"] = time.perf_counter() - t1
        d.close()
        log(f"[islands] {entry}")
        series.append(entry)
        last = (wl, entry, ev, st, infos)
    wl, entry, ev, st, infos = last
    # dominant FMM kernel over the timed solves
    flops = {2: FLOP_PER_PAIR * st["p2p_pairs"] + 32.0 * st["order"] * entry["N"],
             3: 12.0 * st["order"] ** 2 * st["m2l"]}
    kern = 2 if ev[2]["ms"] >= ev[3]["ms"] else 3
    avg_ms = ev[kern]["ms"] / max(ev[kern]["launches"], 1)
    achieved = flops[kern] / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp64"], "traffic": None,
                "kernel": "k_fmm_eval (local expansions + direct pairs of neighbouring leaves, fp64)" if kern == 2
                else "k_fmm_m2l (multipole-to-local translations, fp64)",
                "avg_launch_ms": avg_ms, "launches": ev[kern]["launches"],
                "flop_per_launch": flops[kern]}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline([wl])
        mv = infos[-1]["fp64_matvecs"] + infos[-1]["fp32_matvecs"]
        cpu["solves_per_s_near_only"] = cpu["value"] / (9.0 * entry["N"] ** 2 * mv)
    out = {"metric": f"mobility solves/s, {entry['K']} star-shaped islands, N = {entry['N']} (FMM near sum, FP64, "
                     "residual 1e-10)",
           "value": 1.0 / entry["solve_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * entry["solve_s"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": wl["name"], "K": entry["K"], "N": entry["N"], "nodes_per_island": 350,
                      "area_fraction": 0.2, "near_sum": "fmm", "fmm_order": st["order"], "precond": "block",
                      "tol": 1e-10},
           "roofline": roofline, "cpu_baseline": cpu, "series": series}
    print(json.dumps(out), flush=True)


def bench_stepping(args):
    """Forward-Euler time stepping of the three held-out trajectory cells (seeds 6000-6002,
    70-100 ellipses, dt 0.01) with relaxed FP32 products and the block preconditioner, from
    a zero guess, without the network: --steps steps per cell after one untimed step (which
    builds the preconditioner and captures the iteration graphs). Every step re-sets the
    geometry and solves to the FP64 residual 1e-10. value = steps per second over the three
    cells."""
    import numpy as np
    import torch

    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W
    cells, secs, steps = [], 0.0, 0
    for sd in (6000, 6001, 6002):
        wl = W.trajectory_cell(sd)
        s = spm.Solver("cuda:0", precision=spm.SPM_FP32_RELAXED, precond=spm.SPM_PRECOND_BLOCK).set_workload(wl)
        s.step(0.01, 1, 0.0, wl["centers"], wl["theta"])
        s.set_workload(wl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.step(0.01, args.steps, 0.0, wl["centers"], wl["theta"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        secs += dt
        steps += args.steps
        its = [i["iterations"] for i in r["infos"]]
        cells.append({"seed": sd, "N": s.N, "particles": s.No, "ms_per_step": 1e3 * dt / args.steps,
                      "iterations_mean": float(np.mean(its)),
                      "max_rel_residual": max(i["rel_residual"] for i in r["infos"])})
        log(f"[bench] stepping seed {sd}: {cells[-1]}")
        s.close()
    out = {"metric": "time steps/s of forward-Euler stepping, relaxed FP32 + block preconditioner (FP64 residual 1e-10)",
           "value": steps / secs, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": 3,
           "ms_per_step": 1e3 * secs / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "trajectories_25-100_ellipses_phi0.3_dt0.01", "eval_seeds": "6000-6002",
                      "precision": "fp32_relaxed", "precond": "block", "x0": "zero"},
           "cells": cells, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_learned(args):
    """Time stepping with the learned warm start. Training data: forward-Euler
    trajectories run by the solver itself (seeds 5000..5009, 25-100 ellipses at area
    fraction 0.3, dt 0.01, up to `--train-steps` steps each); the network is trained
    on the device (BF16 matrix-core kernels, Adam). Evaluation: held-out trajectories
    (seeds 6000..6002), `--eval-steps` steps each, every variant to the FP64 residual
    1e-10: (i) FP64 from zero, (ii) FP64 from the previous step, (iii) FP32+IR from zero,
    (iv) network warm start + block preconditioner in FP64, FP32+IR and relaxed FP32; each
    of the ingredients alone beside them. value = steps per second of the fastest variant
    overall (with or without the network); network_effect gives, for each solver, the time
    and iterations with the network's warm start relative to the same solver from zero."""
    import numpy as np
    import torch

    from paper_1912_04501_amd import learned as L
    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W
    train_steps = int(os.environ.get("SPM_BENCH_TRAIN_STEPS", "200"))
    eval_steps = int(os.environ.get("SPM_BENCH_EVAL_STEPS", "50"))
    t0 = time.perf_counter()
    X, T, solves = L.generate(range(5000, 5010), train_steps, log=log)
    t_data = time.perf_counter() - t0
    net = spm.MLP("cuda:0")
    net.set_params(L.init_params(0))
    t0 = time.perf_counter()
    losses = L.train(net, X, T, epochs=30, batch=256, lr=1e-3, lr_final=1e-5, seed=0, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    Z, P, NW, B, IR = spm.SPM_X0_ZERO, spm.SPM_X0_PREVIOUS, spm.SPM_X0_NETWORK, spm.SPM_PRECOND_BLOCK, spm.SPM_FP32_IR
    RX = spm.SPM_FP32_RELAXED
    variants = [("fp64_zero", dict(x0=Z)),
                ("fp64_previous", dict(x0=P)),
                ("fp64_network", dict(x0=NW)),
                ("fp64_zero_precond", dict(x0=Z, precond=B)),
                ("fp64_network_precond", dict(x0=NW, precond=B)),
                ("fp32ir_zero", dict(x0=Z, precision=IR)),
                ("fp32ir_zero_precond", dict(x0=Z, precond=B, precision=IR)),
                ("fp32ir_network_precond", dict(x0=NW, precond=B, precision=IR)),
                ("fp32relaxed_zero", dict(x0=Z, precision=RX)),
                ("fp32relaxed_zero_precond", dict(x0=Z, precond=B, precision=RX)),
                ("fp32relaxed_network_precond", dict(x0=NW, precond=B, precision=RX))]
    res = {}
    for name, cfg in variants:
        its, secs, steps, res_max, fb = [], 0.0, 0, 0.0, 0
        for sd in range(6000, 6003):
            wl = W.trajectory_cell(sd)
            s = spm.Solver("cuda:0", **cfg).set_workload(wl)
            s.set_network(net)
            s.step(0.01, 1, 0.0, wl["centers"], wl["theta"])   # warm-up (graphs, preconditioner)
            s.set_workload(wl)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = s.step(0.01, eval_steps, 0.0, wl["centers"], wl["theta"])
            torch.cuda.synchronize()
            secs += time.perf_counter() - t1
            steps += eval_steps
            its += [i["iterations"] for i in r["infos"]]
            res_max = max(res_max, max(i["rel_residual"] for i in r["infos"]))
            fb += sum(i["fallback"] for i in r["infos"])
            s.close()
        res[name] = {"steps_per_s": steps / secs, "ms_per_step": 1e3 * secs / steps,
                     "iterations_mean": float(np.mean(its)), "max_rel_residual": res_max, "fallbacks": fb}
        log(f"[bench] {name}: {res[name]}")
    best = max(res, key=lambda k: res[k]["steps_per_s"])
    # the network's effect at fixed solver settings: time and iterations with / without it
    effect = {}
    for a, b in (("fp64_network", "fp64_zero"), ("fp64_network_precond", "fp64_zero_precond"),
                 ("fp32ir_network_precond", "fp32ir_zero_precond"),
                 ("fp32relaxed_network_precond", "fp32relaxed_zero_precond")):
        effect[a] = {"time_ratio": res[a]["ms_per_step"] / res[b]["ms_per_step"],
                     "iterations_ratio": res[a]["iterations_mean"] / res[b]["iterations_mean"]}
    best_net = min(effect, key=lambda k: res[k]["ms_per_step"])
    out = {"metric": "time steps/s of forward-Euler stepping, fastest solver (FP64 residual 1e-10)",
           "value": res[best]["steps_per_s"], "unit": "steps/s", "n_gpus": 1, "steps": 3 * eval_steps,
           "warmup": 3, "ms_per_step": res[best]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if best.startswith("fp64") else "f32+f64",
           "data": "synthetic", "config": {"workload": "trajectories_25-100_ellipses_phi0.3_dt0.01",
                                           "train_seeds": "5000-5009", "eval_seeds": "6000-6002",
                                           "train_steps": train_steps, "eval_steps": eval_steps, "best": best,
                                           "best_with_network": best_net},
           "network_effect": effect,
           "training": {"samples": int(X.shape[0]), "solves": solves, "data_s": t_data, "train_s": t_train,
                        "adam_steps": int(len(losses)), "final_loss": float(np.mean(losses[-100:]))},
           "variants": res, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


# Sec. 8: the two runs' stars, centres (1/4, 1/4) and (3/4, 3/4) of the unit cell, and the
# fit window and published fit of mu_eff(t) ~ c |t - t*|^(-beta) (context only)
JAMMING = {4: {"s": 0.25, "second_theta": 0.0, "t_end": 0.46, "window": (0.40, 0.44), "tol": 1e-9,
               "paper": {"c": 2.187, "t_star": 0.458, "beta": 2.431}},
           5: {"s": 0.275, "second_theta": 0.7853981633974483, "t_end": 0.475, "window": (0.40, 0.45), "tol": 1e-8,
               "paper": {"c": 12.16, "t_star": 0.472, "beta": 1.31}}}


def fit_blowup(t, mu):
    """Nonlinear least squares of mu = c |t - t*|^(-beta) in relative residuals, t* beyond
    the last sample; returns (c, t*, beta, relative residual 2-norm)."""
    import numpy as np
    from scipy.optimize import least_squares

    t = np.asarray(t, float)
    mu = np.asarray(mu, float)

    def res(p):
        c, ts, be = p
        return (c * np.abs(ts - t) ** (-be) - mu) / mu

    best = None
    for ts0 in t[-1] + np.array([0.005, 0.02, 0.05, 0.1]):
        for be0 in (1.0, 2.0, 3.0):
            c0 = float(np.median(mu * np.abs(ts0 - t) ** be0))
            r = least_squares(res, [c0, ts0, be0], bounds=([0.0, t[-1] + 1e-9, 0.0], [np.inf, 10.0, 20.0]))
            if best is None or r.cost < best.cost:
                best = r
    c, ts, be = best.x
    return float(c), float(ts), float(be), float(np.linalg.norm(best.fun) / np.sqrt(len(t)))


def bench_jamming(args):
    """Forward Euler of two star-shaped particles r = s (1 + cos(t)/2) in a unit cell
    sheared at rate 1 (Sec. 7, Sec. 8 Examples 4 and 5), plain FP64 GMRES to 1e-10 every
    step, until the particles jam: mu_eff(t) blows up and the solve or the gap check
    stops the run. value = time steps per second; the fit of mu_eff(t) on the examples'
    window is reported beside it with the paper's fit as context."""
    import numpy as np
    import torch

    from paper_1912_04501_amd import spm
    from paper_1912_04501_amd import workloads as W
    ex = JAMMING[args.example]
    t_end = ex["t_end"] if args.t_end is None else args.t_end
    if args.jam_tol is None:
        args.jam_tol = ex["tol"]
    wl = W.two_stars(s=ex["s"], A=0.5, omega=float(args.omega), second_theta=ex["second_theta"], n_nodes=args.nodes)
    s = spm.Solver("cuda:0", precision=spm.SPM_FP64, max_iter=2000, tol=args.jam_tol)
    s.set_workload(wl)
    tuned = None
    if not args.no_tune:   # launch shapes for this node count; they persist while N is unchanged
        tuned = s.autotune(args.tune_cache)
        log(f"[jam] autotuned near sum: {tuned}")
    c, th, t = np.array(wl["centers"], float), np.array(wl["theta"], float), 0.0
    ts, mus, its, gaps = [], [], [], []
    n_total = int(round(t_end / args.dt))
    chunk = 20
    stop = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while len(mus) < n_total and stop is None:
        n = min(chunk, n_total - len(mus))
        try:
            r = s.step(args.dt, n, t, c, th)
        except spm.SpmError:
            # replay the chunk one step at a time from its start to keep every good step
            # (a failed step leaves the handle without particles: set the chunk's start again)
            for _ in range(n):
                try:
                    s.set_workload(dict(wl, centers=c, theta=th, skew=wl["skew"] + t))
                    r = s.step(args.dt, 1, t, c, th)
                except spm.SpmError as e:
                    stop = f"{e} at t = {t:.5f}"
                    break
                ts.append(t)
                mus.append(float(r["mu_eff"][0]))
                its.append(r["infos"][0]["iterations"])
                gaps.append(r["infos"][0]["min_gap"])
                c, th, t = r["centers"], r["theta"], r["t"]
            if stop is None:   # every step of the chunk converged one at a time: go on
                s.set_workload(dict(wl, centers=c, theta=th, skew=wl["skew"] + t))
                log(f"[jam] t = {t:.4f} mu_eff = {mus[-1]:.6g} its = {its[-1]} gap = {gaps[-1]:.3e} (steps taken singly)")
            continue
        ts += [t + k * args.dt for k in range(n)]
        mus += r["mu_eff"].tolist()
        its += [i["iterations"] for i in r["infos"]]
        gaps += [i["min_gap"] for i in r["infos"]]
        c, th, t = r["centers"], r["theta"], r["t"]
        log(f"[jam] t = {t:.4f} mu_eff = {mus[-1]:.6g} its = {its[-1]} gap = {gaps[-1]:.3e}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ts, mus = np.array(ts), np.array(mus)

    def fit_on(lo, hi):
        w = (ts >= lo - 1e-12) & (ts <= hi + 1e-12)
        if w.sum() < 5:
            return None
        cf, tsf, bf, rr = fit_blowup(ts[w], mus[w])
        return {"c": cf, "t_star": tsf, "beta": bf, "rel_residual": rr, "window": [lo, hi], "samples": int(w.sum())}

    lo, hi = ex["window"] if args.window is None else args.window
    fit = fit_on(lo, hi)
    # the same window width ending as far before this run's last step as the paper's
    # window ends before its t*
    lead = ex["paper"]["t_star"] - ex["window"][1]
    width = ex["window"][1] - ex["window"][0]
    fit_end = fit_on(ts[-1] - lead - width, ts[-1] - lead) if len(ts) else None
    every = 1 if args.full_series else max(1, len(ts) // 40)
    out = {"metric": f"time steps/s (two-star jamming, Sec. 8 Example {args.example}, FP64 residual {args.jam_tol:g})",
           "value": len(mus) / secs, "unit": "steps/s", "n_gpus": 1, "steps": len(mus), "warmup": 0,
           "ms_per_step": 1e3 * secs / max(1, len(mus)), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"two_stars_example{args.example}", "nodes_per_star": args.nodes, "dt": args.dt,
                      "tol": args.jam_tol, "autotuned": tuned is not None,
                      "t_end": t_end, "s": ex["s"], "A": 0.5, "omega": args.omega,
                      "second_theta": ex["second_theta"]},
           "stopped": stop, "t_last": float(ts[-1]) if len(ts) else 0.0,
           "state_end": {"t": float(t), "centers": np.asarray(c).reshape(-1).tolist(),
                         "theta": np.asarray(th).tolist()},
           "iterations": {"first": its[0] if its else None, "last": its[-1] if its else None,
                          "max": max(its) if its else None},
           "mu_eff_series": [[float(a), float(b), float(g)] for a, b, g in zip(ts[::every], mus[::every],
                                                                             gaps[::every])]
           + ([[float(ts[-1]), float(mus[-1]), float(gaps[-1])]] if len(ts) else []),
           "fit": fit, "fit_before_end": fit_end, "paper_fit": ex["paper"], "roofline": None,
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
