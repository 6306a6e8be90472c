#!/usr/bin/env python3
"""Benchmark: 3D doubly quasi-periodic Green's function G_d evaluations per second.

Workload (the metric's 3D G_d configuration): k = 3.7, alpha = (0.2, 0.35),
256 x 256 modes in (x1, x2), 64 x3 slices on [-1, 1), 1e7 targets uniform in
[0, 2pi]^2 x [-1, 1] at least 1e-3 from the lattice (seed 2).  One step is the
whole method for one instance: FP64 coefficient fill, inverse FFTs to the
near grid and the far slab (Algorithm 3.1 step 1), and the calculation step
for all 1e7 targets (step 2), with targets already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec c64|c128]
    python bench.py --workload batched2d     # 64 2D instances, uneven x1 sizes, 1e6 targets each
    python bench.py --workload maxwell3d     # Maxwell tensor, 512 x 512 modes, 32 slices, 1e6 targets
    python bench.py --workload surrogate     # MLP surrogate vs the plain method, 1e4 instances x 1e4 targets
    python bench.py --workload g2d_grad      # gradient of the 2D G, 1024 x-modes, 128 slices, 1e7 targets
    python bench.py --workload g2d_hess_diff # second-derivative differences, two wavenumbers, same grid
    python bench.py --workload g2d_ho        # 2D G with the degree-2 and -3 log terms removed, same grid

Prints one JSON line.  The per-kernel durations behind ``roofline`` are HIP
events recorded by the library on the stream its kernels run on.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

K, A1, A2 = 3.7, 0.2, 0.35
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(name, info, counts, esize):
    """Bytes a kernel class must move per launch (what the method reads/writes at least once).
    counts: targets in total, near (|x3| <= c) and far."""
    m1, m2, m3, nf = info.m1, info.m2, info.m3, info.n_fields
    ncell = m1 * m2 * m3
    nfar, nfo = info.far_m1 * info.far_m2 * info.far_slices, info.far_fields
    T, Tn, Tf = counts
    if name == "gather":       # near tiles: their targets in (3 x f64) + result out, the near grid read once
        return Tn * (24 + esize) + ncell * esize * nf
    if name == "gather_far":   # far tiles: their targets + results, the far slab read once
        return Tf * (24 + esize) + nfar * esize * nfo
    if name == "fill":         # coefficient write
        return ncell * esize * nf
    if name in ("fft_t", "fft_2", "fft_1"):
        return 2 * ncell * esize * nf
    if name == "far":          # the far slab written once (in 3D with its x2 transform)
        return nfar * esize * nfo
    if name == "far_fft":      # the x1 pass over the far slab
        return 2 * nfar * esize * nfo
    if name == "bin":          # coordinates read once (counts, then scans of the small count table)
        return T * 24
    if name == "bin_place":    # coordinates read, 32-byte tile-ordered record written per target
        return T * (24 + 32)
    return 0


# timer classes that bracket exactly one kernel launch (candidates for the roofline kernel)
SINGLE_KERNEL = ("fill", "fft_t", "fft_2", "fft_1", "far", "gather", "gather_far", "bin_place")


# the autotuner's cache of FFT tile choices (per length, axis and precision), on the local disk
TUNE_FILE = os.path.join(os.environ.get("TMPDIR", "/tmp"), "qpgf_tune.txt")


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(x_np, sample, info):
    """The oracle as it stands, on the host: its full-size preparation (coefficients and direct-DFT
    grids) plus the evaluation of a seeded sample of the targets (near ones by interpolation, far ones
    by the series), the evaluation extrapolated linearly to all targets.  Returns the record and the
    oracle's values at the sample (for the per-result parity of the GPU results)."""
    import threadpoolctl
    from oracle import method
    t0 = time.perf_counter()
    st = method.prepare_3d(K, A1, A2, info.m1 // 2, info.m2 // 2, info.m3 // 2)
    t1 = time.perf_counter()
    o = method.evaluate_3d(st, x_np[sample])
    t2 = time.perf_counter()
    T, n_sample = len(x_np), len(sample)
    t_full = (t1 - t0) + (t2 - t1) * T / n_sample
    blas = max([p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()] + [1])
    rec = {"value": T / t_full, "unit": "evals/s", "cores": blas, "kind": "oracle",
           "host_cores": os.cpu_count(),
           "threads": f"the direct-DFT grid sums (numpy tensordot) run on the BLAS pool of {blas} threads; "
                      f"the coefficients, the interpolation and the series of the far branch are "
                      f"single-threaded numpy",
           "sample": f"full-size preparation (coefficients + direct-DFT grids, {t1 - t0:.1f} s) + a sample of "
                     f"{n_sample} of {T} targets, seeded ({t2 - t1:.1f} s; far ones by the series), evaluation "
                     f"extrapolated linearly to {T} targets"}
    return rec, o


def parity_err(g, o):
    """max_i |g_i - o_i| / max(|o_i|, RMS |o|) over the finite oracle values."""
    import numpy as np
    ok = np.isfinite(o)
    g, o = np.asarray(g)[ok].astype(np.complex128), o[ok]
    s = np.sqrt(np.mean(np.abs(o) ** 2))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), s)))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prec", choices=["c64", "c128"], default=None,
                    help="gd3d: precision of the headline value (default c128; the other one is timed beside "
                         "it); other workloads: their precision (default c64)")
    ap.add_argument("--targets", type=int, default=10_000_000)
    ap.add_argument("--modes", default="256,256,64")
    ap.add_argument("--cpu-sample", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["gd3d", "batched2d", "maxwell3d", "surrogate", "g2d_grad", "g2d_hess_diff", "g2d_ho"], default="gd3d")
    ap.add_argument("--train-instances", type=int, default=2000)
    ap.add_argument("--train-per", type=int, default=8192)
    ap.add_argument("--train-epochs", type=float, default=4.0)
    ap.add_argument("--members", type=int, default=3)
    ap.add_argument("--query-instances", type=int, default=10000)
    ap.add_argument("--query-per", type=int, default=10000)
    ap.add_argument("--tol", type=float, default=1e-4,
                    help="surrogate: accept a value when its calibrated error estimate is below tol |G_d|")
    ap.add_argument("--calib-instances", type=int, default=200)
    ap.add_argument("--calib-per", type=int, default=4096)
    ap.add_argument("--surrogate-wood", type=float, default=0.3,
                    help="surrogate domain: instances with min |beta| below this take the plain method")
    ap.add_argument("--sequential", action="store_true",
                    help="time prepare + evaluate (no binning beside the preparation) instead of the combined call")
    ap.add_argument("--no-gate", action="store_true",
                    help="skip the second timing at the grid that meets p99 <= 1e-6 against the lattice sum")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling rocprofv3 FETCH/WRITE counters)")
    args = ap.parse_args()
    if args.prec is None:
        args.prec = "c128" if args.workload == "gd3d" else "c64"
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this implementation runs on exactly one GPU (--gpus 1); "
                                   "the decomposition over several GPUs is described, not implemented"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1801_05977_amd import qpgf, workloads

    if args.workload == "batched2d":
        print(json.dumps(run_batched2d(args)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(run_surrogate(args)), flush=True)
        return
    if args.workload == "maxwell3d":
        print(json.dumps(run_maxwell3d(args)), flush=True)
        return
    if args.workload == "g2d_grad":
        print(json.dumps(run_g2d_grad(args)), flush=True)
        return
    if args.workload == "g2d_hess_diff":
        print(json.dumps(run_g2d_hess_diff(args)), flush=True)
        return
    if args.workload == "g2d_ho":
        print(json.dumps(run_g2d_ho(args)), flush=True)
        return
    m1, m2, m3 = (int(v) for v in args.modes.split(","))
    T = args.targets
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    other = qpgf.C128 if prec == qpgf.C64 else qpgf.C64
    pname = {qpgf.C128: "c128", qpgf.C64: "c64"}
    x_np = workloads.targets(T, 3, seed=2)
    x = torch.from_numpy(x_np).cuda()
    Tn = int(np.count_nonzero(np.abs(x_np[:, 2]) <= 0.6))
    counts = (T, Tn, T - Tn)
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(T, args.cpu_sample, replace=False))
    sample_d = torch.from_numpy(sample).cuda()

    def run(pr):
        """Time the step on precision pr; per-kernel durations; results at the parity sample."""
        plan = qpgf.Plan(qpgf.KIND_GD3D, pr, m1, m2, m3)
        # the FFT tiles the autotuner measures for this plan's shapes (qpgf_plan_autotune), once,
        # before anything is timed
        plan.autotune(TUNE_FILE)
        out = plan.out_tensor(T)
        esize = 8 if pr == qpgf.C64 else 16
        print(f"[bench] plan {m1}x{m2}x{m3} {pname[pr]}, T={T}, warmup {args.warmup}, steps {args.steps}",
              file=sys.stderr, flush=True)

        def step():
            if args.sequential:
                plan.prepare(K, A1, A2)
                plan.evaluate(x, out)
            else:
                plan(K, A1, A2, x, out)     # qpgf_gd3d: binning beside the preparation

        t = _timed(step, args.steps, args.warmup)
        print(f"[bench] {pname[pr]}: {t * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        at_sample = out[sample_d].cpu().numpy()
        # per-kernel durations, from HIP events on the stream each kernel runs on; kernels
        # one at a time (prepare, then evaluate), so no duration includes a neighbour's share
        plan.enable_timing(True)
        for _ in range(args.steps):
            plan.prepare(K, A1, A2)
            plan.evaluate(x, out)
        torch.cuda.synchronize()
        tim = plan.timing()
        plan.enable_timing(False)
        kernels = {}
        for name, (ms, n) in tim.items():
            if n:
                avg = ms / n
                b = algorithmic_bytes(name, plan.info, counts, esize)
                kernels[name] = {"avg_ms": round(avg, 5), "launches_per_step": n // args.steps,
                                 "alg_bytes": b, "GBps": round(b / (avg * 1e-3) / 1e9, 1) if b else None}
        for name, v in kernels.items():
            print(f"[bench]   {name:10s} {v['avg_ms']:.4f} ms  {v['GBps']} GB/s", file=sys.stderr, flush=True)
        acc = accuracy_vs_truth(plan)
        info = plan.info
        del out
        plan.close()
        return t, kernels, acc, at_sample, info

    t_main, kernels, acc, g_main, info = run(prec)
    t_oth, kernels_oth, acc_oth, g_oth, _ = run(other)
    value = T / t_main
    dom = max((n for n in kernels if n in SINGLE_KERNEL),
              key=lambda n: kernels[n]["avg_ms"] * kernels[n]["launches_per_step"])
    d = kernels[dom]
    achieved = d["alg_bytes"] / (d["avg_ms"] * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"{dom}_gd3d_{args.prec}_traffic.json")
    if os.path.exists(tfile):
        rec = json.load(open(tfile))
        if rec.get("source_hash") == source_hash(rec.get("sources", [])) and rec.get("prec") == args.prec:
            traffic = rec.get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    if dom == "gather_far":
        # the far gather reads every stencil node from LDS (far_points along x1, far_points_t along
        # x2 and x3 per far target), against the LDS read rate of 128 bytes per clock per CU
        # (256 CUs, 2.4 GHz)
        nodes = info.far_points * info.far_points_t ** 2
        lds_bytes = counts[2] * nodes * (8 if prec == qpgf.C64 else 16)
        lds_peak = 128 * 256 * 2.4e9 / 1e12
        lds_ach = lds_bytes / (d["avg_ms"] * 1e-3) / 1e12
        roofline["lds"] = {"bytes_per_launch": lds_bytes, "achieved": round(lds_ach, 2), "peak": round(lds_peak, 1),
                           "unit": "TB/s", "frac": round(lds_ach / lds_peak, 3)}

    gate = None
    if not args.no_gate:
        gate = {pname[prec]: run_gate(args, x, prec)}
        gate[pname[other]] = run_gate(args, x, other)

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    del x

    base, parity = None, None
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        print(f"[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        # the oracle evaluates the sampled targets (the first entries of the sample order)
        base, o = cpu_baseline(x_np, sample, info)
        parity = {pname[prec]: parity_err(g_main, o), pname[other]: parity_err(g_oth, o), "n": int(len(o)),
                  "reference": "the FP64 oracle (near: the method computed plainly; far: the series) at a seeded "
                               "sample of the benchmark targets; error max_i |g - o| / max(|o|, RMS |o|)"}

    line = {
        "metric": "Green's evals/sec at 1e-6 rel err (3D G_d), plain vs batched/surrogate",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_main * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": pname[prec], "data": "synthetic",
        "config": {"workload": "gd3d k=3.7 alpha=(0.2,0.35)", "modes": [m1, m2], "slices": m3,
                   "targets": T, "method": "plain, prepare + evaluate" if args.sequential else "plain",
                   "parallelism": "none"},
        "roofline": roofline,
        "cpu_baseline": base,
        "accuracy_vs_truth": acc,
        "parity_vs_oracle": parity,
        "gate": gate,
        f"value_{pname[other]}": T / t_oth,
        f"ms_per_step_{pname[other]}": t_oth * 1e3,
        f"accuracy_vs_truth_{pname[other]}": acc_oth,
        "kernel_timing": "HIP events per kernel, kernels one at a time (prepare, then evaluate); the timed "
                         "steps use the combined call, which bins the targets beside the preparation",
        "kernels": kernels,
        f"kernels_{pname[other]}": kernels_oth,
    }
    print(json.dumps(line), flush=True)


TRUTH = os.path.join(ROOT, "tests", "golden", "truth_gd3d_k3.7.txt")
GATE_MODES = (512, 512, 128)


def accuracy_vs_truth(plan):
    """Error of the plan's G_d at the stored exact values (lattice sum at 2000 of the benchmark targets):
    |g - o| / max(|o|, RMS |o|), median / 99th percentile / max."""
    import numpy as np
    import torch
    if not os.path.exists(TRUTH):
        return None
    d = np.loadtxt(TRUTH)
    o = d[:, 4] + 1j * d[:, 5]
    g = plan(K, A1, A2, torch.from_numpy(d[:, 1:4].copy()).cuda()).cpu().numpy().astype(np.complex128)
    s = np.sqrt(np.mean(np.abs(o) ** 2))
    e = np.abs(g - o) / np.maximum(np.abs(o), s)
    return {"p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)), "max": float(e.max()),
            "n": int(len(o)), "reference": "lattice sum eq. 1.3 at 2000 benchmark targets with |x3| >= 0.02"}


def run_gate(args, x, prec):
    """The same instance and targets on the smallest power-of-two grid whose p99 error against the
    lattice sum is <= 1e-6 (512 x 512 modes, 128 slices)."""
    import torch
    from paper_1801_05977_amd import qpgf
    plan = qpgf.Plan(qpgf.KIND_GD3D, prec, *GATE_MODES)
    plan.autotune(TUNE_FILE)
    out = plan.out_tensor(x.shape[0])
    t = _timed(lambda: plan(K, A1, A2, x, out), args.steps, args.warmup)
    acc = accuracy_vs_truth(plan)
    plan.enable_timing(True)
    for _ in range(args.steps):     # kernels one at a time, as for the main configuration
        plan.prepare(K, A1, A2)
        plan.evaluate(x, out)
    torch.cuda.synchronize()
    kern = {k_: round(v[0] / v[1], 5) for k_, v in plan.timing().items() if v[1]}
    plan.close()
    del out
    print(f"[bench] gate grid {GATE_MODES}: {t * 1e3:.3f} ms/step, p99 {acc and acc['p99']}", file=sys.stderr,
          flush=True)
    return {"modes": list(GATE_MODES[:2]), "slices": GATE_MODES[2], "value": x.shape[0] / t, "ms_per_step": t * 1e3,
            "accuracy_vs_truth": acc, "kernels_avg_ms": kern}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def run_batched2d(args):
    """64 instances k ~ U[1,20], alpha ~ U[-0.5,0.5] (Wood and special cases rejected),
    x1 sizes 256 * U{1..8}, 128 transverse slices, 1e6 targets each, complex64."""
    import numpy as np
    import torch
    from paper_1801_05977_amd import qpgf, workloads
    n, per, M2 = 64, 1_000_000, 128
    k, a = workloads.instances_2d(n, seed=1, k_range=(1.0, 20.0), n2_max=M2 // 2)
    m1 = workloads.x1_sizes_2d(n, seed=1)
    t_off = np.arange(n + 1, dtype=np.int64) * per
    x = torch.from_numpy(workloads.targets(n * per, 2, seed=1)).cuda()
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    P = qpgf.Plan(qpgf.KIND_G2D, prec, max(m1), M2)
    P.autotune(TUNE_FILE)
    out = P.out_tensor(n * per)
    t_batched = _timed(lambda: P.batched(k, a, m1, t_off, x, out), args.steps, args.warmup)
    # the same work as a loop of single-instance calls (one plan per x1 size)
    plans = {M: qpgf.Plan(qpgf.KIND_G2D, prec, M, M2) for M in sorted(set(m1))}
    for p_ in plans.values():
        p_.autotune(TUNE_FILE)
    xs = [x[i * per:(i + 1) * per] for i in range(n)]
    outs = [out[i * per:(i + 1) * per] for i in range(n)]

    def loop():
        for i in range(n):
            plans[m1[i]](k[i], a[i], 0.0, xs[i], outs[i])
    t_loop = _timed(loop, max(1, args.steps // 2), 1)
    T = n * per
    return {"metric": "Green's evals/sec, batched 2D instances", "value": T / t_batched, "unit": "evals/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_batched * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
            "data": "synthetic",
            "config": {"workload": "g2d batched: 64 instances k~U[1,20] alpha~U[-0.5,0.5]",
                       "x1_modes": sorted(set(m1)), "slices": M2, "targets": T, "method": "batched+graph"},
            "loop_of_single_instances": {"value": T / t_loop, "ms_per_step": t_loop * 1e3}}


def run_maxwell3d(args):
    """Maxwell tensor: k = 5.3, alpha = (0.1, 0.4), 512 x 512 modes, 32 slices, 1e6 targets, complex64."""
    import torch
    from paper_1801_05977_amd import qpgf, workloads
    T = 1_000_000
    x = torch.from_numpy(workloads.targets(T, 3, seed=3)).cuda()
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    P = qpgf.Plan(qpgf.KIND_MAXWELL3D, prec, 512, 512, 32)
    P.autotune(TUNE_FILE)
    out = P.out_tensor(T)
    t = _timed(lambda: P(5.3, 0.1, 0.4, x, out), args.steps, args.warmup)
    P.enable_timing(True)
    for _ in range(args.steps):
        P(5.3, 0.1, 0.4, x, out)
    torch.cuda.synchronize()
    kern = {k_: round(v[0] / v[1], 5) for k_, v in P.timing().items() if v[1]}
    return {"metric": "Maxwell tensor evals/sec (6 components)", "value": T / t, "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
            "config": {"workload": "maxwell3d k=5.3 alpha=(0.1,0.4)", "modes": [512, 512], "slices": 32,
                       "targets": T, "method": "plain"},
            "kernels_avg_ms": kern}


def run_g2d_grad(args):
    """Gradient of the 2D G (Section 2.4.1): k = 2.1, alpha = 0.3, 1024 x-modes, 128 slices,
    1e7 targets U([0, 2pi] x [-1, 1]), complex64; one prepare + evaluate per step."""
    import torch
    from paper_1801_05977_amd import qpgf, workloads
    T, M1, M2 = 10_000_000, 1024, 128
    x = torch.from_numpy(workloads.targets(T, 2, seed=0)).cuda()
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    P = qpgf.Plan(qpgf.KIND_G2D_GRAD, prec, M1, M2)
    out = P.out_tensor(T)
    t = _timed(lambda: P(2.1, 0.3, 0.0, x, out), args.steps, args.warmup)
    P.enable_timing(True)
    for _ in range(args.steps):
        P(2.1, 0.3, 0.0, x, out)
    torch.cuda.synchronize()
    kern = {k_: round(v[0] / v[1], 5) for k_, v in P.timing().items() if v[1]}
    # the same step with the cut-off ring interpolated (ring_interp), beside
    Pr = qpgf.Plan(qpgf.KIND_G2D_GRAD, prec, M1, M2, ring_interp=1)
    tr = _timed(lambda: Pr(2.1, 0.3, 0.0, x, out), args.steps, args.warmup)
    Pr.enable_timing(True)
    for _ in range(args.steps):
        Pr(2.1, 0.3, 0.0, x, out)
    torch.cuda.synchronize()
    kern_r = {k_: round(v[0] / v[1], 5) for k_, v in Pr.timing().items() if v[1]}
    Pr.close()
    esize = 8 if prec == qpgf.C64 else 16
    # gather: 16 B in, two results and a flag byte out per target, both near fields and far slabs once
    grid_bytes = 2 * (P.info.grid_bytes + P.info.far_grid_bytes)
    alg = T * (16 + 2 * esize + 1) + grid_bytes
    ach = alg / (kern["gather"] * 1e-3) / 1e9
    return {"metric": "2D gradient evals/sec (dG/dx1 and dG/dx2)", "value": T / t, "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
            "config": {"workload": "g2d gradient k=2.1 alpha=0.3", "x1_modes": M1, "slices": M2, "targets": T,
                       "method": "plain"},
            "kernels_avg_ms": kern,
            "ring_interp_1": {"ms_per_step": tr * 1e3, "kernels_avg_ms": kern_r},
            "roofline": {"bound": "hbm", "kernel": "gather", "achieved": round(ach, 1), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(ach / 8000.0, 4), "traffic": None}}


def run_g2d_hess_diff(args):
    """Differences of second derivatives of the 2D G (Section 2.4.2): k1 = 2.1, k2 = 4.35, alpha = 0.3,
    1024 x-modes, 128 slices, 1e7 targets U([0, 2pi] x [-1, 1]), complex64; one prepare + evaluate per step."""
    import torch
    from paper_1801_05977_amd import qpgf, workloads
    T, M1, M2 = 10_000_000, 1024, 128
    x = torch.from_numpy(workloads.targets(T, 2, seed=0)).cuda()
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    P = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, prec, M1, M2)
    out = P.out_tensor(T)
    t = _timed(lambda: P.hess_diff(2.1, 4.35, 0.3, x, out), args.steps, args.warmup)
    P.enable_timing(True)
    for _ in range(args.steps):
        P.hess_diff(2.1, 4.35, 0.3, x, out)
    torch.cuda.synchronize()
    kern = {k_: round(v[0] / v[1], 5) for k_, v in P.timing().items() if v[1]}
    # the same step with the cut-off ring interpolated (ring_interp), beside
    Pr = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, prec, M1, M2, ring_interp=1)
    tr = _timed(lambda: Pr.hess_diff(2.1, 4.35, 0.3, x, out), args.steps, args.warmup)
    Pr.enable_timing(True)
    for _ in range(args.steps):
        Pr.hess_diff(2.1, 4.35, 0.3, x, out)
    torch.cuda.synchronize()
    kern_r = {k_: round(v[0] / v[1], 5) for k_, v in Pr.timing().items() if v[1]}
    Pr.close()
    esize = 8 if prec == qpgf.C64 else 16
    # gather: 16 B in, three results and a flag byte out per target, the three fields once
    alg = T * (16 + 3 * esize + 1) + 3 * (P.info.grid_bytes + P.info.far_grid_bytes)
    ach = alg / (kern["gather"] * 1e-3) / 1e9
    return {"metric": "2D second-derivative-difference evals/sec (d11, d12, d22 of G_k1 - G_k2)", "value": T / t,
            "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
            "data": "synthetic",
            "config": {"workload": "g2d second-derivative differences k1=2.1 k2=4.35 alpha=0.3", "x1_modes": M1,
                       "slices": M2, "targets": T, "method": "plain"},
            "kernels_avg_ms": kern,
            "ring_interp_1": {"ms_per_step": tr * 1e3, "kernels_avg_ms": kern_r},
            "roofline": {"bound": "hbm", "kernel": "gather", "achieved": round(ach, 1), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(ach / 8000.0, 4), "traffic": None}}


def run_g2d_ho(args):
    """The 2D G with the terms of degree 2 and 3 of the log singularity removed as well
    (sing_order = 3, Remark 5.3) and K interpolated in the cut-off ring (ring_interp = 1):
    k = 2.1, alpha = 0.3, 1024 x-modes, 128 slices, 1e7 targets U([0, 2pi] x [-1, 1]); one
    prepare + evaluate per step.  The same step with sing_order 3 alone and with the paper's
    Algorithm 2.1 (sing_order 1, ring_interp 0) is timed beside it."""
    import torch
    from paper_1801_05977_amd import qpgf, workloads
    T, M1, M2 = 10_000_000, 1024, 128
    x = torch.from_numpy(workloads.targets(T, 2, seed=0)).cuda()
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    res = {}
    for order, ring in ((3, 1), (3, 0), (1, 0)):
        P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2, sing_order=order, ring_interp=ring)
        out = P.out_tensor(T)
        t = _timed(lambda: P(2.1, 0.3, 0.0, x, out), args.steps, args.warmup)
        P.enable_timing(True)
        for _ in range(args.steps):
            P(2.1, 0.3, 0.0, x, out)
        torch.cuda.synchronize()
        kern = {k_: round(v[0] / v[1], 5) for k_, v in P.timing().items() if v[1]}
        res[order, ring] = (t, kern, P.info.grid_bytes + P.info.far_grid_bytes)
        P.close()
    t, kern, gb = res[3, 1]
    esize = 8 if prec == qpgf.C64 else 16
    # gather: 16 B in, one result and a flag byte out per target, the near field and far slab once
    alg = T * (16 + esize + 1) + gb
    ach = alg / (kern["gather"] * 1e-3) / 1e9
    return {"metric": "2D G evals/sec, degree-3 singular removal and ring interpolation", "value": T / t,
            "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
            "data": "synthetic",
            "config": {"workload": "g2d k=2.1 alpha=0.3, sing_order 3, ring_interp 1", "x1_modes": M1,
                       "slices": M2, "targets": T, "method": "plain"},
            "kernels_avg_ms": kern,
            "sing_order_3_only": {"ms_per_step": res[3, 0][0] * 1e3, "kernels_avg_ms": res[3, 0][1]},
            "algorithm_2_1": {"ms_per_step": res[1, 0][0] * 1e3, "kernels_avg_ms": res[1, 0][1]},
            "roofline": {"bound": "hbm", "kernel": "gather", "achieved": round(ach, 1), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(ach / 8000.0, 4), "traffic": None}}


def _instances_3d(n, seed, k_range=(1.0, 10.0), a_range=(-0.5, 0.5), min_beta=1e-3, special_tol=1e-6, m3=64):
    """n (k, alpha1, alpha2) with every |k^2 - |alpha + n|^2|^(1/2) >= min_beta (Wood anomalies redrawn) and
    no propagating beta within special_tol of j3 pi (c~ = 1, |j3| <= m3 / 2; special coefficients redrawn)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    j = np.arange(-12, 13)
    J = np.arange(0, m3 // 2 + 1) * math.pi
    while len(out) < n:
        k, a1, a2 = rng.uniform(*k_range), rng.uniform(*a_range), rng.uniform(*a_range)
        d = k * k - (a1 + j[:, None]) ** 2 - (a2 + j[None, :]) ** 2
        if np.sqrt(np.abs(d)).min() < min_beta:
            continue
        b = np.sqrt(d[d > 0])
        if b.size and np.abs(b[:, None] - J[None, :]).min() < special_tol:
            continue
        out.append((k, a1, a2))
    return np.array(out)


def run_surrogate(args):
    """MLP surrogate of the smooth part vs the plain method (Algorithm 3.1, 256 x 256 x 64).

    Training: `train_instances` instances (k ~ U[1,10], alpha ~ U[-1/2,1/2]^2, seed 4, min |beta| >=
    `surrogate_wood`: near a Wood anomaly one mode's amplitude 1/beta is near-singular in (k, alpha), so
    those instances are outside the surrogate's domain and fall back) x `train_per` near-region targets,
    rows from qpgf_surrogate_make_data, Adam with a cosine learning rate in qpgf_surrogate_train.
    Calibration: `calib_instances` further instances (seed 6) x `calib_per` near targets; kappa = 2 x the
    largest ratio |L_mean - L_N| / spread (qpgf_surrogate_calibrate).  Queries: `query_instances` fresh
    instances (seed 5) x `query_per` targets uniform in [0, 2pi]^2 x [-1, 1]; a value is accepted when
    kappa spread <= tol |G_d|, everything else takes the plain method.  A step is all queries through
    qpgf_surrogate_eval; the plain method is timed on the same queries as one qpgf_gd3d call per
    instance."""
    import numpy as np
    import torch
    from paper_1801_05977_amd import qpgf, workloads
    M = (256, 256, 64)
    prec = qpgf.C64 if args.prec == "c64" else qpgf.C128
    P = qpgf.Plan(qpgf.KIND_GD3D, prec, *M)
    mdl = qpgf.Mlp(args.members, 65536, seed=7)
    # ---- training data from the plain method
    t0 = time.perf_counter()
    tr = _instances_3d(args.train_instances, seed=4, min_beta=args.surrogate_wood)
    per = args.train_per
    xtr = torch.from_numpy(workloads.targets(len(tr) * per, 3, seed=40, zmax=0.6)).cuda()
    q, y = mdl.make_data(P, tr[:, 0], tr[:, 1], tr[:, 2], np.arange(len(tr) + 1) * per, xtr)
    del xtr
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    # ---- training
    B = 16384
    n = q.shape[0]
    steps = max(1, int(args.train_epochs * n / B))
    t0 = time.perf_counter()
    loss = mdl.train(q, y, batch=B, steps=steps, lr_max=2e-3, lr_min=1e-5, seed=100)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    final_loss = [float(v) for v in loss.cpu()]
    del q, y
    # ---- calibration of the error estimate on held-out instances
    t0 = time.perf_counter()
    ca = _instances_3d(args.calib_instances, seed=6, min_beta=args.surrogate_wood)
    xc = torch.from_numpy(workloads.targets(len(ca) * args.calib_per, 3, seed=60, zmax=0.6)).cuda()
    kappa = mdl.calibrate(P, ca[:, 0], ca[:, 1], ca[:, 2], np.arange(len(ca) + 1) * args.calib_per, xc,
                          quantile=1.0, safety=2.0)
    del xc
    t_cal = time.perf_counter() - t0
    # ---- queries
    qi = _instances_3d(args.query_instances, seed=5)
    nq, pq = len(qi), args.query_per
    T = nq * pq
    x = torch.from_numpy(workloads.targets(T, 3, seed=5)).cuda()
    t_off = np.arange(nq + 1, dtype=np.int64) * pq
    out = P.out_tensor(T)
    fell = torch.empty(T, dtype=torch.uint8, device="cuda")
    nfb = [0]

    def surrogate():
        nfb[0] = mdl.evaluate(P, qi[:, 0], qi[:, 1], qi[:, 2], t_off, x, args.tol, wood_tol=args.surrogate_wood,
                              rmin=1e-3, out=out, fell_back=fell)[2]
    # seconds per step: at most 3 timed steps and 1 warm-up step
    steps_q, warmup = min(args.steps, 3), min(args.warmup, 1)
    t_s = _timed(surrogate, steps_q, warmup)
    fl = fell.cpu().numpy()
    flag_frac = {name: float(np.count_nonzero(fl & bit)) / T
                 for name, bit in (("far", 2), ("estimate_above_tol", 4), ("wood", 8), ("near_lattice", 16))}
    out_plain = P.out_tensor(T)

    def plain():
        for i in range(nq):
            P(qi[i, 0], qi[i, 1], qi[i, 2], x[i * pq:(i + 1) * pq], out_plain[i * pq:(i + 1) * pq])
    t_p = _timed(plain, steps_q, 1)
    # forward alone (all members, all queries) for the matrix-core roofline
    qall = torch.empty((min(T, 65536 * 16), 6), dtype=torch.float64, device="cuda")
    qall[:, :3] = x[:qall.shape[0]]
    qall[:, 3:] = torch.tensor(qi[0], dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mdl.forward(qall, 0)
    ev0.record()
    for e in range(args.members):
        mdl.forward(qall, e)
    ev1.record()
    torch.cuda.synchronize()
    t_fwd = ev0.elapsed_time(ev1) / 1e3
    flop_q = 2 * (64 * 256 + 3 * 256 * 256 + 2 * 256)
    fwd_tflops = flop_q * qall.shape[0] * args.members / t_fwd / 1e12
    # every accepted value against the plain method in complex128 (relative to |G_d|)
    ref_plan = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C128, *M)
    errs = []
    acc_inst = np.nonzero(np.add.reduceat((fl == 0).astype(np.int64), t_off[:-1]) > 0)[0]
    for i in acc_inst:
        sl = slice(i * pq, (i + 1) * pq)
        ok = fl[sl] == 0
        ref = ref_plan(qi[i, 0], qi[i, 1], qi[i, 2], x[sl]).cpu().numpy()[ok]
        got = out[sl].cpu().numpy().astype(np.complex128)[ok]
        errs.append(np.abs(got - ref) / np.abs(ref))
    errs = np.concatenate(errs) if errs else np.zeros(0)
    acc_err = ({"p50": float(np.percentile(errs, 50)), "p99": float(np.percentile(errs, 99)),
                "max": float(errs.max()), "n": int(errs.size)} if errs.size else {"n": 0})
    return {"metric": "Green's evals/sec, 3D G_d through the MLP surrogate (with fallback)", "value": T / t_s,
            "unit": "evals/s", "n_gpus": 1, "steps": steps_q, "warmup": warmup, "ms_per_step": t_s * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 network, " + args.prec,
            "data": "synthetic",
            "config": {"workload": f"gd3d surrogate: {nq} instances x {pq} targets, k~U[1,10] alpha~U[-0.5,0.5]^2",
                       "modes": [256, 256], "slices": 64, "members": args.members, "tol": args.tol,
                       "surrogate_wood": args.surrogate_wood, "calib_samples": int(len(ca) * args.calib_per),
                       "train_samples": int(len(tr) * per), "train_steps_per_member": steps, "batch": B},
            "kappa": kappa,
            "accepted_fraction": 1.0 - nfb[0] / T,
            "fallback_by_flag": flag_frac,
            "plain_method": {"value": T / t_p, "ms_per_step": t_p * 1e3},
            "gain_vs_plain": t_p / t_s,
            "accepted_rel_err": acc_err,
            "training": {"data_s": t_data, "train_s": t_train, "calibrate_s": t_cal, "final_loss": final_loss},
            "roofline": {"bound": "mfma", "kernel": "forward (all members)", "achieved": fwd_tflops,
                         "peak": 2500.0, "unit": "TFLOP/s", "frac": fwd_tflops / 2500.0, "traffic": None}}


if __name__ == "__main__":
    main()
