#!/usr/bin/env python
"""Benchmark of the MI355X tiled QR: one JSON line on stdout.

Default workload: the square least-squares problem A x = b with A 10240 x
10240 (p = q = 40 tiles of nb = 256) built as U diag(s) V^T from seeded Haar
U, V and log-spaced singular values (condition number kappa), 4 right-hand
sides b = A x_true.  One step = factorization with Q^T b in the same
executor launch + triangular solve + iterative refinement to a backward error
of 1e-12 (the hot path).  The plain FP64 path (the same step without
refinement) is timed beside it on the same input.

With --tree auto (the default) each precision first runs the exhaustive
autotuner over a fixed candidate list of (tree, BS, kernel family) at the
given nb, timing whole steps on the bench input (untimed for the result),
and the timed region then uses each precision's winner (the first listed
candidate within 1% of the fastest); the FP64 path gets the same search.

Throughput counts 2 m n^2 - 2 n^3 / 3 flops per factorization (the
Householder count, Sec. 2.2 of the paper) per step.  Inputs are resident in
HBM before the timed region.

Usage: python bench.py [--steps K] [--warmup W] [--upd f32|bf16|f64]
                       [--workload square|tall] [--kappa K]
                       [--tree auto|flat|greedy|...] [--bs BS] [--kern default|tt|ts]
"""

import argparse
import json
import os
import sys
import time

METRIC = "tiled-QR GFLOP/s & % MFMA peak: mixed+refined vs FP64 at equal LS accuracy"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
HBM_TBPS = 8.0
TREES = {"flat": 0, "sameh-kuck": 1, "binary": 2, "fibonacci": 3, "greedy": 4, "plasma": 5, "asap": 6, "grasap": 7, "hadri": 8}
UPD = {"f64": 0, "f32": 1, "bf16": 2}
KERNS = {"default": 0, "tt": 1, "ts": 2}
# Candidates of the bench's exhaustive autotuner: (tree, BS, kernel family).
# Candidates within TUNE_TIE of the fastest count as ties (timing noise) and
# the earliest in this list wins, so that equivalent trees do not flip from
# run to run.
TUNE_CANDIDATES = [("plasma", 16, "ts"), ("flat", 1, "ts"), ("plasma", 8, "ts"), ("plasma", 32, "ts"),
                   ("greedy", 1, "tt"), ("greedy", 1, "ts"), ("fibonacci", 1, "ts"), ("asap", 1, "ts")]
TUNE_TIE = 0.01
# Table 1 weights by task kind (GEQRT, UNMQR, TSQRT, TSMQR, TTQRT, TTMQR).
UNITS = (4, 6, 6, 12, 2, 6)
# Algorithmic HBM bytes per task in FP64 tiles (nb^2 * 8 bytes), each operand
# read once and each result written once: GEQRT reads and writes a tile;
# UNMQR reads half a tile of reflectors and reads and writes its target;
# TSQRT reads and writes two tiles; TSMQR reads a tile of reflectors and two
# targets and writes the targets; TTQRT reads and writes two triangles;
# TTMQR reads a triangle of reflectors and two targets, writes the targets.
TILE_RW = (2.0, 2.5, 4.0, 5.0, 2.0, 4.5)
# HBM bytes per launch of the executor from rocprofv3 FETCH_SIZE + WRITE_SIZE
# (calibrated by a plain copy; profiles/hbm_traffic_square10240_nb256.md),
# keyed by (workload, update precision, tree, BS, kernels, nb) and valid for
# the executor sources with the given SHA-256 prefix only.
TRAFFIC = {("square", "f32", "flat", 1, "ts", 256): (58.44e9, "2b079dbf6a3a457d"),
           ("square", "bf16", "flat", 1, "ts", 256): (57.58e9, "2b079dbf6a3a457d"),
           ("square", "f64", "flat", 1, "ts", 256): (84.43e9, "2b079dbf6a3a457d")}


def executor_source_hash():
    import hashlib
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in ("kernels.hip", "device.hpp", "hip_prims.hpp"):
        with open(os.path.join(here, "paper_1104_4475_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["square", "tall"], default="square")
    ap.add_argument("--kappa", type=float, default=1e2)
    ap.add_argument("--matrix", choices=["conditioned", "gaussian"], default="conditioned",
                    help="square workload: U diag(s) V^T with condition number kappa, or N(0,1) entries")
    ap.add_argument("--upd", choices=list(UPD), default="f32")
    ap.add_argument("--tree", choices=["auto"] + list(TREES), default="auto")
    ap.add_argument("--kern", choices=list(KERNS), default="default")
    ap.add_argument("--bs", type=int, default=1)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other update precision and the condition-number sweep")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (HBM counter calibration under rocprofv3 --pmc)")
    return ap.parse_args()


def flops(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def update_flop_fraction(p, q, tree, bs, kern):
    """Share of the Table 1 work units spent in update kernels (UNMQR, TSMQR,
    TTMQR) in the task list of (tree, BS, kernel family)."""
    from paper_1104_4475_amd import _lib
    tasks, _ = _lib.schedule(p, q, tree, bs, kern)
    units = [UNITS[k] for k in tasks[:, 0]]
    upd = [UNITS[k] for k in tasks[:, 0] if k in (1, 3, 5)]
    return sum(upd) / sum(units)


def algorithmic_bytes(p, q, nb, tree, bs, kern):
    """HBM bytes of one factorization: TILE_RW tiles per task of the task list
    of (tree, BS, kernel family), FP64 tiles of nb^2 doubles."""
    from paper_1104_4475_amd import _lib
    tasks, _ = _lib.schedule(p, q, tree, bs, kern)
    return sum(TILE_RW[k] for k in tasks[:, 0]) * nb * nb * 8.0


def cpu_baseline(nb, tree, bs, kern, kappa):
    """The FP64 oracle (plain NumPy tiled QR) on a bounded sample of the same
    workload: the conditioned matrix at 1792 x 1792 (p = q = 7 tiles of the
    same nb), with BLAS on all host cores of this process, and once more on
    one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import tqr_inputs
    from oracle import tiled
    n = 7 * nb
    bs = min(bs, 7)  # PlasmaTree's domain size (GRASAP's k) is at most 7 in the sample
    A = tqr_inputs.conditioned(n, kappa, 102, 103)
    cores = len(os.sched_getaffinity(0))
    out = {}
    for threads in (cores, 1):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            tiled.tiled_qr(A, nb, tree, bs, kern)
            out[threads] = time.perf_counter() - t0
    dt = out[cores]
    return {"value": flops(n, n) / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "oracle tiled QR of a %dx%d conditioned matrix (kappa %g), nb=%d, same tree (BS %d) and "
                      "kernels, %d BLAS threads, %.1f s" % (n, n, kappa, nb, bs, cores, dt),
            "seconds": dt, "value_1_thread": flops(n, n) / out[1] / 1e9, "seconds_1_thread": out[1],
            "host_cpus": cores}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the tiled QR here is a single-GPU library "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1104_4475_amd as tqr
    import tqr_inputs

    dev = "cuda"
    nb, nrhs = args.nb, args.nrhs

    def square_matrix(kappa):
        return tqr_inputs.conditioned_device(10240, kappa, tqr_inputs.SEED_C3, tqr_inputs.SEED_C3 + 1, dev).t()

    if args.workload == "square" and args.matrix == "conditioned":
        m = n = 10240
        A = square_matrix(args.kappa)
        workload = "square LS %dx%d, kappa %g, nb %d, %d rhs" % (m, n, args.kappa, nb, nrhs)
    elif args.workload == "square":
        m = n = 10240
        A = tqr_inputs.gaussian_device(m, n, tqr_inputs.SEED_C3, dev).t()
        workload = "square LS %dx%d N(0,1), nb %d, %d rhs" % (m, n, nb, nrhs)
    else:
        m, n = 16384, 2048
        A = tqr_inputs.gaussian_device(m, n, tqr_inputs.SEED_C2, dev).t()
        workload = "tall %dx%d N(0,1), nb %d, %d rhs" % (m, n, nb, nrhs)
    g = torch.Generator(device=dev)
    g.manual_seed(tqr_inputs.SEED_C3_RHS)
    Xt = torch.randn((nrhs, n), generator=g, dtype=torch.float64, device=dev).t()

    def rhs(Am):
        return (Am @ Xt).t().contiguous().t()

    B = rhs(A)
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p, q = m // nb, n // nb
    F = flops(m, n)

    def step(Fh, Am, Bm, tol):
        # One step: factorization with Q^T B in the same executor launch, then
        # the triangular solve and (mixed) refinement against A.
        QtB = Fh.refactor_qtb(Am, Bm)
        return Fh.lstsq(Bm, A0=Am, tol=tol, QtB=QtB)

    def tune(upd, refine):
        """Exhaustive autotuner over TUNE_CANDIDATES: the best of two timed
        steps after one warm-up, per candidate."""
        if args.tree != "auto":
            return (args.tree, args.bs, args.kern), []
        tol = args.tol if refine else 0.0
        table = []
        for tname, bs, kname in TUNE_CANDIDATES:
            if bs > p:
                continue
            Fh = tqr.factor(A, nb, TREES[tname], bs, KERNS[kname], UPD[upd])
            step(Fh, A, B, tol)
            best = float("inf")
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                step(Fh, A, B, tol)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            Fh.sync()
            del Fh
            table.append(((tname, bs, kname), round(1e3 * best, 3)))
        best = min(t for _, t in table)
        return next(c for c, t in table if t <= best * (1.0 + TUNE_TIE)), table

    def measure(upd, refine, choice, Am, Bm, steps, warmup):
        tname, bs, kname = choice
        Fh = tqr.factor(Am, nb, TREES[tname], bs, KERNS[kname], UPD[upd])
        Fh.sync()
        tol = args.tol if refine else 0.0
        for _ in range(warmup):
            X, info = step(Fh, Am, Bm, tol)
        torch.cuda.synchronize()
        times, execs, infos = [], [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, info = step(Fh, Am, Bm, tol)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            execs.append(Fh.exec_ms())
            infos.append(info)
        Fh.sync()
        r = Bm - Am @ X
        eta = (torch.linalg.norm(r, dim=0) /
               (torch.linalg.norm(Am) * torch.linalg.norm(X, dim=0) + torch.linalg.norm(Bm, dim=0))).max().item()
        del Fh
        return {"ms_per_step": 1e3 * sum(times) / len(times), "exec_ms": sum(execs) / len(execs),
                "gflops": F / (sum(times) / len(times)) / 1e9, "backward_err": eta,
                "refine_iters": infos[-1]["iters"], "converged": infos[-1]["converged"], "X": X,
                "choice": choice}

    def run(upd, refine):
        choice, table = tune(upd, refine)
        res = measure(upd, refine, choice, A, B, args.steps, args.warmup)
        res["tune"] = table
        return res

    def peak_for(upd, choice):
        if upd == "f64":
            return PEAK_TFLOPS["f64"]
        tname, bs, kname = choice
        fu = update_flop_fraction(p, q, TREES[tname], bs, KERNS[kname])
        return 1.0 / (fu / PEAK_TFLOPS[upd] + (1.0 - fu) / PEAK_TFLOPS["f64"])

    fp64 = run("f64", refine=False)
    main_res = fp64 if args.upd == "f64" else run(args.upd, refine=True)
    fwd = (torch.linalg.norm(main_res["X"] - fp64["X"]) / torch.linalg.norm(fp64["X"])).item()

    # Dominant kernel: the executor (all tile kernels of the factorization).
    exec_s = main_res["exec_ms"] / 1e3
    tname, bs, kname = main_res["choice"]
    peak = peak_for(args.upd, main_res["choice"])
    achieved = F / exec_s / 1e12
    alg_bytes = algorithmic_bytes(p, q, nb, TREES[tname], bs, KERNS[kname])
    traffic = None
    key = (args.workload, args.upd, tname, bs, kname, nb)
    if key in TRAFFIC and TRAFFIC[key][1] == executor_source_hash():
        traffic = TRAFFIC[key][0]
    # The floor that binds the executor: compute at the MFMA peak, or HBM
    # bytes (the measured traffic when it is current, else the algorithmic
    # bytes) at 8 TB/s.
    t_mfma = F / (peak * 1e12)
    t_hbm = (traffic if traffic is not None else alg_bytes) / (HBM_TBPS * 1e12)
    bound = "hbm" if t_hbm > t_mfma else "mfma"
    if bound == "mfma":
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4)}
    else:
        gbps = alg_bytes / exec_s / 1e9  # algorithmic bytes per launch over its duration
        roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_TBPS * 1e3, "unit": "GB/s",
                "frac": round(gbps / (HBM_TBPS * 1e3), 4)}
    roof.update({"traffic": traffic, "algorithmic_bytes": alg_bytes, "floor_ms": {"mfma": round(1e3 * t_mfma, 3),
                 "hbm": round(1e3 * t_hbm, 3)}, "kernel": "exec_persistent<%d>" % nb,
                 "kernel_ms": round(main_res["exec_ms"], 3), "tflops": round(achieved, 3)})
    line = {
        "metric": METRIC,
        "value": round(main_res["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.upd == "f64" else "f64 panels/residuals + %s MFMA updates" % args.upd,
        "data": "synthetic",
        "config": {"workload": workload, "tree": tname, "bs": bs, "kernels": kname, "nb": nb, "m": m, "n": n,
                   "upd": args.upd, "refine_tol": args.tol if args.upd != "f64" else None,
                   "tuned": args.tree == "auto"},
        "roofline": roof,
        "fp64": {"gflops": round(fp64["gflops"], 2), "ms_per_step": round(fp64["ms_per_step"], 3),
                 "exec_ms": round(fp64["exec_ms"], 3), "backward_err": fp64["backward_err"],
                 "tree": "%s bs %d %s" % fp64["choice"],
                 "frac_fp64_peak": round(F / (fp64["exec_ms"] / 1e3) / 1e12 / PEAK_TFLOPS["f64"], 4)},
        "speedup_vs_fp64": round(main_res["gflops"] / fp64["gflops"], 3),
        "accuracy": {"backward_err": main_res["backward_err"], "refine_iters": main_res["refine_iters"],
                     "converged": main_res["converged"], "fwd_diff_vs_fp64": fwd},
    }
    if args.tree == "auto":
        line["autotune_ms_per_step"] = {"fp64": {"%s bs %d %s" % c: t for c, t in fp64["tune"]}}
        if args.upd != "f64":
            line["autotune_ms_per_step"][args.upd] = {"%s bs %d %s" % c: t for c, t in main_res["tune"]}
    # The other update precision at the same kappa, tuned the same way.
    if args.upd in ("f32", "bf16") and not args.no_extra:
        other = "bf16" if args.upd == "f32" else "f32"
        o = run(other, refine=True)
        ofwd = (torch.linalg.norm(o["X"] - fp64["X"]) / torch.linalg.norm(fp64["X"])).item()
        line[other] = {"gflops": round(o["gflops"], 2), "ms_per_step": round(o["ms_per_step"], 3),
                       "exec_ms": round(o["exec_ms"], 3), "tree": "%s bs %d %s" % o["choice"],
                       "speedup_vs_fp64": round(o["gflops"] / fp64["gflops"], 3),
                       "frac_blended_peak": round(F / (o["exec_ms"] / 1e3) / 1e12 / peak_for(other, o["choice"]), 4),
                       "backward_err": o["backward_err"], "refine_iters": o["refine_iters"],
                       "converged": o["converged"], "fwd_diff_vs_fp64": ofwd,
                       "autotune_ms_per_step": {"%s bs %d %s" % c: t for c, t in o["tune"]}}
        # Harder conditioning of the square workload: each precision with its
        # tree from the tuning above, FP64 beside it.
        if args.workload == "square" and args.matrix == "conditioned":
            sweep = {}
            choices = {"f64": fp64["choice"], args.upd: main_res["choice"], other: o["choice"]}
            del A, B
            for kappa in (1e6, 1e10):
                Ak = square_matrix(kappa)
                Bk = rhs(Ak)
                ref = measure("f64", False, choices["f64"], Ak, Bk, 2, 1)
                cell = {"fp64": {"ms_per_step": round(ref["ms_per_step"], 3), "backward_err": ref["backward_err"]}}
                for u in ("f32", "bf16"):
                    r = measure(u, True, choices[u], Ak, Bk, 2, 1)
                    cell[u] = {"ms_per_step": round(r["ms_per_step"], 3), "exec_ms": round(r["exec_ms"], 3),
                               "speedup_vs_fp64": round(ref["ms_per_step"] / r["ms_per_step"], 3),
                               "backward_err": r["backward_err"], "refine_iters": r["refine_iters"],
                               "converged": r["converged"],
                               "fwd_diff_vs_fp64": (torch.linalg.norm(r["X"] - ref["X"]) /
                                                    torch.linalg.norm(ref["X"])).item()}
                sweep["%g" % kappa] = cell
                del Ak, Bk
                torch.cuda.empty_cache()
            line["kappa_sweep"] = sweep
            # The tall workload (16384 x 2048 N(0,1), same nb and right-hand
            # sides): Greedy with the TS-hybrid kernels, the fastest FP64 tree
            # of its tree sweep, for FP64 and the mixed path beside it.
            mt, nt = 16384, 2048
            At = tqr_inputs.gaussian_device(mt, nt, tqr_inputs.SEED_C2, dev).t()
            gt = torch.Generator(device=dev)
            gt.manual_seed(tqr_inputs.SEED_C3_RHS)
            Bt = (At @ torch.randn((nrhs, nt), generator=gt, dtype=torch.float64, device=dev).t()).t().contiguous().t()
            Ft = flops(mt, nt)
            tall = {"workload": "tall %dx%d N(0,1), nb %d, %d rhs, greedy ts" % (mt, nt, nb, nrhs)}
            for u in ("f64", args.upd):
                r = measure(u, u != "f64", ("greedy", 1, "ts"), At, Bt, args.steps, args.warmup)
                tall[u] = {"ms_per_step": round(r["ms_per_step"], 3), "exec_ms": round(r["exec_ms"], 3),
                           "gflops": round(Ft / (r["ms_per_step"] / 1e3) / 1e9, 2),
                           "backward_err": r["backward_err"], "refine_iters": r["refine_iters"],
                           "converged": r["converged"]}
            tall["speedup_vs_fp64"] = round(tall["f64"]["ms_per_step"] / tall[args.upd]["ms_per_step"], 3)
            line["tall"] = tall
            del At, Bt
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(nb, TREES[tname], bs, KERNS[kname], args.kappa)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
