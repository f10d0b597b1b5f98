#!/usr/bin/env python3
"""Throughput of the partition-method factor-and-solve on one MI355X.

Workload: the block tridiagonal system of the trapezoidal discretization of
y' = M(t) y + q(t) on [0,1], N = 65536 steps, block size m = 8, separated
boundary conditions (4 components at each end), FP64: n = 524296 unknowns.
One step = one numeric factorization (pf_refactor, in the handle's memory)
plus one solve (pf_solve), i.e. every phase of the method: per-partition
elimination, the recursive reduced solve and the back substitution.

Prints one JSON line: unknowns solved per second (whole job, inputs resident
in HBM), the roofline fraction of the dominant kernel (the finest-level
factor kernel, timed with HIP events on its stream), and the CPU oracle's
rate on the same system.
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


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--m", type=int, default=8)
    ap.add_argument("--partitions", type=int, default=0, help="finest-level p (0 = planner)")
    ap.add_argument("--block-rows", type=int, default=0)
    ap.add_argument("--coarse-rows", type=int, default=0)
    ap.add_argument("--split", action="store_true",
                    help="time pf_refactor + pf_solve instead of the fused pf_factor_solve")
    ap.add_argument("--map", choices=["auto", "rows"], default="auto",
                    help="factor lane mapping: planner default (segments), or rows on every level")
    ap.add_argument("--lane-entries", type=int, default=0,
                    help="segment mapping at level 0: block entries per lane (0 = planner)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM counters)")
    return ap.parse_args()


def kernel_bytes(kind, phase, level_nb, m, nrhs, f32=False):
    """Algorithmic bytes one launch moves: the blocks it must read and the
    factors / vectors it must write (8-byte words; 4 for FP32 factors)."""
    w = 4 if f32 else 8
    mm = m * m
    if phase == "factor+forward":   # the factor's blocks plus f read and t written
        return kernel_bytes(kind, "factor", level_nb, m, nrhs, f32) + level_nb * 2 * m * 8 * nrhs
    if kind == 0:  # block tridiagonal
        if phase == "factor":   # read D, Lo, Up; write E, R, Z, X
            return level_nb * (3 * mm * 8 + 4 * mm * w)
        if phase == "forward":  # read Lo, E, R, f; write t
            return level_nb * (mm * 8 + 2 * mm * w + 2 * m * 8 * nrhs)
        return level_nb * (2 * mm * w + 2 * m * 8 * nrhs)   # read Z, X, t; write x
    if phase == "factor":       # read D, Lo; write E, Z
        return level_nb * (2 * mm * 8 + 2 * mm * w)
    if phase == "forward":      # read Lo, E, f; write t
        return level_nb * (mm * 8 + mm * w + 2 * m * 8 * nrhs)
    return level_nb * (mm * w + 2 * m * 8 * nrhs)           # read Z, t; write x


KERNEL_SOURCES = ("kernels_common.h", "kernels_seg.hip", "kernels_rows.hip", "kernels_solve.hip")


def source_hash():
    """Hash of the kernel sources the recorded counters belong to."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0912_3678_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name):
    """HBM traffic measured by rocprofv3 counters for the current kernel
    source, if recorded (profiles/traffic.json), else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("kernels", {}).get(kernel_name)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the method's multi-GPU "
              "sharding is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0912_3678_amd import pf
    from paper_0912_3678_amd import workloads as wl

    dev = torch.device("cuda", 0)
    s = wl.trapezoid_bvp_btri(N=args.N, m=args.m)
    m, nb = s.m, s.nb
    n = m * nb
    D = wl.to_device_blocks(s.D, dev)
    Lo = wl.to_device_blocks(s.Lo, dev)
    Up = wl.to_device_blocks(s.Up, dev)
    f = wl.to_device_rhs(s.f, dev)
    x = torch.empty_like(f)
    A = pf.make_matrix(pf.PF_BTRI, m, nb, D, Lo, Up)
    flags = {"auto": 0, "rows": pf.PF_FLAG_MAP_ROWS}[args.map]
    opts = pf.make_opts(partitions=args.partitions, block_rows=args.block_rows,
                        coarse_rows=args.coarse_rows, flags=flags, lane_entries=args.lane_entries)
    F = pf.pf_factor(A, opts)
    levels = pf.pf_factor_levels(F)
    torch.cuda.synchronize()

    def step_fused():
        pf.pf_factor_solve(F, f, x, want_info=False)

    def step_split():
        pf.pf_refactor(F)
        pf.pf_solve(F, f, x, want_info=False)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            step()
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall * 1e3 / args.steps, np.array([a.elapsed_time(b) for a, b in evs])

    split_ms, _ = timed(step_split)
    step = step_split if args.split else step_fused
    ms_per_step, per = timed(step)

    # acceptance of the result: FP64 residual with torch block products
    # (independent of the library's kernels)
    X = x[0].view(nb, m, 1)
    At = lambda B: B.transpose(1, 2).contiguous()             # column-major -> math blocks
    r = torch.bmm(At(D), X)
    r[1:] += torch.bmm(At(Lo), X[:-1])
    r[:-1] += torch.bmm(At(Up), X[1:])
    r = f[0].view(nb, m, 1) - r
    rowsum = At(D).abs().sum(2)
    rowsum[1:] += At(Lo).abs().sum(2)
    rowsum[:-1] += At(Up).abs().sum(2)
    eta = float(r.abs().max() / (rowsum.max() * x.abs().max() + f.abs().max()))
    status = pf.pf_sync_status(F).status

    # per-kernel durations (HIP events around each launch on its stream)
    pf.pf_profile_enable(F, True)
    acc = {}
    for _ in range(args.profile_steps):
        step()
        for ph, lvl, ms in pf.pf_profile_read(F):
            acc.setdefault((ph, lvl), []).append(ms)
    pf.pf_profile_enable(F, False)
    kernels = []
    total_alg = 0
    for (ph, lvl), v in sorted(acc.items(), key=lambda kv: (kv[0][1], kv[0][0])):
        kind, lnb, lp = levels[lvl]
        b = kernel_bytes(kind, ph, lnb, m, 1)
        total_alg += b
        avg = float(np.mean(v))
        kernels.append({"phase": ph, "level": lvl, "nb": lnb, "p": lp, "avg_us": round(avg * 1e3, 2),
                        "alg_MB": round(b / 1e6, 3), "GBps": round(b / (avg * 1e-3) / 1e9, 1)})
    dom = max(kernels, key=lambda k: k["avg_us"])
    M = 1 << (m - 1).bit_length()
    E = 0 if args.map == "rows" else (args.lane_entries or {8: 2, 16: 4, 32: 0}.get(M, 1))
    names = {"factor": (f"k_btri_seg<{M}, {E}, double, false, false>" if E else
                        f"k_btri_factor<{M}, double, false>"),
             "factor+forward": f"k_btri_seg<{M}, {E}, double, false, true>",
             "forward": f"k_fwd<0, {M}, 1, double, false>", "backward": f"k_bwd<0, {M}, 1, double>"}
    dom_name = names[dom["phase"]] if dom["level"] == 0 else f"{dom['phase']} level {dom['level']}"
    dom_bytes = dom["alg_MB"] * 1e6
    achieved = dom_bytes / (dom["avg_us"] * 1e-6) / 1e9
    traffic = load_traffic(dom_name)

    value = n / (ms_per_step * 1e-3)
    out = {
        "metric": "unknowns solved/sec (N*m) at residual<=1e-12",
        "value": value if (eta <= 1e-12 and status == 0) else 0.0,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "trapezoid_bvp_btri", "N": args.N, "m": m, "nb": nb,
                   "unknowns": n, "nrhs": 1,
                   "partitions": args.partitions or "planner",
                   "lane_mapping": "rows" if args.map == "rows" else f"segments of {E}",
                   "levels": [[k, a, b] for k, a, b in levels],
                   "step": "pf_refactor + pf_solve" if args.split else
                           "pf_factor_solve (refactor + solve, forward sweep fused per level)"},
        "eta": eta,
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                       "mean_events": float(per.mean())},
        "split_ms_per_step": split_ms,
        "step_alg_GBps": round(total_alg / (per.mean() * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": dom_name, "level": dom["level"],
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "alg_bytes_per_launch": int(dom_bytes),
                     "avg_launch_us": dom["avg_us"],
                     "traffic": traffic},
        "kernels": kernels,
    }

    pf.pf_destroy(F)

    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = src.numel() * 8

    if not args.no_cpu_baseline:
        import oracle
        times = []
        t_end = time.perf_counter() + args.cpu_seconds
        while time.perf_counter() < t_end or not times:
            t1 = time.perf_counter()
            xo = oracle.btri_solve(s.D, s.Lo, s.Up, s.f)
            times.append(time.perf_counter() - t1)
        med = float(np.median(times))
        xg = x[0].cpu().numpy()
        out["cpu_baseline"] = {"value": n / med, "unit": "unknowns/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the full system (n={n}), band LU with partial pivoting "
                                         f"(kl=ku={2 * m - 1}), median of {len(times)} solves",
                               "gpu_vs_oracle_rel_err": float(np.abs(xg - xo).max() / np.abs(xo).max())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
