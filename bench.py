#!/usr/bin/env python3
"""Throughput of the partition-method factor-and-solve on one MI355X.

Default workload (--workload batch): 512 independent block tridiagonal
systems drawn by the batched workload's law -- block size m uniform on
{4, 8, 16, 32}, N log-uniform in [2^8, 2^16], diagonal blocks 4I + N(0,1/m),
off-diagonal blocks N(0,1/m), 1..64 right-hand sides each -- factored and
solved as one batch (grouped launches replayed from a HIP graph), in FP64
(the line's value) and with FP32 factors + FP64 refinement (beside it).
One step = one pf_batch_run: every phase of the method for every system.
Prints one JSON line: unknowns x right-hand sides solved per second (whole
job, inputs resident in HBM, only if every result meets eta <= 1e-12), the
roofline of the dominant grouped launch (timed by events its dispatch
stamps on its stream) and of the whole step, the CPU oracle on a bounded
sample of the same law (one core and all cores), and p50 / p99 latency of
the serving law under load (Poisson arrivals at 0.8 x saturation).

Other workloads (one JSON line each, same fields where they apply):
  bvp      the block tridiagonal system of the trapezoidal discretization of
           y' = M(t) y + q(t) on [0,1], N = 65536 steps, m = 8, separated
           boundary conditions, FP64; one step = pf_factor_solve
           (--partitions 256 for the literal top-level p; cold-cache timing
           beside the warm one);
  babd     BABD from the trapezoid rule with non-separated boundary
           conditions, m = 16, N = 262144 steps, FP32 factors + FP64
           refinement to eta <= 1e-12 (--prec fp64 for plain FP64);
  serving  Poisson arrivals of factor-and-solve requests (m in {8,16,32},
           N lognormal with median 2^14 clamped to 2^20, 30 % repeat
           right-hand sides on kept factors) through the request scheduler:
           p50 / p99 latency and throughput at fractions of the saturation
           rate;
  ivp      the trapezoid rule for an initial value problem, solved in
           parallel over sub-intervals (Sec. 3);
  tridiag  a scalar tridiagonal system (m = 1; sub/super diagonals
           U[-1,1], diagonal 4+U[0,1]) of --n-tri unknowns, FP64, timed
           like bvp.
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
    ap.add_argument("--workload", choices=["batch", "bvp", "babd", "serving", "ivp", "tridiag"],
                    default="batch")
    ap.add_argument("--prec", choices=["fp64", "fp32ir"], default=None,
                    help="babd: precision (default fp32ir); batch: run only this precision "
                         "(default: both, FP64 is the line's value)")
    ap.add_argument("--ir-steps", type=int, default=3,
                    help="batch: timed steps of the FP32 + refinement run")
    ap.add_argument("--no-serving", action="store_true",
                    help="batch: skip the serving-latency leg")
    ap.add_argument("--serve-count", type=int, default=160,
                    help="batch: requests of the serving-latency leg")
    ap.add_argument("--count", type=int, default=0,
                    help="batch: systems (default 512); serving: requests (default 240)")
    ap.add_argument("--n-hi", type=int, default=0,
                    help="batch / serving: largest block count (default 2^16 / 2^20)")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serving: memory budget")
    ap.add_argument("--autotune", action="store_true",
                    help="batch: the autotuner's launch shapes (PF_FLAG_AUTOTUNE, tuned per "
                         "shape class at batch creation) instead of the batch planner's")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (batch 20, others 50)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (batch 2, others 5)")
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--m", type=int, default=8)
    ap.add_argument("--n-tri", type=int, default=1 << 24, help="tridiag: unknowns")
    ap.add_argument("--partitions", type=int, default=0, help="finest-level p (0 = planner)")
    ap.add_argument("--block-rows", type=int, default=0)
    ap.add_argument("--coarse-rows", type=int, default=0)
    ap.add_argument("--split", action="store_true",
                    help="time pf_refactor + pf_solve instead of the fused pf_factor_solve")
    ap.add_argument("--map", choices=["auto", "segments", "rows"], default="auto",
                    help="factor lane mapping: planner default (matrix cores at the finest "
                         "level for m = 8, segments elsewhere), segments only, or rows")
    ap.add_argument("--lane-entries", type=int, default=0,
                    help="segment mapping at level 0: block entries per lane (0 = planner)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="fold two rocprofv3 --pmc csv outputs into profiles/traffic.json (host only)")
    ap.add_argument("--traffic-note", default="", help="--record-traffic: the workload and commands")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM counters)")
    return ap.parse_args()


def kernel_bytes(kind, phase, level_nb, m, nrhs, f32=False, split=False, whole=False):
    """Algorithmic bytes of one launch by the method's per-unit figures
    (8-byte words; 4 for FP32 factors): one read of the input blocks, the
    right-hand-side read and the solution write.  The factors' stores and
    their re-reads count only when factor and solve are separate calls
    (split: pf_refactor, then pf_solve); inside one factor-and-solve call
    they are the method's intermediate state.  whole: one launch does the
    level's factor, forward sweep and back substitution."""
    w = 4 if f32 else 8
    mm = m * m
    nblk = 3 if kind == 0 else 2            # D, Lo, Up (block tridiagonal) or D, Lo
    nfac = 4 if kind == 0 else 2            # E, R, Z, X or E, Z
    rhs = level_nb * m * 8 * nrhs
    if whole:
        return level_nb * nblk * mm * 8 + 2 * rhs
    if phase == "factor+forward":           # A read, f read (t is intermediate)
        return level_nb * nblk * mm * 8 + rhs
    if phase == "factor":
        return level_nb * (nblk * mm * 8 + (nfac * mm * w if split else 0))
    if phase == "forward":                  # f read (+ Lo, E, R when split)
        return rhs + (level_nb * (mm * 8 + (nfac // 2) * mm * w) if split else 0)
    return rhs + (level_nb * (nfac // 2) * mm * w if split else 0)   # x write (+ Z, X)


# Sources each profiled kernel is built from: its recorded counters stay valid
# while these files are unchanged.
_COMMON = ("pf_internal.h", "kernels_common.h")
KERNEL_SOURCES = {
    "k_btri_mfma": _COMMON + ("kernels_gj.h", "kernels_mfma.hip"),
    "k_btri_seg": _COMMON + ("kernels_gj.h", "kernels_seg.h", "kernels_seg.hip"),
    "k_babd_seg": _COMMON + ("kernels_gj.h", "kernels_seg.h", "kernels_seg.hip"),
    "k_fwd": _COMMON + ("kernels_solve.h", "kernels_solve.hip"),
    "k_bwd": _COMMON + ("kernels_solve.h", "kernels_solve.hip"),
    "k_btri_factor": _COMMON + ("kernels_rows.hip",),
    "k_babd_factor": _COMMON + ("kernels_rows.hip",),
    "k_tri_factor": _COMMON + ("kernels_tri.h", "kernels_tri.hip"),
    "k_tri_bwd": _COMMON + ("kernels_tri.h", "kernels_tri.hip"),
    "k_tri_fwd": _COMMON + ("kernels_tri.h", "kernels_tri.hip"),
    "kb_btri_mfma32": _COMMON + ("kernels_gj.h", "kernels_mfma_tiles.h", "kernels_mfma_tiles.hip"),
    "kb_btri_mfma16": _COMMON + ("kernels_gj.h", "kernels_mfma_tiles.h", "kernels_mfma_tiles.hip"),
    "kb_fwdt": _COMMON + ("kernels_gj.h", "kernels_mfma_tiles.h", "kernels_mfma_tiles.hip"),
    "kb_bwdt": _COMMON + ("kernels_gj.h", "kernels_mfma_tiles.h", "kernels_mfma_tiles.hip"),
}
_ALL_SOURCES = _COMMON + ("kernels_gj.h", "kernels_seg.h", "kernels_seg.hip", "kernels_mfma.hip",
                          "kernels_mfma_tiles.h", "kernels_mfma_tiles.hip", "kernels_mfma_tiles32.hip", "kernels_rows.hip", "kernels_solve.h",
                          "kernels_solve.hip", "kernels_tri.h", "kernels_tri.hip")


def source_hash(kernel_name):
    """Hash of the sources the named kernel is built from."""
    files = KERNEL_SOURCES.get(kernel_name.split("<")[0], _ALL_SOURCES)
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_0912_3678_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name, grid=None):
    """HBM traffic measured by rocprofv3 counters for the kernel's current
    sources (and, when given, the same grid in threads), if recorded
    (profiles/traffic.json), else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(kernel_name)
    if not ent or ent.get("source_hash") != source_hash(kernel_name):
        return None
    if grid is not None and ent.get("grid") != grid:
        return None
    return ent


def record_traffic(fetch_dir, write_dir, note):
    """Fold two rocprofv3 counter runs (--pmc FETCH_SIZE, --pmc WRITE_SIZE,
    csv output, each of a bench.py run with --copy-probe) into
    profiles/traffic.json: per library kernel, the HBM bytes of its largest
    dispatch (the finest level), each counter scaled by what it reads for
    the 256 MiB copy of the probe, keyed with the hash of the kernel's
    sources.  Runs on the host; no device is touched."""
    import csv
    import re

    def load(d, counter):
        path = os.path.join(d, "run_counter_collection.csv")
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows
                  if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 131072]
        if not copies:
            raise SystemExit(f"{path}: no 256 MiB copy-probe dispatch")
        scale = 262144.0 / sorted(copies)[len(copies) // 2]   # KiB the copy moved / KiB read
        best = {}
        for r in rows:
            m = re.search(r"pf::\(anonymous namespace\)::([^(]+)\(", r["Kernel_Name"])
            if not m:
                continue
            name, grid = m.group(1), int(r["Grid_Size"])
            if name not in best or grid > best[name][0]:
                best[name] = (grid, float(r["Counter_Value"]) * 1024 * scale)
        return best, scale

    fetch, sf = load(fetch_dir, "FETCH_SIZE")
    write, sw = load(write_dir, "WRITE_SIZE")
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        rec = {"kernels": {}}
    rec.setdefault("runs", []).append({"note": note, "fetch_scale": round(sf, 4),
                                       "write_scale": round(sw, 4)})
    for name, (grid, fb) in fetch.items():
        if name not in write:
            continue
        wb = write[name][1]
        rec["kernels"][name] = {"grid": grid, "fetch_bytes": int(fb), "write_bytes": int(wb),
                                "total_bytes": int(fb + wb), "source_hash": source_hash(name),
                                "run": note}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"recorded {len(fetch)} kernels into {path} (FETCH x {sf:.3f}, WRITE x {sw:.3f})")


def main():
    args = parse()
    if args.record_traffic:
        record_traffic(args.record_traffic[0], args.record_traffic[1], args.traffic_note)
        return
    if args.steps is None:
        args.steps = 20 if args.workload == "batch" else 50
    if args.warmup is None:
        args.warmup = 2 if args.workload == "batch" else 5
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the method's multi-GPU "
              "sharding is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)
    run = {"bvp": run_bvp, "babd": run_babd, "batch": run_batch, "serving": run_serving,
           "ivp": run_ivp, "tridiag": run_bvp}
    out = run[args.workload](args)
    if args.copy_probe:
        # a plain 256 MiB device copy: what the HBM counters read for known bytes
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = src.numel() * 8
    print(json.dumps(out), flush=True)


def run_bvp(args):
    import numpy as np
    import torch

    from paper_0912_3678_amd import pf
    from paper_0912_3678_amd import workloads as wl

    dev = torch.device("cuda", 0)
    tri = args.workload == "tridiag"
    s = wl.scalar_tridiagonal(n=args.n_tri) if tri else wl.trapezoid_bvp_btri(N=args.N, m=args.m)
    m, nb = s.m, s.nb
    n = m * nb
    D = wl.to_device_blocks(s.D, dev)
    Lo = wl.to_device_blocks(s.Lo, dev)
    Up = wl.to_device_blocks(s.Up, dev)
    f = wl.to_device_rhs(s.f, dev)
    x = torch.empty_like(f)
    A = pf.make_matrix(pf.PF_BTRI, m, nb, D, Lo, Up)
    flags = {"auto": 0, "segments": pf.PF_FLAG_MAP_SEGMENTS, "rows": pf.PF_FLAG_MAP_ROWS}[args.map]
    opts = pf.make_opts(partitions=args.partitions, block_rows=args.block_rows,
                        coarse_rows=args.coarse_rows, flags=flags, lane_entries=args.lane_entries)
    F = pf.pf_factor(A, opts)
    levels = pf.pf_factor_levels(F)
    torch.cuda.synchronize()
    # small scalar systems: pf_factor_solve is one launch of local cyclic reduction
    cr = (tri and args.map == "auto" and not args.split and nb <= 4096 and levels[0][2] <= 64)

    def step_fused():
        pf.pf_factor_solve(F, f, x, want_info=False)

    def step_split():
        pf.pf_refactor(F)
        pf.pf_solve(F, f, x, want_info=False)

    def timed(step):
        # throughput: K steps back to back between two synchronizations;
        # then the same K steps again, each between its own two events, for
        # the per-step latencies (the event commands would otherwise sit
        # between the steps of the timed run)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for a, b in evs:
            a.record()
            step()
            b.record()
        torch.cuda.synchronize()
        return wall * 1e3 / args.steps, np.array([a.elapsed_time(b) for a, b in evs])

    split_ms, _ = timed(step_split)
    step = step_split if args.split else step_fused
    ms_per_step, per = timed(step)

    # cold steps: the 256 MB last-level cache (MALL) is flushed before each
    # by writing a 1 GiB buffer; each step timed alone with events
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    cold = []
    for _ in range(max(3, min(args.steps, 20))):
        flush.fill_(1.0)
        a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_ev.record()
        step()
        b_ev.record()
        torch.cuda.synchronize()
        cold.append(a_ev.elapsed_time(b_ev))
    del flush

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
        whole = tri and cr and lvl == 0 and ph == "factor+forward"
        b = kernel_bytes(kind, ph, lnb, m, 1, split=args.split, whole=whole)
        total_alg += b
        avg = float(np.mean(v))
        kernels.append({"phase": ph, "level": lvl, "nb": lnb, "p": lp, "avg_us": round(avg * 1e3, 2),
                        "alg_MB": round(b / 1e6, 3), "GBps": round(b / (avg * 1e-3) / 1e9, 1)})
    dom = max(kernels, key=lambda k: k["avg_us"])
    M = 1 << (m - 1).bit_length()
    E = 0 if args.map == "rows" else (args.lane_entries or {8: 2, 16: 4, 32: 0}.get(M, 1))
    mfma = args.map == "auto" and not args.lane_entries and M == 8
    # m = 1: rows staged through LDS (chains of up to 5, 9, 13 or 17 blocks)
    # (longer chains run on the segment kernel with one entry per lane)
    nint0 = levels[0][1] - (levels[0][2] - 1)
    km = next(k for k in (5, 9, 13, 17, 10 ** 9) if -(-nint0 // levels[0][2]) <= k)
    trik = args.map == "auto" and M == 1 and km <= 17
    names = {"factor": ("k_btri_mfma<false>" if mfma else
                        f"k_tri_factor<{km}, false, false>" if trik else
                        f"k_btri_seg<{M}, {E}, double, false, false>" if E else
                        f"k_btri_factor<{M}, double, false>"),
             "factor+forward": ("k_btri_mfma<true>" if mfma else
                                f"k_tri_factor<{km}, false, true>" if trik else
                                f"k_btri_seg<{M}, {E}, double, false, true>"),
             "forward": f"k_tri_fwd<{km}, false>" if trik else f"k_fwd<0, {M}, 1, double, false>",
             "backward": f"k_tri_bwd<{km}>" if trik else f"k_bwd<0, {M}, 1, double>"}
    if cr:
        names["factor+forward"] = "k_tri_cr_whole"
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
        "config": {"workload": "scalar_tridiagonal" if tri else "trapezoid_bvp_btri",
                   "N": nb if tri else args.N, "m": m, "nb": nb,
                   "unknowns": n, "nrhs": 1,
                   "partitions": args.partitions or "planner",
                   "lane_mapping": ("rows" if args.map == "rows" else
                                    "matrix cores at level 0, segments above" if mfma else
                                    "one partition per lane, rows staged through LDS" if trik else
                                    f"segments of {E}"),
                   "levels": [[k, a, b] for k, a, b in levels],
                   "step": "pf_refactor + pf_solve" if args.split else
                           "pf_factor_solve (refactor + solve, forward sweep fused per level)"},
        "eta": eta,
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                       "mean_events": float(per.mean())},
        "split_ms_per_step": split_ms,
        "cold_ms_per_step": float(np.median(cold)),
        "warm_ms_per_step_events": float(np.median(per)),
        "step_alg_GBps": round(total_alg / (per.mean() * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": dom_name, "level": dom["level"],
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "alg_bytes_per_launch": int(dom_bytes),
                     "avg_launch_us": dom["avg_us"],
                     "traffic": traffic["total_bytes"] if traffic else None,
                     "traffic_split": ({"fetch_bytes": traffic["fetch_bytes"],
                                        "write_bytes": traffic["write_bytes"]} if traffic else None)},
        "kernels": kernels,
    }

    pf.pf_destroy(F)


    if not args.no_cpu_baseline:
        import oracle
        times = []
        t_end = time.perf_counter() + args.cpu_seconds
        while time.perf_counter() < t_end or not times:
            t1 = time.perf_counter()
            if tri:
                xo = oracle.thomas(s.Lo.ravel(), s.D.ravel(), s.Up.ravel(), s.f)
            else:
                xo = oracle.btri_solve(s.D, s.Lo, s.Up, s.f)
            times.append(time.perf_counter() - t1)
        med = float(np.median(times))
        xg = x[0].cpu().numpy()
        how = ("Thomas elimination" if tri else
               f"band LU with partial pivoting (kl=ku={2 * m - 1})")
        out["cpu_baseline"] = {"value": n / med, "unit": "unknowns/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the full system (n={n}), {how}, "
                                         f"median of {len(times)} solves",
                               "gpu_vs_oracle_rel_err": float(np.abs(xg - xo).max() / np.abs(xo).max())}
    return out


def _eta_btri_torch(D, Lo, Up, f, x, m, nb):
    """FP64 normwise backward error of x (columns of shape (k, n)) for a block
    tridiagonal system with column-major device blocks, with torch products
    (independent of the library's kernels)."""
    import torch
    k = x.shape[0]
    At = lambda B: B.transpose(1, 2).contiguous()
    X = x.view(k, nb, m).permute(1, 2, 0).contiguous()            # (nb, m, k)
    r = torch.bmm(At(D), X)
    r[1:] += torch.bmm(At(Lo), X[:-1].contiguous())
    r[:-1] += torch.bmm(At(Up), X[1:].contiguous())
    r = f.view(k, nb, m).permute(1, 2, 0) - r
    rowsum = At(D).abs().sum(2)
    rowsum[1:] += At(Lo).abs().sum(2)
    rowsum[:-1] += At(Up).abs().sum(2)
    na = rowsum.max()
    rn = r.abs().amax(dim=(0, 1))
    xn = x.abs().amax(dim=1)
    fn = f.abs().amax(dim=1)
    return float((rn / (na * xn + fn)).max())


def _eta_babd_torch(D, Lo, C, f, x, m, nb):
    import torch
    At = lambda B: B.transpose(1, 2).contiguous()
    X = x[0].view(nb, m, 1)
    r = torch.bmm(At(D), X)
    r[1:] += torch.bmm(At(Lo), X[:-1].contiguous())
    r[0] += At(C)[0] @ X[-1]
    r = f[0].view(nb, m, 1) - r
    rowsum = At(D).abs().sum(2)
    rowsum[1:] += At(Lo).abs().sum(2)
    rowsum[0] += At(C)[0].abs().sum(1)
    return float(r.abs().max() / (rowsum.max() * x.abs().max() + f.abs().max()))


def _profile_dominant(pf, F, step, levels, m, f32, steps):
    """Per-launch event timings over a few steps; the dominant launch and
    its algorithmic bandwidth."""
    import numpy as np
    pf.pf_profile_enable(F, True)
    acc = {}
    for _ in range(steps):
        step()
        for ph, lvl, ms in pf.pf_profile_read(F):
            acc.setdefault((ph, lvl), []).append(ms)
    pf.pf_profile_enable(F, False)
    kernels = []
    for (ph, lvl), v in sorted(acc.items(), key=lambda kv: (kv[0][1], kv[0][0])):
        kind, lnb, lp = levels[lvl]
        b = kernel_bytes(kind, ph, lnb, m, 1, f32 and lvl == 0)
        avg = float(np.mean(v))
        kernels.append({"phase": ph, "level": lvl, "nb": lnb, "p": lp, "avg_us": round(avg * 1e3, 2),
                        "alg_MB": round(b / 1e6, 3), "GBps": round(b / (avg * 1e-3) / 1e9, 1)})
    return kernels, max(kernels, key=lambda k: k["avg_us"])


def run_ivp(args):
    """Time-parallel linear IVP (Sec. 3): y' = L y + g(t) on [0, 1], m = 8,
    N = 65536 trapezoid steps over a coarse mesh of p = 4096 sub-intervals of
    16 steps.  One step = one pf_ivp_run on a plan made once (build the
    eq. (My) system on the device, factor and solve it with the sub-intervals
    as partitions; synchronized).  The one-shot pf_ivp_solve, which also
    allocates and frees, is timed beside it.  Checked against the oracle's
    sequential stepping of the same discretization."""
    import numpy as np
    import torch

    from paper_0912_3678_amd import pf
    from paper_0912_3678_amd import workloads as wl

    m, steps = args.m, args.N
    p = args.partitions or 4096
    if steps % p:
        raise SystemExit(f"--N {steps} is not a multiple of the {p} sub-intervals")
    Nsub = steps // p
    dev = torch.device("cuda", 0)
    L, g, y0, t0, T = wl.ivp_problem(m, p, Nsub, seed=wl.seed_for(6))
    Ld = torch.tensor(np.ascontiguousarray(L.T).reshape(-1), dtype=torch.float64, device=dev)
    gd = torch.tensor(g.reshape(-1), dtype=torch.float64, device=dev)
    y0d = torch.tensor(y0, dtype=torch.float64, device=dev)
    y = torch.empty(((steps + 1) * m,), dtype=torch.float64, device=dev)
    y2 = torch.empty_like(y)
    opts = pf.make_opts(block_rows=args.block_rows, coarse_rows=args.coarse_rows)
    plan = pf.pf_ivp_create(m, p, Nsub, opts)
    infos = []

    def step():
        infos.append(pf.pf_ivp_run(plan, Ld, t0, T, gd, y0d, y))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        step()
        per.append((time.perf_counter() - t1) * 1e3)
    wall = (time.perf_counter() - t_start) * 1e3 / args.steps
    pf.pf_ivp_destroy(plan)
    # the one-shot driver: create + run + destroy per call
    pf.pf_ivp_solve(m, Ld, t0, T, p, Nsub, gd, y0d, y2, opts=opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(max(1, args.steps // 4)):
        pf.pf_ivp_solve(m, Ld, t0, T, p, Nsub, gd, y0d, y2, opts=opts)
    oneshot_ms = (time.perf_counter() - t1) * 1e3 / max(1, args.steps // 4)
    same = bool(torch.equal(y, y2))
    import oracle
    h = (T - t0) / steps
    ref = oracle.ivp_trapezoid(L, h, g, y0)
    # CPU baseline: the oracle's structured LU with partial pivoting (C) on
    # the same eq. (My) system
    eye = np.eye(m)
    Dh = np.concatenate([eye[None], np.repeat((eye - 0.5 * h * L)[None], steps, 0)])
    Loh = np.repeat((-(eye + 0.5 * h * L))[None], steps, 0)
    fh = np.concatenate([y0[None], 0.5 * h * (g[:-1] + g[1:])]).reshape(-1)
    t1 = time.perf_counter()
    oracle.babd_solve(Dh, Loh, np.zeros((m, m)), fh)
    seq_s = time.perf_counter() - t1
    rel = float(np.abs(y.cpu().numpy().reshape(steps + 1, m) - ref).max() / np.abs(ref).max())
    n = (steps + 1) * m
    ok = rel <= 1e-11 and all(i.status == 0 for i in infos)
    out = {
        "metric": "unknowns solved/sec (time-parallel IVP, trapezoid rule)",
        "value": n / (wall * 1e-3) if ok else 0.0,
        "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ivp_trapezoid", "m": m, "steps": steps, "subintervals": p,
                   "steps_per_subinterval": Nsub, "unknowns": n,
                   "step": "pf_ivp_run on a plan (device build + factor-and-solve, synchronized)"},
        "rel_err_vs_sequential": rel,
        "one_shot_ms_per_call": oneshot_ms, "one_shot_same_result": same,
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = {"value": n / seq_s, "unit": "unknowns/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the full eq. (My) system ({steps + 1} blocks of "
                                         f"{m}): the oracle's structured LU with partial "
                                         f"pivoting (C), one solve"}
    return out


def run_babd(args):
    """BABD, m = 16, N = 262144 steps (nb = 262145), FP32 factors + FP64
    refinement (or FP64): one step = pf_factor_solve with the refinement."""
    import numpy as np
    import torch

    from paper_0912_3678_amd import pf
    from paper_0912_3678_amd import workloads as wl

    prec = args.prec or "fp32ir"
    N = args.N if args.N != 65536 else 262144
    m = args.m if args.m != 8 else 16
    dev = torch.device("cuda", 0)
    s = wl.trapezoid_babd(N=N, m=m)
    nb = s.nb
    n = nb * m
    D = wl.to_device_blocks(s.D, dev)
    Lo = wl.to_device_blocks(s.Lo, dev)
    C = wl.to_device_blocks(s.C[None], dev)
    f = wl.to_device_rhs(s.f, dev)
    x = torch.empty_like(f)
    A = pf.make_matrix(pf.PF_BABD, m, nb, D, Lo, None, C)
    opts = pf.make_opts(prec=pf.PF_FP32_IR if prec == "fp32ir" else pf.PF_FP64,
                        block_rows=args.block_rows, coarse_rows=args.coarse_rows,
                        lane_entries=args.lane_entries)
    F = pf.pf_factor(A, opts)
    levels = pf.pf_factor_levels(F)
    infos = []

    def step():
        infos.append(pf.pf_factor_solve(F, f, x))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        step()                        # synchronizes (refinement loop / info)
        per.append((time.perf_counter() - t1) * 1e3)
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    info = infos[-1]
    eta = _eta_babd_torch(D, Lo, C, f, x, m, nb)
    kernels, dom = _profile_dominant(pf, F, step, levels, m, prec == "fp32ir", 3)
    achieved = dom["alg_MB"] * 1e6 / (dom["avg_us"] * 1e-6) / 1e9
    out = {
        "metric": "unknowns solved/sec (N*m) at residual<=1e-12",
        "value": n / (wall * 1e-3) if (eta <= 1e-12 and info.status == 0) else 0.0,
        "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 factors + f64 refinement" if prec == "fp32ir" else "f64",
        "data": "synthetic",
        "config": {"workload": "trapezoid_babd", "N": N, "m": m, "nb": nb, "unknowns": n,
                   "nrhs": 1, "levels": [[k, a, b] for k, a, b in levels],
                   "step": "pf_factor_solve" + (" with FP64 refinement" if prec == "fp32ir" else "")},
        "eta": eta, "refine_iters": info.refine_iters,
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "roofline": {"bound": "hbm", "kernel": f"{dom['phase']} level {dom['level']}",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "alg_bytes_per_launch": int(dom["alg_MB"] * 1e6),
                     "avg_launch_us": dom["avg_us"], "traffic": None},
        "kernels": kernels,
    }
    pf.pf_destroy(F)
    if not args.no_cpu_baseline:
        import oracle
        sub = wl.trapezoid_babd(N=min(N, 32768), m=m)
        times = []
        t_end = time.perf_counter() + args.cpu_seconds
        while time.perf_counter() < t_end or not times:
            t1 = time.perf_counter()
            oracle.babd_solve(sub.D, sub.Lo, sub.C, sub.f)
            times.append(time.perf_counter() - t1)
        out["cpu_baseline"] = {"value": sub.nb * m / float(np.median(times)), "unit": "unknowns/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"the same BABD law at N={sub.nb - 1} (structured BABD LU with "
                                         f"partial pivoting), median of {len(times)} solves"}
    return out


def _device_btri(m, nb, k, seed, dev):
    """A random block tridiagonal system of the batched workload's law,
    generated on the device (diagonal 4I + N(0,1/m), off-diagonal N(0,1/m),
    right-hand sides N(0,1)); blocks column-major."""
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    sc = 1.0 / (m ** 0.5)
    D = torch.randn((nb, m, m), generator=g, device=dev, dtype=torch.float64) * sc
    D += 4.0 * torch.eye(m, device=dev, dtype=torch.float64)
    Lo = torch.randn((nb - 1, m, m), generator=g, device=dev, dtype=torch.float64) * sc
    Up = torch.randn((nb - 1, m, m), generator=g, device=dev, dtype=torch.float64) * sc
    f = torch.randn((k, nb * m), generator=g, device=dev, dtype=torch.float64)
    return D, Lo, Up, f


FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32
RIDGE_FP64 = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)   # flop per byte


def cpu_model():
    """The host CPU's model name and the cores this process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return name, cores


def batch_kernel_name(L):
    """The kernel a grouped batch launch runs (pf_launch_info as a dict)."""
    M, f32, lvl = L["m"], L["f32"], L["level"]
    V = "float" if f32 else "double"
    add = "true" if (lvl > 0 and L["kind"] == 0) else "false"
    if L["phase"] == 0:
        mp = L["mapping"]
        if mp == -1:
            return "kb_btri_mfma"
        if mp == -2:
            return f"kb_btri_mfma32<{add}, {V}>"
        if mp == -3:
            return f"kb_babd_mfma16<{V}>"
        if mp == -4:
            return f"kb_btri_mfma16<{add}, {V}>"
        if mp > 0:
            return f"kb_{'btri' if L['kind'] == 0 else 'babd'}_seg<{M}, {mp}, {V}, {add}>"
        return f"kb_{'btri' if L['kind'] == 0 else 'babd'}_factor<{M}, {V}, {add}>"
    tiled = M in (16, 32)
    fwd = L["phase"] == 1
    if tiled:
        return (f"kb_fwdt<{M}, {L['kind']}, *, {add}, {V}>" if fwd
                else f"kb_bwdt<{M}, {L['kind']}, *, {V}>")
    return f"kb_fwd<{L['kind']}, {M}, *, {V}, {add}>" if fwd else f"kb_bwd<{L['kind']}, {M}, *, {V}>"


def batch_launch_roofline(L, m_true):
    """Algorithmic work of a grouped launch by the per-unit figures of the
    method (8-byte words), and the roofline that bounds it.
    Factor: the partition elimination reads the input blocks D, Lo, Up once
    (3 m^2 words per block row) and does 12.7 m^3 flops per block row (the
    partition method's count for block tridiagonal matrices).  Forward
    sweep: reads the right-hand sides (m words per block row and column),
    6 m^2 flops per block row and column (t, the next f', the separator
    row).  Back substitution: writes the solution (m words per block row and
    column), 4 m^2 flops per block row and column.  Factor stores and their
    re-reads are not algorithmic here: the batch step factors and solves in
    one call.  Returns (bytes, flops, bound)."""
    m = m_true
    if L["phase"] == 0:
        byt = 3 * m * m * 8 * L["rows"]
        fl = 12.7 * m ** 3 * L["rows"]
    elif L["phase"] == 1:
        byt = m * 8 * L["rhs_rows"]
        fl = 6 * m * m * L["rhs_rows"]
    else:
        byt = m * 8 * L["rhs_rows"]
        fl = 4 * m * m * L["rhs_rows"]
    bound = "mfma" if fl / max(byt, 1) > RIDGE_FP64 else "hbm"
    return byt, fl, bound


def _batch_device_systems(specs, dev):
    import torch
    from paper_0912_3678_amd import pf
    mats, keep, fs, xs = [], [], [], []
    unknowns = 0
    for (m, nb, k, seed) in specs:
        D, Lo, Up, f = _device_btri(m, nb, k, seed, dev)
        keep.append((D, Lo, Up))
        mats.append(pf.make_matrix(pf.PF_BTRI, m, nb, D, Lo, Up))
        fs.append(f)
        xs.append(torch.empty_like(f))
        unknowns += m * nb * k
    torch.cuda.synchronize()
    return mats, keep, fs, xs, unknowns


def _time_batch(args, B, sync_each, steps, warmup):
    """Warm-up, then `steps` replays between synchronizations; returns
    (ms per step, per-step ms list, infos of the last run)."""
    import torch
    import numpy as np
    infos = None
    for _ in range(warmup):
        infos = B.run(want_info=sync_each)
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        infos = B.run(want_info=sync_each)
        if sync_each:
            per.append((time.perf_counter() - t1) * 1e3)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    if not per:
        per = [wall]
    return wall, np.array(per), infos


def run_batch(args):
    """Batched workload: 512 independent block tridiagonal systems (m in
    {4, 8, 16, 32}, N log-uniform in [2^8, 2^16], 1..64 right-hand sides),
    one pf_batch replayed from a HIP graph per step, in FP64 and with FP32
    factors + FP64 refinement.  Throughput counts m*nb unknowns per system
    per right-hand side, only if every result meets eta <= 1e-12."""
    import numpy as np
    import torch

    from paper_0912_3678_amd import pf
    from paper_0912_3678_amd import workloads as wl

    dev = torch.device("cuda", 0)
    count = args.count or 512
    n_hi = args.n_hi or 2 ** 16
    specs = wl.batch_specs(count=count, n_hi=n_hi)
    mats, keep, fs, xs, unknowns = _batch_device_systems(specs, dev)
    nrhs = [k for _, _, k, _ in specs]
    flags = pf.PF_FLAG_AUTOTUNE if args.autotune else 0
    precs = [args.prec] if args.prec else ["fp64", "fp32ir"]
    res = {}
    for prec in precs:
        opts = pf.make_opts(prec=pf.PF_FP32_IR if prec == "fp32ir" else pf.PF_FP64, flags=flags,
                            block_rows=args.block_rows, coarse_rows=args.coarse_rows)
        t_c = time.perf_counter()
        B = pf.Batch(mats, opts, nrhs, fs, xs)
        create_s = time.perf_counter() - t_c
        ir = prec == "fp32ir"
        steps = args.steps if not ir else max(1, min(args.steps, args.ir_steps))
        wall, per, infos = _time_batch(args, B, ir, steps, args.warmup if not ir else 1)
        if infos is None:
            infos = B.run(want_info=True)
        etas = [_eta_btri_torch(*keep[i], fs[i], xs[i], specs[i][0], specs[i][1])
                for i in range(len(specs))]
        bad = sum(1 for i in infos if i.status != 0)
        launches = B.profile()
        B.destroy()
        ok = max(etas) <= 1e-12 and bad == 0
        r = {"ms_per_step": wall, "value": unknowns / (wall * 1e-3) if ok else 0.0,
             "eta_max": max(etas), "bad_status": bad, "create_s": round(create_s, 2),
             "steps": steps, "latency_ms": {"p50": float(np.percentile(per, 50)),
                                             "p99": float(np.percentile(per, 99))},
             "launches": launches}
        if ir:
            its = [i.refine_iters for i in infos]
            r["refine_iters"] = {str(v): its.count(v) for v in sorted(set(its))}
        res[prec] = r
    # give the batch's device memory back before the serving stream, whose
    # server may hold up to its budget (250 GB) of the 288 GB
    del mats, keep, fs, xs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    main = res["fp64"] if "fp64" in res else res[precs[0]]
    mprec = "fp64" if "fp64" in res else precs[0]
    # dominant grouped launch of the main run, its roofline by the method's
    # per-unit figures (m_true = the block size of the systems it covers)
    dom = max(main["launches"], key=lambda L: L["ms"])
    m_true = dom["m"]
    byt, fl, bound = batch_launch_roofline(dom, m_true)
    t = dom["ms"] * 1e-3
    kname = batch_kernel_name(dom)
    traffic = load_traffic(kname, grid=dom["workgroups"] * 64)
    if bound == "mfma":
        peak = FP32_PEAK_TFLOPS if dom["f32"] else FP64_PEAK_TFLOPS
        roof = {"bound": "mfma", "achieved": round(fl / t / 1e12, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(fl / t / 1e12 / peak, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(byt / t / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(byt / t / 1e9 / HBM_PEAK_GBS, 4)}
    roof.update({"kernel": kname, "level": dom["level"], "m": dom["m"],
                 "alg_bytes_per_launch": int(byt), "alg_flops_per_launch": int(fl),
                 "avg_launch_us": round(dom["ms"] * 1e3, 1),
                 "traffic": traffic["total_bytes"] if traffic else None,
                 "traffic_split": ({"fetch_bytes": traffic["fetch_bytes"],
                                    "write_bytes": traffic["write_bytes"]} if traffic else None)})
    # whole-step roofline: sum over systems of max(bytes / BW, flops / peak)
    t_roof = 0.0
    for (m, nb, k, _) in specs:
        b_sys = 3 * m * m * 8 * nb + 2 * m * 8 * nb * k
        f_sys = 12.7 * m ** 3 * nb + 10 * m * m * nb * k
        t_roof += max(b_sys / (HBM_PEAK_GBS * 1e9), f_sys / (FP64_PEAK_TFLOPS * 1e12))
    for r in res.values():
        # kernel time per block size, finest level and reduced levels apart
        by_m = {}
        for L in r["launches"]:
            e = by_m.setdefault(str(L["m"]), {"level0_ms": 0.0, "reduced_ms": 0.0})
            e["level0_ms" if L["level"] == 0 else "reduced_ms"] += L["ms"]
        r["kernel_ms_by_m"] = {k: {kk: round(vv, 3) for kk, vv in v.items()}
                               for k, v in sorted(by_m.items(), key=lambda kv: int(kv[0]))}
        r["launches"] = sorted(
            [{"kernel": batch_kernel_name(L), "phase": L["phase"], "level": L["level"],
              "m": L["m"], "rows": L["rows"], "rhs_rows": L["rhs_rows"],
              "us": round(L["ms"] * 1e3, 1)} for L in r["launches"]],
            key=lambda d: -d["us"])[:12]
    out = {
        "metric": "unknowns solved/sec (N*m per right-hand side) at residual<=1e-12; "
                  "p50/p99 solve latency under load",
        "value": main["value"],
        "unit": "unknowns/s", "n_gpus": 1, "steps": main["steps"], "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mprec == "fp64" else "f32 factors + f64 refinement",
        "data": "synthetic",
        "config": {"workload": "batched_btri_512", "systems": count,
                   "unknowns_x_rhs": unknowns, "n_range": [2 ** 8, n_hi],
                   "m_mix": {str(mm): sum(1 for s_ in specs if s_[0] == mm) for mm in (4, 8, 16, 32)},
                   "matrix_GB": round(sum(3 * m * m * 8 * nb for m, nb, _, _ in specs) / 1e9, 2),
                   "rhs_GB": round(sum(8 * m * nb * k for m, nb, k, _ in specs) / 1e9, 2),
                   "autotune": bool(args.autotune),
                   "block_rows": args.block_rows, "coarse_rows": args.coarse_rows,
                   "step": "pf_batch_run: factor + solve of every system, grouped launches "
                           "replayed from a HIP graph with one branch per block size"},
        "eta_max": main["eta_max"],
        "latency_ms": main["latency_ms"],
        "step_roofline": {"t_roof_ms": round(t_roof * 1e3, 2),
                          "frac": round(t_roof * 1e3 / main["ms_per_step"], 4),
                          "rule": "sum over systems of max(A + f + x bytes / 8 TB/s, "
                                  "(12.7 m^3 + 10 m^2 k) flops per block row / 78.6 TFLOP/s)"},
        "roofline": roof,
        "precisions": {k: {kk: vv for kk, vv in v.items()} for k, v in res.items()},
        "mall": "working set 63 GB >> 256 MB MALL: cold and warm steps coincide",
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(args, specs)
    if not args.no_serving:
        out["serving"] = serving_summary(args)
    return out


def batch_cpu_baseline(args, specs):
    """The oracle (band LU with partial pivoting, FP64) on a bounded sample
    of the batched workload: systems in workload order whose estimated cost
    is at most a few seconds each, until about --cpu-seconds of one core
    are spent; then the same sample spread over all cores (one system per
    thread).  Rates in unknowns x right-hand sides per second."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    from paper_0912_3678_amd import workloads as wl

    name, cores = cpu_model()
    sample, est = [], 0.0
    for (m, nb, k, seed) in specs:
        cost = 16.0 * nb * m ** 3 + 12.0 * nb * m * m * k   # band LU flops + the k solves
        if cost > 3e9:
            continue
        sample.append((m, nb, k, seed))
        est += cost
        if est > args.cpu_seconds * 1.2e9:
            break

    def system(sp):
        m, nb, k, seed = sp
        s = wl.random_btri(nb, m, seed=seed, manufactured=False)
        f = np.random.default_rng(seed + 1).standard_normal((nb * m, k))
        return s, f

    data = [system(sp) for sp in sample]
    t0 = time.perf_counter()
    for s, f in data:
        oracle.btri_solve(s.D, s.Lo, s.Up, f)
    one = time.perf_counter() - t0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda sf: oracle.btri_solve(sf[0].D, sf[0].Lo, sf[0].Up, sf[1]), data))
    allc = time.perf_counter() - t0
    u = sum(m * nb * k for m, nb, k, _ in sample)
    return {"value": u / one, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sample)} systems of the batched workload's law in workload order "
                      f"(those with m^3 nb below 3 GF of band LU work), {u} unknowns x "
                      f"right-hand sides, band LU with partial pivoting, one pass",
            "cpu": name, "all_cores": {"value": u / allc, "cores": cores,
                                       "how": "one system per thread"}}


def serving_summary(args):
    """p50 / p99 latency under load for the batched line: the serving law
    (block sizes 8, 16, 32; N lognormal, median 2^14, clamped to 2^20; 30 %
    repeat right-hand sides on kept factors) through the request scheduler
    under a 250 GB budget: saturation first, then Poisson arrivals at 0.8 x
    that rate; FP64, and FP32 factors + FP64 refinement (key fp32ir)."""
    res = {}
    for prec in ("fp64", "fp32ir"):
        out = _serving(args, count=args.serve_count, n_hi=2 ** 20, budget=250e9, pool_n=64,
                       fracs=(0.8,), prec=prec)
        res[prec] = _serving_line(args, out)
    line = dict(res["fp64"])
    line["fp32ir"] = res["fp32ir"]
    return line


def _serving_line(args, out):
    load = out["load"][-1]
    return {"workload": "serving_stream", "prec": out["prec"], "requests": args.serve_count,
            "n_max": 2 ** 20, "budget_GB": 250, "pool_matrices": 64,
            "saturation_req_s": round(out["saturation"]["throughput_req_s"], 1),
            "saturation_unknowns_s": out["saturation"]["unknowns_per_s"],
            "at_qps": round(load["qps"], 1), "p50_ms": load["p50_ms"], "p99_ms": load["p99_ms"],
            "unknowns_per_s": load["unknowns_per_s"], "eta_max_sample":
                max(out["saturation"]["eta_max_sample"], load["eta_max_sample"]),
            "bad_status": out["saturation"]["bad_status"] + load["bad_status"],
            "host_submit_max_ms": load["host_submit_max_ms"],
            "host_setup_ms_max": load["host_setup_ms_max"],
            "refine_iters": load["refine_iters"], "reserved_GB": out["reserved_GB"]}


def run_serving(args):
    out = _serving(args, count=args.count or 240, n_hi=args.n_hi or 2 ** 20,
                   budget=args.budget_gb * 1e9, pool_n=64, fracs=(0.5, 0.8),
                   prec=args.prec or "fp64")
    sat, runs = out["saturation"], out["load"]
    ok = all(r["bad_status"] == 0 and r["eta_max_sample"] <= 1e-12 for r in [sat] + runs)
    return {
        "metric": "p50/p99 solve latency under load; unknowns solved/sec at residual<=1e-12",
        "value": runs[-1]["unknowns_per_s"] if ok else 0.0, "unit": "unknowns/s",
        "n_gpus": 1, "steps": len(runs) and runs[-1]["requests"], "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 factors + f64 refinement" if out["prec"] == "fp32ir" else "f64",
        "data": "synthetic",
        "config": {"workload": "serving_stream", "requests": args.count or 240,
                   "pool": out["pool"], "n_max": args.n_hi or 2 ** 20,
                   "budget_GB": args.budget_gb},
        "saturation": sat, "load": runs, "reserved_GB": out["reserved_GB"],
        "reserve_s": out["reserve_s"],
        "latency_ms": {"p50": runs[-1]["p50_ms"], "p99": runs[-1]["p99_ms"],
                       "at_qps": runs[-1]["qps"]},
    }


def _serving(args, count, n_hi, budget, pool_n, fracs, prec="fp64"):
    """Request stream through the scheduler.  A pool of matrices drawn from
    the workload's law is generated on the device once; each new request
    factors one of them (the scheduler does not know they repeat), 30 % of
    the requests bring a fresh right-hand side for a kept factor.  The
    saturation throughput is measured first (all requests at once), then the
    stream runs at 0.5x and 0.8x that rate; latency = submission to the
    device completion event."""
    import numpy as np
    import torch

    from paper_0912_3678_amd import pf
    from paper_0912_3678_amd import workloads as wl

    dev = torch.device("cuda", 0)
    pool_specs = wl.serving_stream(pool_n, 1.0, seed=wl.seed_for(5, 1), n_max=n_hi)
    pool = []
    for i, r in enumerate(pool_specs):
        D, Lo, Up, _ = _device_btri(r["m"], r["nb"], 1, r["seed"], dev)
        pool.append((pf.make_matrix(pf.PF_BTRI, r["m"], r["nb"], D, Lo, Up), (D, Lo, Up),
                     r["m"], r["nb"]))
    torch.cuda.synchronize()
    budget = int(budget)

    # one server for every stream of the run: its memory pool, grown by the
    # first (saturation) stream, is reused by the later ones
    opts = pf.make_opts(prec=pf.PF_FP32_IR if prec == "fp32ir" else pf.PF_FP64)
    S = pf.Server(budget, opts, max_inflight=16, nstreams=4)
    # map the stream's device memory ahead (a server's start-up, not timed):
    # every new request keeps its factor until the end of its pass
    per = [pf.pf_factor_bytes(A, opts) + pf.pf_solve_bytes_per_rhs(A, opts) for A, _, _, _ in pool]
    need = sum(per[i % len(pool)] for i, r in enumerate(wl.serving_stream(count, 1e9, n_max=n_hi))
               if not r["repeat"])
    t_r = time.perf_counter()
    S.reserve(min(budget, int(need * 1.1)))
    reserve_s = time.perf_counter() - t_r

    def run_stream(qps):
        stream = wl.serving_stream(count, qps if qps else 1e9, n_max=n_hi)
        # a request's matrix: new requests cycle through the pool, repeats
        # pick a kept factor; each brings a fresh right-hand side
        g = torch.Generator(device=dev)
        g.manual_seed(wl.seed_for(5, 2))
        bufs = [None] * len(stream)
        torch.cuda.synchronize()
        st0 = S.stats()
        kept = []
        tickets = []
        host_submit = 0.0
        submit_ms = []
        t0 = time.perf_counter()
        for i, r in enumerate(stream):
            while qps and time.perf_counter() - t0 < r["t"]:
                S.stats()                                   # keeps the scheduler moving
            if r["repeat"] and kept:
                fac, pi = kept[int(r["pick"] * len(kept))]
            else:
                fac, pi = -1, i % len(pool)
            A, _, m, nb = pool[pi]
            f = torch.randn((1, m * nb), generator=g, device=dev, dtype=torch.float64)
            x = torch.empty_like(f)
            th = time.perf_counter()
            try:
                t = S.submit(A, f, x, keep=(fac < 0), factor=fac)
            except pf.PFError:
                # the kept factor was evicted meanwhile: factor again
                t = S.submit(A, f, x, keep=True)
                fac = -1
            host_submit += time.perf_counter() - th
            submit_ms.append((time.perf_counter() - th) * 1e3)
            if fac < 0:
                kept.append((t, pi))
            tickets.append((t, pi, fac))
            bufs[i] = (f, x)
        infos = [S.wait(t) for t, _, _ in tickets]
        wall = time.perf_counter() - t0
        times = [S.times(t) for t, _, _ in tickets]
        st = S.stats()
        for t, _ in kept:
            S.release(t)
        lat = np.array([d - sub for sub, _, d in times])
        unknowns = sum(pool[pi][2] * pool[pi][3] for _, pi, _ in tickets)
        # acceptance on a sample of results
        etas = []
        for (t, pi, fac), (f, x) in list(zip(tickets, bufs))[::max(1, len(tickets) // 16)]:
            _, (D, Lo, Up), m, nb = pool[pi]
            etas.append(_eta_btri_torch(D, Lo, Up, f, x, m, nb))
        return {"qps": qps, "requests": len(tickets), "wall_s": round(wall, 3),
                "throughput_req_s": len(tickets) / wall, "unknowns_per_s": unknowns / wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "bad_status": sum(1 for i in infos if i.status != 0), "eta_max_sample": max(etas),
                "evictions": st["evictions"] - st0["evictions"],
                "repeats": sum(1 for _, _, fac in tickets if fac >= 0),
                "host_setup_ms_max": round(st["setup_ms_max"], 2),
                "host_launch_ms_max": round(st["launch_ms_max"], 2),
                "host_submit_ms": round(host_submit * 1e3, 1),
                "host_submit_max_ms": round(max(submit_ms), 2),
                "host_submit_slowest": [int(i) for i in np.argsort(submit_ms)[-5:]],
                "refine_iters": {str(v): sum(1 for i in infos if i.refine_iters == v)
                                 for v in sorted({i.refine_iters for i in infos})}}

    sat = run_stream(0)
    rate = sat["throughput_req_s"]
    runs = [run_stream(frac * rate) for frac in fracs]
    S.destroy()
    return {"saturation": sat, "load": runs, "pool": len(pool), "prec": prec,
            "reserved_GB": round(min(budget, int(need * 1.1)) / 1e9, 2),
            "reserve_s": round(reserve_s, 3)}


if __name__ == "__main__":
    main()
