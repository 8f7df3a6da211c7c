#!/usr/bin/env python3
"""Time-to-solution benchmark of the subdomain-levelset deflated PCG path on one MI355X.

One step = the whole hot path for one permeability field already resident in HBM:
transmissibilities -> subdomain-levelset labels -> E = Z^T A Z with its Cholesky inverse
-> deflated PCG to ||b - A x|| <= 1e-8 ||b|| (float32 CG inside float64 refinement by
default; the plain float64 path is timed beside it). Prints one JSON line.

Workload (default): the 256 x 256 x 128 channelized field (8.4 M cells; Gaussian random
field with correlation length 16 thresholded into 30 % channels, log-normal permeability in
each facies, contrast 1e6), 16 x 16 x 8 subdomains x 2 levelsets with every region split into
its connected pieces (d = 4139), p = 0 on the x = 0 face, unit source / sink in opposite
corners. Its working set (~0.5 GB) exceeds the 256 MiB Infinity Cache, so the kernels stream
from HBM. Kernel durations are taken inside real solves (events around every launch of the
kernel on the solve's stream, launches that exit at once after convergence left out).
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

METRIC = ("time-to-1e-8 rel. residual (s), iterations, SpMV HBM GB/s vs plain FP64 DPCG")
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c1": "layered2d 64x64, 4x4 subdomains x 2 levelsets",
    "c2": "layered3d 128x128x64, 8 layers log-normal K (sigma 1), layer means 1 / 1e-6, "
          "8x8x4 subdomains x 2 levelsets",
    "c3": "channelized 256x256x128 (GRF corr. length 16, 30% channels), contrast 1e6, "
          "16x16x8 subdomains x 2 levelsets",
    "c3cc": "channelized 256x256x128 (GRF corr. length 16, 30% channels), contrast 1e6, "
            "16x16x8 subdomains x 2 levelsets, each region split into connected components",
    "c4": "batch of 64 layered cubes, side U{32..96} (seed-drawn), contrast log-uniform "
          "1e4..1e6, 4x4x4 subdomains x 2 levelsets, well columns; solved together",
    "c5": "learned start vector: 128x128x64 layered / channelized instances (contrast "
          "log-uniform 1e4..1e6, well columns), 8x8x4 subdomains x 2; 4-level bf16 conv net "
          "(16/32/48/64 channels) trained on plain float64 solutions",
}

BF16_MFMA_PEAK_TFLOPS = 2500.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kernel: str, grid, d: int, m_faces: int, w: int, two: bool,
                      coarse_sym: bool = False, face_tables: bool = False) -> float:
    """Bytes one launch must move at minimum (each array touched once), w = word size.

    two=True: the two-reduction loop (float32 path); False: the single-reduction loop.
    coarse_sym: the coarse product reads the lower triangle of the symmetric E^-1 and
    writes and re-reads one share of e per (row block, column block) of 64.
    face_tables: the float32 update reads each cut face as one packed word and its T
    (4 + w bytes instead of 12 + w); the per-tile tables of coarse values (a few labels
    per tile, cache-resident) are not counted.
    """
    nx, ny, nz = grid
    n = nx * ny * nz
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    if kernel == "direction":   # split stencil step: read u, p_prev; write p
        return 3 * w * n
    if kernel == "stencil_split":   # its plain stencil: read p, Tx, Ty, Tz, slot; write q
        return 2 * w * n + w * faces + 1 * n
    if kernel == "stencil":
        if two:   # read u, p_prev, Tx, Ty, Tz, slot; write p, q = A p
            return 4 * w * n + w * faces + 1 * n
        return 2 * w * n + w * faces + 1 * n + w * n   # read r, u, T, slot; write v = A u
    if kernel == "update":
        if two:   # read q, r, p, x, 1/diag; write r, x, u; + the cut faces of A Z
            return 8 * w * n + m_faces * ((4 if face_tables else 12) + w)
        return 12 * w * n + m_faces * (12 + w)   # read v, r, u, p, q, x, 1/diag; write 5
    if kernel == "coarse":           # read E^-1 (float64), s; write e
        if coarse_sym:
            nb = (d + 63) // 64
            return 8.0 * d * (d + 1) / 2 + 2 * 8.0 * nb * nb * 64 + 4 * 8 * d
        return 8.0 * d * d + 4 * 8 * d
    if kernel == "cheb_step":         # read y, r, 1/diag, d, T; write y
        return float(w) * (4 * n + faces) + float(w) * n
    if kernel.startswith("gs_pass"):  # read nv basis vectors and w, write w (float64)
        nv = int(kernel.split("_")[-1])
        return (nv + 2) * 8.0 * n
    raise KeyError(kernel)


SOLVER_NAMES = {
    "dpcg": lambda a: "DEF1-PCG",
    "gmres": lambda a: (f"deflated GMRES({a.restart})" +
                        (f" with Chebyshev preconditioner (degree {a.gmres_degree})"
                         if a.gmres_degree >= 2 else "")),
    "poly": lambda a: f"DEF1-PCG with Chebyshev preconditioner (degree {a.degree}, ratio {a.ratio:g})",
}
SOLVER_TAGS = {
    "dpcg": lambda a: "dpcg",
    "gmres": lambda a: (f"pdgmres({a.restart})" +
                        (f"-cheb(degree {a.gmres_degree}, ratio 30)" if a.gmres_degree >= 2 else "")),
    "poly": lambda a: f"dpcg-cheb(degree {a.degree}, ratio {a.ratio:g})",
}


def counter_traffic(kernel: str, workload: str, mode: str, coarse_sym: int = 0,
                    tile_cells=None, wide_tiles: int = 0):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter summary
    (FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel calibration), or None when no
    summary covers this kernel, workload, mode and tiling (tile size, wide tiles) or the
    kernel source changed since."""
    import glob
    import hashlib
    src_path = os.path.join(ROOT, "paper_1510_02148_amd", "csrc", "psl_solve.hip")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.md"))):
        fields = {}
        for line in open(path):
            k, sep, v = line.strip().partition(": ")
            if sep:
                fields[k] = v.strip()
        if (fields.get("bench_kernel"), fields.get("workload"), fields.get("mode")) != \
                (kernel, workload, mode):
            continue
        if kernel == "coarse" and int(fields.get("coarse_sym", "0")) != int(coarse_sym):
            continue
        if (fields.get("tile_cells"), fields.get("wide_tiles")) != \
                (str(tile_cells), str(int(wide_tiles))):
            continue
        src = open(src_path).read()
        # the kernel and every device function it inlines, each from its marker to the
        # end of its body
        markers = fields.get("source_markers", fields.get("source_marker", "\0")).split(" | ")
        bodies = []
        for m in markers:
            i = src.find(m)
            if i < 0:
                return None
            bodies.append(src[i - 4:src.index("\n}\n", i)])
        if hashlib.sha256("\n".join(bodies).encode()).hexdigest() != \
                fields.get("kernel_source_sha256"):
            return None
        kib = 1024.0
        return (float(fields["fetch_kib_per_dispatch"]) * float(fields["fetch_factor"]) +
                float(fields["write_kib_per_dispatch"]) * float(fields["write_factor"])) * kib
    return None


def make_problem(name: str, seed: int):
    import psl_inputs as pi
    if name in ("c3", "c3cc"):
        return pi.config("c3", seed=seed, contrast=1e6)
    return pi.config(name, seed=seed)


def in_solve_kernel_times(psl, ctx, b, tol, mode, kernel_ids, max_launches=8192):
    """Per kernel: durations of its launches inside one real solve (events on the solve's
    stream around each launch; psl_profile_kernel). Launches shorter than a quarter of the
    median are the ones enqueued past convergence that return at once: left out."""
    import numpy as np
    out = {}
    for name, kid in kernel_ids.items():
        psl.psl_profile_kernel(ctx, kid, mode, max_launches)
        psl.psl_solve(ctx, b, tol=tol, mode=mode)
        dur = np.array(psl.psl_profile_read(ctx, max_launches))
        psl.psl_profile_kernel(ctx, -1, mode)
        if dur.size == 0:
            continue
        keep = dur[dur >= 0.25 * np.median(dur)]
        out[name] = {"us": float(keep.mean()), "launches": int(keep.size),
                     "early_exit_launches": int(dur.size - keep.size),
                     "total_ms": float(keep.sum() * 1e-3)}
    return out


def run_batched(args):
    """64 uneven systems solved together (psl_solve_batched, float64 CG): one step =
    set-up of every system (tuned tile sizes) + the batched solve to 1e-8 each."""
    import numpy as np
    import torch

    import psl_inputs as pi
    from paper_1510_02148_amd import autotune, pipeline, psl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    probs = pi.batch(nsys=64, seed=args.seed)
    ntot = sum(p.n for p in probs)
    log(f"workload c4: 64 systems, sides {min(p.grid[0] for p in probs)}.."
        f"{max(p.grid[0] for p in probs)}, {ntot} cells")
    Ks = [torch.as_tensor(p.K, dtype=torch.float64, device="cuda") for p in probs]
    bs = [torch.as_tensor(p.q, dtype=torch.float64, device="cuda") for p in probs]
    table = autotune.load_table()
    tiles = autotune.tiles_for([p.grid for p in probs], table)
    if any(t is None for t in tiles):
        log("no tuned tile sizes for this GPU: tuning (outside the timed region)")
        table = autotune.tune(probs, log=log)
        tiles = autotune.tiles_for([p.grid for p in probs], table)
    torch.cuda.synchronize()

    def setup_all(tl):
        return [pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr), tile_cells=t)
                for p, K, t in zip(probs, Ks, tl)]

    def step(tl, mode=psl.FP64):
        t0 = time.perf_counter()
        setups = setup_all(tl)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xs, stats, rc = psl.psl_solve_batched([s.ctx for s in setups], bs, mode=mode)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return setups, xs, stats, rc, t1 - t0, t2 - t1

    def leg(tl, label, mode=psl.FP64):
        for _ in range(args.warmup):
            step(tl, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = [step(tl, mode) for _ in range(args.steps)]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        setups, xs, stats, rc = rec[-1][:4]
        log(f"{label}: {wall * 1e3:.2f} ms/step, setup {np.median([r[4] for r in rec]) * 1e3:.1f}"
            f" ms, solve {np.median([r[5] for r in rec]) * 1e3:.1f} ms, status {rc}")
        return rec, wall

    rec, wall = leg(tiles, "batched, tuned tiles")
    setups, xs, stats, rc = rec[-1][:4]
    solve_s = float(np.median([r[5] for r in rec]))
    setup_s = float(np.median([r[4] for r in rec]))
    ok = rc == 0 and all(st["relres_true"] <= 1e-8 for st in stats)
    # the same systems solved one after another by psl_solve
    torch.cuda.synchronize()
    seq = []
    for _ in range(max(1, args.steps // 2)):
        t0 = time.perf_counter()
        for s, b in zip(setups, bs):
            psl.psl_solve(s.ctx, b, mode=psl.FP64)
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t0)
    seq_s = float(np.median(seq))
    log(f"sequential psl_solve: {seq_s * 1e3:.1f} ms")
    _, wall_def = leg([None] * len(probs), "batched, library-default tiles")
    # the same batch in mixed precision (float32 refinement steps for all systems together)
    rec_m, wall_m = leg(tiles, "batched mixed, tuned tiles", mode=psl.MIXED)
    stats_m, rc_m = rec_m[-1][2], rec_m[-1][3]
    mixed_leg = {"s_per_step": round(wall_m, 6),
                 "solve_s": float(np.median([r[5] for r in rec_m])),
                 "converged": bool(rc_m == 0 and all(st["relres_true"] <= 1e-8 for st in stats_m)),
                 "iterations_mean": round(float(np.mean([st["iters"] for st in stats_m])), 1),
                 "fell_back": int(sum(st["fell_back"] for st in stats_m)),
                 "speedup_vs_fp64_batched": round(wall / wall_m, 3)}
    # effective bandwidth of the whole batched solve (stencil + coarse + update per iteration)
    total_bytes = 0.0
    for p, s, st in zip(probs, setups, stats):
        info = psl.psl_get_info(s.ctx)
        per_it = sum(algorithmic_bytes(k, p.grid, s.d, int(info["m_faces"]), 8, False)
                     for k in ("stencil", "coarse", "update"))
        total_bytes += st["iters"] * per_it
    gbs = total_bytes / solve_s / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import psl_oracle as O
        sample = sorted(range(len(probs)), key=lambda i: probs[i].n)[::16][:3]
        ns = sum(probs[i].n for i in sample)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            for i in sample:
                p = probs[i]
                A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
                lab, dd = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
                O.dpcg(A, bh, O.deflation_matrix(lab, dd), tol=p.tol)
            t_s = time.perf_counter() - t0
        cpu = {"value": round(t_s * ntot / ns, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"systems {sample} ({ns} of {ntot} cells) solved whole by the oracle "
                         f"in {t_s:.2f} s on 1 thread, scaled by cells to the batch"}
        log(f"cpu oracle sample: {t_s:.2f} s for {ns} cells")
    out = {
        "metric": METRIC, "value": round(wall, 6), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"], "systems": len(probs), "cells": ntot,
                   "tol": 1e-8, "mode": "fp64", "seed": args.seed},
        "converged": bool(ok), "iterations_max": max(st["iters"] for st in stats),
        "iterations_mean": round(float(np.mean([st["iters"] for st in stats])), 1),
        "setup_s": setup_s, "solve_s": solve_s, "sequential_solve_s": seq_s,
        "speedup_vs_sequential": round(seq_s / solve_s, 3),
        "default_tiles_s_per_step": round(wall_def, 6),
        "mixed": mixed_leg,
        "tiles": {str(k): v["tile_cells"] for k, v in sorted(table.items())},
        "roofline": {"bound": "hbm", "kernel": "batched CG (stencil + coarse + update)",
                     "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _gen_instance(seed):
    import psl_inputs as pi
    return pi.learned_x0_instance(seed)


def run_learned(args):
    """Learned start vector on held-out instances: one step = network inference + scale +
    float64 solve from that start, against the same solve from x0 = 0. Training (outside
    the timed region) uses a reduced set of instances and steps."""
    import multiprocessing as mp

    import numpy as np
    import torch

    from paper_1510_02148_amd import nn, x0net, x0train
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ntr, nte = args.train_instances, args.test_instances
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        tr = pool.map(_gen_instance, [1000 + i for i in range(ntr)])
        te = pool.map(_gen_instance, [5000 + i for i in range(nte)])
    log(f"generated {ntr} + {nte} instances in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    dtr, dte = x0train.prepare(tr), x0train.prepare(te)
    log(f"reference solves in {time.perf_counter() - t0:.1f} s")
    grid = tuple(tr[0].grid)
    net = x0net.X0Net(grid, seed=args.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = x0train.train(net, dtr, args.train_steps, lr=1e-3, log=log, log_every=500,
                           loss=args.loss)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"training: {args.train_steps} steps in {t_train:.1f} s "
        f"({t_train / args.train_steps * 1e3:.2f} ms/step), loss {losses[:50].mean():.4f} -> "
        f"{losses[-50:].mean():.4f}")
    for _ in range(args.warmup):
        x0train.evaluate(net, dte[:1])
    ev = x0train.evaluate(net, dte, repeats=args.steps)
    t_zero = float(np.mean([r["t_zero"] for r in ev]))
    t_net = float(np.mean([r["t_net"] for r in ev]))
    it_zero = float(np.mean([r["iters_zero"] for r in ev]))
    it_net = float(np.mean([r["iters_net"] for r in ev]))
    ok = all(r["relres_net"] <= 1e-8 for r in ev)
    log(f"test: iterations {it_zero:.1f} (x0 = 0) vs {it_net:.1f} (learned), time "
        f"{t_zero * 1e3:.2f} vs {t_net * 1e3:.2f} ms, start loss "
        f"{np.mean([r['loss_net'] for r in ev]):.4f}")
    # dominant convolution: the full-resolution decoder layer (largest forward time)
    L = net.P["d0"]
    n0 = net.ns[0]
    flops = 2.0 * 27 * L["cin"] * L["cout"] * n0
    stream = torch.cuda.current_stream()
    nn.conv3(net.grids[0], net.A["cat0"], L["cin"], L["w"], L["cout"], L["pb"], True, net.A["d0"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        nn.conv3(net.grids[0], net.A["cat0"], L["cin"], L["w"], L["cout"], L["pb"], True,
                 net.A["d0"])
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / 20
    tfs = flops / (us * 1e-6) / 1e12
    e0.record(stream)
    for _ in range(5):
        net.forward()
    e1.record(stream)
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 5
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import psl_oracle as O
        p = te[0]
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
            lab, dd = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
            res = O.dpcg(A, bh, O.deflation_matrix(lab, dd), tol=p.tol)
            cpu_s = time.perf_counter() - t0
        cpu = {"value": round(cpu_s, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"test instance 0 solved by the oracle from x0 = 0 ({res.iters} "
                         f"iterations), 1 thread"}
    out = {
        "metric": METRIC, "value": round(t_net, 6), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_net * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-net/f64-solve", "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"], "grid": list(grid), "train_instances": ntr,
                   "test_instances": nte, "train_steps": args.train_steps, "loss": args.loss,
                   "tol": 1e-8, "seed": args.seed},
        "converged": bool(ok), "iterations_zero_start": it_zero, "iterations_learned": it_net,
        "time_zero_start_s": t_zero, "speedup_vs_zero_start": round(t_zero / t_net, 3),
        "start_loss": float(np.mean([r["loss_net"] for r in ev])),
        "train_s": round(t_train, 2), "train_ms_per_step": round(t_train / args.train_steps * 1e3, 3),
        "train_loss_first": float(losses[:50].mean()), "train_loss_last": float(losses[-50:].mean()),
        "inference_ms": round(fwd_ms, 3),
        "roofline": {"bound": "mfma", "kernel": "conv3 d0 forward (48->16, 1M cells, bf16)",
                     "achieved": round(tfs, 1), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tfs / BF16_MFMA_PEAK_TFLOPS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3cc", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--kernel-reps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain float64 comparison")
    ap.add_argument("--train-instances", type=int, default=128)
    ap.add_argument("--test-instances", type=int, default=16)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--loss", default="energy", choices=["energy", "diag", "l2"])
    ap.add_argument("--labels", default=None, choices=["regions", "components"],
                    help="deflation space: one vector per (subdomain, class) region, or per "
                         "connected component of each region (psl_build_Z_cc); default: "
                         "components for c3cc, regions otherwise")
    ap.add_argument("--solver", default="dpcg", choices=["dpcg", "gmres", "poly"],
                    help="deflated CG (default), the paper's deflated GMRES(m), or deflated "
                         "CG with the Chebyshev polynomial preconditioner; the last two float64")
    ap.add_argument("--restart", type=int, default=30, help="m of GMRES(m)")
    ap.add_argument("--gmres-degree", type=int, default=0,
                    help="GMRES preconditioner: 0 diag(A), 2..16 Chebyshev steps")
    ap.add_argument("--degree", type=int, default=3, help="Chebyshev steps (--solver poly)")
    ap.add_argument("--ratio", type=float, default=30.0,
                    help="Chebyshev interval [2 / ratio, 2] (--solver poly)")
    ap.add_argument("--tiles", default=None,
                    help="tile sizes 'f64,f32' instead of the tuned ones (tuning runs)")
    ap.add_argument("--coarse", default="auto", choices=["auto", "sym", "dense"],
                    help="coarse product over the lower block triangle of E^-1 or the dense "
                         "one (default: the library's choice by d)")
    ap.add_argument("--quick", action="store_true",
                    help="one step, no comparison legs (for profiler counter runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the single-system PSL solve "
                          "is not sharded across GPUs, and no multi-GPU run is made",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.labels is None:
        args.labels = "components" if args.workload == "c3cc" else "regions"
    if args.quick:
        args.steps, args.warmup, args.no_fp64, args.no_cpu_baseline = 1, 0, True, True
    if args.workload == "c4":
        return run_batched(args)
    if args.workload == "c5":
        return run_learned(args)

    import numpy as np
    import torch

    from paper_1510_02148_amd import autotune, pipeline, psl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = make_problem(args.workload, args.seed)
    log(f"workload {args.workload} grid={prob.grid} nsub={prob.nsub} n={prob.n}")
    # tile size per precision from the autotuner's table (tuned now, outside the timed
    # region, when this machine has no entry)
    tiles = {}
    for prec in ("f64", "f32"):
        t = autotune.tiles_for([prob.grid], precision=prec, kind="single")[0]
        if t is None:
            log(f"no tuned {prec} tile size for this shape class: tuning")
            entries = autotune.tune_single(prob, prec, log=log)
            autotune.save_table(entries)
            t = autotune.tiles_for([prob.grid], entries, precision=prec, kind="single")[0]
        tiles[prec] = t
    if args.tiles:
        tiles["f64"], tiles["f32"] = (int(v) for v in args.tiles.split(","))
    log(f"tile sizes: float64 {tiles['f64']}, mixed {tiles['f32']}")
    K = torch.as_tensor(prob.K, dtype=torch.float64, device=dev)
    b = torch.as_tensor(prob.q, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def step(mode):
        t0 = time.perf_counter()
        s = pipeline.setup(prob.grid, K, prob.dirichlet_mask, prob.nsub, list(prob.thr),
                           tile_cells=tiles["f32" if mode == psl.MIXED else "f64"],
                           components=args.labels == "components",
                           coarse_sym={"auto": 0, "sym": 1, "dense": -1}[args.coarse])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if args.solver == "gmres":
            x, st = psl.psl_solve_gmres(s.ctx, b, tol=prob.tol, restart=args.restart,
                                        degree=args.gmres_degree)
        elif args.solver == "poly":
            x, st = psl.psl_solve_poly(s.ctx, b, tol=prob.tol, degree=args.degree,
                                       ratio=args.ratio, mixed=mode == psl.MIXED)
        else:
            x, st = psl.psl_solve(s.ctx, b, tol=prob.tol, mode=mode)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return s, x, st, t1 - t0, t2 - t1

    def run_leg(mode, steps, warmup, label):
        for i in range(warmup):
            s, x, st, _, _ = step(mode)
            log(f"{label} warmup {i}: status={st['status_str']} iters={st['iters']}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = []
        for _ in range(steps):
            s, x, st, ts, tv = step(mode)
            rec.append((st, ts, tv))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        st = rec[-1][0]
        log(f"{label}: {wall * 1e3:.3f} ms/step  status={st['status_str']} iters={st['iters']} "
            f"outer={st['outer']} relres={st['relres_true']:.2e}")
        return s, x, rec, wall

    if args.solver == "gmres":
        args.mode = "fp64"        # the GMRES path is float64 only
    mode = psl.MIXED if args.mode == "mixed" else psl.FP64
    s, x, rec, wall = run_leg(mode, args.steps, args.warmup, args.mode)
    st = rec[-1][0]
    ok = all(r[0]["status"] == 0 and r[0]["relres_true"] <= prob.tol for r in rec)
    setup_s = float(np.median([r[1] for r in rec]))
    solve_s = float(np.median([r[2] for r in rec]))

    fp64 = None
    if not args.no_fp64 and mode != psl.FP64:
        s64, x64, rec64, wall64 = run_leg(psl.FP64, args.steps, min(args.warmup, 1), "fp64")
        st64 = rec64[-1][0]
        fp64 = {"s_per_step": wall64, "setup_s": float(np.median([r[1] for r in rec64])),
                "solve_s": float(np.median([r[2] for r in rec64])), "iters": st64["iters"],
                "relres_true": st64["relres_true"], "status": st64["status_str"]}
        del s64, x64
    # the same workload with the Chebyshev polynomial preconditioner (float64), for context
    cheb = {}
    if not args.no_fp64 and args.solver == "dpcg":
        for label, cmode in (("fp64", psl.FP64), ("mixed", psl.MIXED)):
            args.solver = "poly"
            sp, xp, recp, wallp = run_leg(cmode, args.steps, min(args.warmup, 1),
                                          f"chebyshev {label}")
            args.solver = "dpcg"
            stp = recp[-1][0]
            cheb[label] = {"s_per_step": wallp, "setup_s": float(np.median([r[1] for r in recp])),
                           "solve_s": float(np.median([r[2] for r in recp])),
                           "iters": stp["iters"], "outer": stp["outer"],
                           "relres_true": stp["relres_true"], "status": stp["status_str"],
                           "degree": args.degree, "ratio": args.ratio}
            del sp, xp

    # ---- per-kernel durations with events on the stream the kernels run on ----------
    w = 4 if mode == psl.MIXED else 8
    d = s.d
    info = psl.psl_get_info(s.ctx)
    m_faces = int(info["m_faces"])
    kernels = {}
    stream = torch.cuda.current_stream()
    ids = {"stencil": psl.KERNEL_STENCIL, "coarse": psl.KERNEL_COARSE,
           "update": psl.KERNEL_UPDATE}
    small = args.solver == "dpcg" and mode == psl.FP64 and bool(info["small_solve"])
    if small:
        # small grids: the whole float64 inner solve is one launch of one workgroup
        t = in_solve_kernel_times(psl, s.ctx, b, prob.tol, mode,
                                  {"small_solve": psl.KERNEL_SMALL_SOLVE})["small_solve"]
        iters = max(1, int(st["iters"]))
        kernels["small_solve"] = {"us": round(t["us"], 3), "launches": t["launches"],
                                  "us_per_iteration": round(t["us"] / iters, 3),
                                  "total_ms": round(t["total_ms"], 3), "timing": "in-solve"}
    elif args.solver == "dpcg":
        # inside real solves: every launch of the kernel in the solve's own precision (the
        # direction pass has launches only where the float32 stencil step is split)
        if mode == psl.MIXED:
            ids["direction"] = psl.KERNEL_DIRECTION
        times = in_solve_kernel_times(psl, s.ctx, b, prob.tol, mode, ids)
        for name, t in times.items():
            model = "stencil_split" if (name == "stencil" and "direction" in times) else name
            nbytes = algorithmic_bytes(model, prob.grid, d, m_faces, w, mode == psl.MIXED,
                                       bool(info["coarse_sym"]), bool(info["face_tables"]))
            kernels[name] = {"us": round(t["us"], 3), "alg_bytes": int(nbytes),
                             "gbs": round(nbytes / (t["us"] * 1e-6) / 1e9, 1),
                             "launches": t["launches"],
                             "early_exit_launches": t["early_exit_launches"],
                             "total_ms": round(t["total_ms"], 3), "timing": "in-solve"}
    else:
        if args.solver == "gmres":
            # the Gram-Schmidt pass (update fused with the dots) at the restart length's
            # largest basis; the CG stencil stays as the SpMV bandwidth reference
            ids = {"stencil": psl.KERNEL_STENCIL,
                   f"gs_pass_{min(args.restart, 32)}": psl.KERNEL_GMRES_PASS}
        else:
            # the last Chebyshev step (the widest pass of a degree >= 3 application); the
            # CG stencil stays as the SpMV bandwidth reference
            ids = {"stencil": psl.KERNEL_STENCIL, "cheb_step": psl.KERNEL_POLY_STEP}
        for name, kid in ids.items():
            psl.psl_bench_kernel(s.ctx, kid, mode, 3)            # warm
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            psl.psl_bench_kernel(s.ctx, kid, mode, args.kernel_reps)
            e1.record(stream)
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
            nbytes = algorithmic_bytes(name, prob.grid, d, m_faces, w, mode == psl.MIXED)
            kernels[name] = {"us": round(us, 3), "alg_bytes": int(nbytes),
                             "gbs": round(nbytes / (us * 1e-6) / 1e9, 1),
                             "timing": "back-to-back replays"}
    # plain copy of 1 GiB for the achievable-bandwidth reference
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    psl.psl_bench_copy(src, dst)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        psl.psl_bench_copy(src, dst)
    e1.record(stream)
    e1.synchronize()
    copy_us = e0.elapsed_time(e1) * 1e3 / 10
    copy_gbs = 2 * src.numel() * 4 / (copy_us * 1e-6) / 1e9
    del src, dst
    if small:
        # one workgroup on one compute unit: bound by its barriers and dependent sums,
        # not by HBM (the whole working set is a few hundred KiB)
        kd = kernels["small_solve"]
        roofline = {"bound": "latency", "kernel": "small_solve",
                    "achieved": kd["us_per_iteration"], "unit": "us/iteration", "peak": None,
                    "frac": None, "traffic": None, "copy_kernel_gbs": round(copy_gbs, 1)}
        spmv_gbs = None
    else:
        if args.solver == "dpcg":
            dominant = max(kernels, key=lambda k: kernels[k]["total_ms"])
        else:   # the solver's own pass; the CG stencil is only the SpMV reference there
            dominant = next(k for k in kernels if k != "stencil")
        kd = kernels[dominant]
        traffic = counter_traffic(dominant, args.workload, args.mode, int(info["coarse_sym"]),
                                  tiles["f32" if args.mode == "mixed" else "f64"],
                                  int(info["wide_tiles"]))
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": kd["gbs"],
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4),
                    "traffic": (round(traffic) if traffic is not None else None),
                    "traffic_over_algorithmic": (round(traffic / kd["alg_bytes"], 3)
                                                 if traffic is not None else None),
                    "copy_kernel_gbs": round(copy_gbs, 1)}
        spmv_gbs = kernels["stencil"]["gbs"]

    # ---- CPU baseline: the oracle on the same workload -------------------------------
    cpu = None
    if not args.no_cpu_baseline and args.workload in ("c3", "c3cc") and args.solver == "dpcg":
        # 8.4 M cells: the oracle's full solve takes minutes, so it is timed on a bounded
        # sample (its set-up, and the first 10 and 30 iterations of its DEF1 loop) and the
        # loop is scaled to the iteration count of the float64 GPU solve (which follows the
        # oracle's own count to within 2 %)
        from threadpoolctl import threadpool_limits

        from oracle import psl_oracle as O
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            A, bh = O.assemble(prob.K, prob.grid, prob.dirichlet_mask, prob.q)
            label_fn = (O.levelset_components if args.labels == "components"
                        else O.levelset_labels)
            lab, dd = label_fn(prob.grid, prob.K, prob.nsub, prob.thr)
            Z = O.deflation_matrix(lab, dd)
            co = O.Coarse(A, Z)
            t_setup = time.perf_counter() - t0
            t0 = time.perf_counter()
            O.dpcg(A, bh, Z, tol=prob.tol, maxit=10, coarse=co)
            t10 = time.perf_counter() - t0
            t0 = time.perf_counter()
            r30 = O.dpcg(A, bh, Z, tol=prob.tol, maxit=30, coarse=co)
            t30 = time.perf_counter() - t0
        per_it = (t30 - t10) / 20.0
        fixed = max(0.0, t10 - 10 * per_it)
        iters_ref = fp64["iters"] if fp64 else st["iters"]
        cpu_s = t_setup + fixed + per_it * iters_ref
        cpu = {"value": round(cpu_s, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"oracle on the same field ({args.labels} labels, d = {dd}): assembly, "
                         f"labels, E and its Cholesky factor timed whole ({t_setup:.2f} s); "
                         f"its DEF1-PCG loop timed for 10 and 30 iterations ({t10:.2f} s, "
                         f"{t30:.2f} s: {per_it:.3f} s per iteration) and scaled to the "
                         f"{iters_ref} iterations of the float64 GPU solve; 1 thread",
               "host_cores_available": len(os.sched_getaffinity(0)),
               "oracle_relres_after_30": float(r30.history[-1] / np.linalg.norm(bh)),
               "gpu_relres_by_oracle": float(O.relres(A, bh, x.cpu().numpy()))}
        log(f"cpu oracle (sampled): {cpu_s:.2f} s est., {per_it:.3f} s/iteration")
    elif not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import psl_oracle as O
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            A, bh = O.assemble(prob.K, prob.grid, prob.dirichlet_mask, prob.q)
            label_fn = (O.levelset_components if args.labels == "components"
                        else O.levelset_labels)
            lab, dd = label_fn(prob.grid, prob.K, prob.nsub, prob.thr)
            Z = O.deflation_matrix(lab, dd)
            if args.solver == "gmres":
                res = O.pdgmres(A, bh, Z, m=args.restart, tol=prob.tol, degree=args.gmres_degree)
            elif args.solver == "poly":
                res = O.dpcg_poly(A, bh, Z, degree=args.degree, ratio=args.ratio, tol=prob.tol)
            else:
                res = O.dpcg(A, bh, Z, tol=prob.tol)
            cpu_s = time.perf_counter() - t0
        xg = x.cpu().numpy()
        cpu = {"value": round(cpu_s, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"one full {args.workload} solve (assembly, {args.labels} labels, E + Cholesky, "
                         f"{SOLVER_NAMES[args.solver](args)}"
                         f" to 1e-8), {res.iters} iterations, 1 thread",
               "host_cores_available": len(os.sched_getaffinity(0)),
               "gpu_vs_oracle_rel_err": float(np.linalg.norm(xg - res.x) / np.linalg.norm(res.x)),
               "gpu_relres_by_oracle": float(O.relres(A, bh, xg))}
        log(f"cpu oracle: {cpu_s:.2f} s, {res.iters} iterations")

    dtype = "f32-inner/f64-refine" if mode == psl.MIXED else "f64"
    out = {
        "metric": METRIC, "value": round(wall, 6), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "grid": list(prob.grid),
                   "nsub": list(prob.nsub), "d": d, "labels": args.labels,
                   "solver": SOLVER_TAGS[args.solver](args),
                   "tol": prob.tol,
                   "mode": args.mode, "seed": args.seed, "tile_cells": tiles},
        "converged": bool(ok), "iterations": st["iters"], "outer": st["outer"],
        "relres_true": st["relres_true"], "setup_s": setup_s, "solve_s": solve_s,
        "spmv_gbs": spmv_gbs, "ctx_info": info, "kernels": kernels, "roofline": roofline,
        "fp64_plain": fp64,
        "speedup_vs_fp64": (round(fp64["s_per_step"] / wall, 3) if fp64 else None),
        "chebyshev": cheb or None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
