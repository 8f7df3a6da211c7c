"""Tile-size autotuner for the work tiles of psl_setup_E_ex.

A work tile is one workgroup's box of cells (inside one subdomain). Its size trades the
number of workgroups (latency hiding, early exit of finished systems) against the work
and registers per workgroup, and the best value depends on the grid shape: this module
measures it. For every shape class (cell count rounded to a power of two) `tune` builds
contexts for a sample of that class's systems with each candidate tile size, times the
batched float64 solve (warm, best of a few runs) and keeps the fastest; `tune_single` does
the same for one system's solve in a given precision (float64 and float32 loops move
different amounts per cell and prefer different sizes). Results are kept in a JSON table
keyed by GPU architecture and by solve kind, precision and shape class, so tuning runs
once per machine type; `tiles_for` looks sizes up for a list of grids.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence

import torch

from . import pipeline, psl

CANDIDATES = (256, 384, 512, 768, 1024)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def shape_class(n: int) -> int:
    """Shape class of a grid with n cells: round(log2 n)."""
    return int(round(math.log2(max(1, n))))


def arch() -> str:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def load_table(path: str = TABLE_PATH) -> Dict[str, dict]:
    """Entries of the table for this GPU architecture ({} if none)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data.get(arch(), {})


def save_table(entries: Dict[str, dict], path: str = TABLE_PATH) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(arch(), {}).update(entries)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def _key(precision: str, cls: int, kind: str = "batch") -> str:
    """Table key: solve kind (batch / single), precision (f64 / f32), shape class."""
    return f"{kind}-{precision}:{cls}"


def _time_batch(problems, tensors, tile: int, reps: int) -> float:
    setups = [pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr), tile_cells=tile)
              for p, (K, _) in zip(problems, tensors)]
    ctxs = [s.ctx for s in setups]
    bs = [b for _, b in tensors]
    psl.psl_solve_batched(ctxs, bs, check=True)           # warm: plan, graph, caches
    best = math.inf
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        psl.psl_solve_batched(ctxs, bs, check=True)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    for s in setups:
        s.ctx.destroy()
    return best


def tune(problems: Sequence, candidates: Iterable[int] = CANDIDATES, sample: int = 8,
         reps: int = 2, precision: str = "f64", log=print) -> Dict[str, dict]:
    """Time each candidate tile size per shape class of `problems` (psl_inputs.Problem
    objects) for the batched solve; returns the table entries
    {"batch-<precision>:<class>": {"tile_cells", "ms", "systems"}}."""
    by_class: Dict[int, List] = {}
    for p in problems:
        by_class.setdefault(shape_class(p.n), []).append(p)
    entries = {}
    for cls in sorted(by_class):
        group = by_class[cls][:sample]
        tensors = [(torch.as_tensor(p.K, dtype=torch.float64, device="cuda"),
                    torch.as_tensor(p.q, dtype=torch.float64, device="cuda")) for p in group]
        times = {}
        for tile in candidates:
            times[int(tile)] = _time_batch(group, tensors, int(tile), reps) * 1e3
        best = min(times, key=times.get)
        entries[_key(precision, cls, "batch")] = {"tile_cells": best,
                                         "ms": {str(k): round(v, 3) for k, v in times.items()},
                                         "systems": len(group)}
        if log:
            log(f"[autotune] class 2^{cls} ({len(group)} systems): "
                + " ".join(f"{k}:{v:.1f}ms" for k, v in times.items()) + f" -> {best}")
    return entries


def tune_single(problem, precision: str = "f64", candidates: Iterable[int] = CANDIDATES,
                reps: int = 3, log=print, components: bool = False) -> Dict[str, dict]:
    """Time the single-system solve (psl_solve in the given precision, from set-up to
    1e-8) of one problem for each candidate tile size; the table entry for its class.
    components: deflation vectors by connected components (psl_build_Z_cc)."""
    K = torch.as_tensor(problem.K, dtype=torch.float64, device="cuda")
    b = torch.as_tensor(problem.q, dtype=torch.float64, device="cuda")
    mode = psl.MIXED if precision == "f32" else psl.FP64
    times = {}
    for tile in candidates:
        s = pipeline.setup(problem.grid, K, problem.dirichlet_mask, problem.nsub,
                           list(problem.thr), tile_cells=int(tile), components=components)
        psl.psl_solve(s.ctx, b, tol=problem.tol, mode=mode)       # warm
        best = math.inf
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psl.psl_solve(s.ctx, b, tol=problem.tol, mode=mode)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        times[int(tile)] = best * 1e3
        s.ctx.destroy()
    win = min(times, key=times.get)
    cls = shape_class(problem.n)
    if log:
        log(f"[autotune] single {precision} class 2^{cls}: "
            + " ".join(f"{k}:{v:.2f}ms" for k, v in times.items()) + f" -> {win}")
    return {_key(precision, cls, "single"): {"tile_cells": win,
                                             "ms": {str(k): round(v, 3) for k, v in times.items()},
                                             "systems": 1}}


def tiles_for(grids: Sequence[Sequence[int]], table: Optional[Dict[str, dict]] = None,
              precision: str = "f64", kind: str = "batch") -> List[Optional[int]]:
    """Tuned tile size for each grid (None where the table has no entry for its class:
    psl_setup_E then chooses)."""
    table = load_table() if table is None else table
    out = []
    for g in grids:
        e = table.get(_key(precision, shape_class(int(g[0]) * int(g[1]) * int(g[2])), kind))
        out.append(int(e["tile_cells"]) if e else None)
    return out


def main(argv=None):
    """python -m paper_1510_02148_amd.autotune [--single NAME] [--labels L]: tune the
    single-system tile sizes (float64 and float32) of a named workload's shape class and
    store them in the table."""
    import argparse
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import psl_inputs as pi

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--single", default="c3", help="workload name of psl_inputs.config")
    ap.add_argument("--labels", default="components", choices=["regions", "components"])
    ap.add_argument("--precision", default="both", choices=["f64", "f32", "both"])
    a = ap.parse_args(argv)
    prob = pi.config(a.single, contrast=1e6) if a.single == "c3" else pi.config(a.single)
    entries = {}
    for prec in (("f64", "f32") if a.precision == "both" else (a.precision,)):
        entries.update(tune_single(prob, prec, components=a.labels == "components"))
    save_table(entries)


if __name__ == "__main__":
    main()
