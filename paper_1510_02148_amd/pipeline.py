"""Chain the C-ABI calls for one problem: K -> T -> labels -> E -> x.

Argument marshalling only; every step runs in libpsl's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import torch

from . import psl


@dataclasses.dataclass
class Setup:
    grid: tuple
    Tx: torch.Tensor
    Ty: torch.Tensor
    Tz: torch.Tensor
    labels: torch.Tensor
    d: int
    ctx: psl.Context


def setup(grid: Sequence[int], K: torch.Tensor, dirichlet_mask: int, nsub: Sequence[int],
          thr: Sequence[float], cls: Optional[torch.Tensor] = None, ncls: int = 0,
          tile_cells: Optional[int] = None, components: bool = False,
          finish_kernels: int = 0, coarse_sym: int = 0, stencil_split: int = 0,
          face_tables: int = 0, wide_tiles: int = 0) -> Setup:
    """psl_assemble_tpfa -> psl_build_Z (or psl_build_Z_cc) -> psl_setup_E on the current
    stream."""
    Tx, Ty, Tz = psl.psl_assemble_tpfa(grid, K, dirichlet_mask)
    labels, d = psl.psl_build_Z(grid, K, nsub, thr, cls=cls, ncls=ncls, components=components)
    ctx = psl.psl_setup_E(grid, Tx, Ty, Tz, labels, d, nsub=nsub, tile_cells=tile_cells,
                          finish_kernels=finish_kernels, coarse_sym=coarse_sym,
                          stencil_split=stencil_split, face_tables=face_tables,
                          wide_tiles=wide_tiles)
    return Setup(tuple(int(v) for v in grid), Tx, Ty, Tz, labels, d, ctx)


def solve_problem(problem, mode: int = psl.FP64, device: str = "cuda", tol: Optional[float] = None,
                  **solve_kw):
    """Whole path for a psl_inputs.Problem; returns (x, stats, Setup)."""
    K = torch.as_tensor(problem.K, dtype=torch.float64, device=device)
    b = torch.as_tensor(problem.q, dtype=torch.float64, device=device)
    s = setup(problem.grid, K, problem.dirichlet_mask, problem.nsub, list(problem.thr))
    x, stats = psl.psl_solve(s.ctx, b, tol=problem.tol if tol is None else tol, mode=mode,
                             **solve_kw)
    return x, stats, s
