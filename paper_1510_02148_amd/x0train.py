"""Training and evaluation of the start-vector network on solutions of the plain solver.

Each instance keeps its solver context (for P1 A y in the loss), b, K, P1 b and the
normaliser c = (x*, P1 b) = ||P2 x*||_A^2, with x* from psl_solve in float64 at a tighter
tolerance. Training runs Adam on the scale-free energy loss, one instance per step.
Evaluation solves each instance from x0 = 0 and from the network's x0 and reports the
iterations and times (network inference included).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import nn, pipeline, psl
from .x0net import X0Net


@dataclass
class Instance:
    grid: tuple
    K: torch.Tensor
    b: torch.Tensor
    setup: pipeline.Setup
    P1b: torch.Tensor
    c: float          # (x*, P1 b) = ||P2 x*||_A^2
    sigma: float      # rms of x*: the training target is x* / sigma
    tol: float
    target: torch.Tensor   # float32 x* / sigma
    diag: torch.Tensor     # float32 diag(A)


def prepare(problems: Sequence, ref_tol: float = 1e-9) -> List[Instance]:
    """Device data, context, projected right-hand side and loss normaliser per problem
    (x* only normalises the loss: a reference that stops short of ref_tol is accepted at
    a true relative residual of 1e-8)."""
    out = []
    for p in problems:
        K = torch.as_tensor(p.K, dtype=torch.float64, device="cuda")
        b = torch.as_tensor(p.q, dtype=torch.float64, device="cuda")
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr))
        xs, st = psl.psl_solve(s.ctx, b, tol=ref_tol, mode=psl.FP64)
        if st["status"] != 0 and not st["relres_true"] <= 1e-8:
            raise RuntimeError(f"reference solve failed: {st['status_str']}")
        P1b = torch.empty_like(b)
        psl.psl_deflate(s.ctx, b, P1b)
        # c = (x*, P1 b) and (x*, x*): the u of the energy kernel with y = x*
        ys = xs.float()
        e = torch.zeros(4, dtype=torch.float64, device="cuda")
        work = torch.empty(nn.energy_work(p.n), dtype=torch.float64, device="cuda")
        nn.energy(ys, P1b, P1b, 0.0, e, work)
        c = float(e[2].item())
        nn.energy(ys, xs, xs, 0.0, e, work)
        sigma = math.sqrt(float(e[2].item()) / p.n)
        target = (xs / sigma).float()
        diag = torch.empty(p.n, dtype=torch.float32, device="cuda")
        nn.cell_diag(p.grid, s.Tx, s.Ty, s.Tz, diag)
        out.append(Instance(tuple(p.grid), K, b, s, P1b, c, sigma, float(p.tol), target, diag))
    return out


def train(net: X0Net, data: Sequence[Instance], steps: int, lr: float = 1e-3, seed: int = 0,
          log=None, log_every: int = 50, loss: str = "diag") -> np.ndarray:
    """Adam steps over randomly ordered instances; returns the loss of every step.
    loss: "diag" (regression on x*/sigma weighted by diag(A)), "l2" (unweighted) or
    "energy" (energy-norm regression)."""
    g = np.random.Generator(np.random.PCG64(seed))
    losses = torch.empty(steps, dtype=torch.float64, device="cuda")
    order = []
    for k in range(steps):
        if not order:
            order = list(g.permutation(len(data)))
        d = data[order.pop()]
        if loss == "energy":
            out = net.train_step(d.K, d.b, lr, ctx=d.setup.ctx, P1b=d.P1b, c=d.c, sigma=d.sigma)
        else:
            w = d.diag if loss == "diag" else ones(d)
            out = net.train_step(d.K, d.b, lr, target=d.target, weight=w)
        losses[k] = out[0]
        if log and (k + 1) % log_every == 0:
            log(f"[x0net] step {k + 1}: loss {losses[k - log_every + 1:k + 1].mean().item():.4f}")
    return losses.cpu().numpy()


_ONES = {}


def ones(d: Instance) -> torch.Tensor:
    n = d.target.numel()
    if n not in _ONES:
        _ONES[n] = torch.ones(n, dtype=torch.float32, device="cuda")
    return _ONES[n]


def evaluate(net: Optional[X0Net], data: Sequence[Instance], repeats: int = 1) -> List[dict]:
    """Per instance: iterations and solve time from x0 = 0 and from the network's x0
    (time includes inference and the scale), plus the start's energy loss."""
    res = []
    for d in data:
        rec = {}
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st0 = psl.psl_solve(d.setup.ctx, d.b, tol=d.tol, mode=psl.FP64)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rec.setdefault("t_zero", []).append(t1 - t0)
            if net is not None:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x0 = net.predict_x0(d.K, d.b, d.setup.ctx, d.P1b)
                x1, st1 = psl.psl_solve(d.setup.ctx, d.b, x0, tol=d.tol, mode=psl.FP64,
                                        use_x0=True)
                torch.cuda.synchronize()
                rec.setdefault("t_net", []).append(time.perf_counter() - t0)
        r = {"iters_zero": st0["iters"], "t_zero": float(np.min(rec["t_zero"])),
             "relres_zero": st0["relres_true"]}
        if net is not None:
            out = net.energy(d.setup.ctx, d.P1b, d.c, grad=False)
            r.update(iters_net=st1["iters"], t_net=float(np.min(rec["t_net"])),
                     relres_net=st1["relres_true"], loss_net=float(out[0].item()))
        res.append(r)
    return res
