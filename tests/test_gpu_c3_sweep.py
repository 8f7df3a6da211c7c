"""256x256x128 channelized workload (8.4 M cells) at every contrast of its definition,
element by element against the oracle.

One instance per contrast (seeds 0..3 give contrasts 1e4, 1e5, 1e6, 1e7). The reference
x_ref is the oracle's own DEF1 solve to relative residual 1e-12 with connected-component
vectors (its assembly, labels, E and loop; the solution of A x = b does not depend on the
deflation space), computed in worker processes while the GPU solves run. The bars:
  * relative residual ||b - A x|| / ||b|| <= tol in the oracle's float64 matrix;
  * relative solution error ||x - x_ref|| / ||x_ref|| <= 1e-6.
A 1e-8 residual pins the solution to 1e-6 only when the effective condition number is
below about 100; where the solve at 1e-8 misses the error bar, the same solve is repeated
at 1e-9 and the error bar is asserted there (the error at 1e-8 is printed, not loosened).
"""
import concurrent.futures as cf
import multiprocessing as mp

import numpy as np
import pytest

import psl_inputs as pi
from oracle import psl_oracle as O
from tests import oracle_workers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEEDS = [0, 1, 2, 3]


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def references():
    """Futures of the oracle references, started before the first GPU solve."""
    ex = cf.ProcessPoolExecutor(max_workers=len(SEEDS), mp_context=mp.get_context("spawn"))
    futs = {s: ex.submit(oracle_workers.c3_reference, s) for s in SEEDS}
    yield futs
    ex.shutdown(wait=True, cancel_futures=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _errors(xg, xr):
    e = xg - xr
    return np.linalg.norm(e) / np.linalg.norm(xr), np.abs(e).max() / np.abs(xr).max()


def _check(psl, s, b, A, bh, xr, mode, label):
    """Solve at 1e-8; if the error bar is missed there, solve at 1e-9 and hold it."""
    errs = {}
    for tol in (1e-8, 1e-9):
        x, st = psl.psl_solve(s.ctx, b, tol=tol, mode=mode)
        xg = x.cpu().numpy()
        rel = O.relres(A, bh, xg)
        err, emax = _errors(xg, xr)
        errs[tol] = err
        say(f"  {label} tol={tol:g}: status={st['status_str']} iters={st['iters']} "
            f"outer={st['outer']} relres={rel:.2e} err={err:.2e} max-err={emax:.2e} "
            f"zt_r_drift={st['zt_r_drift']:.1e}")
        assert st["status"] == 0 and rel <= tol
        assert abs(rel - st["relres_true"]) <= 1e-3 * rel + 1e-15
        if err <= 1e-6:
            break
    assert min(errs.values()) <= 1e-6, errs
    return errs


@pytest.mark.parametrize("seed", SEEDS, ids=[f"contrast{c:g}" for c in (1e4, 1e5, 1e6, 1e7)])
def test_channelized_contrast_sweep(gpu_lib, references, seed):
    psl = gpu_lib
    from paper_1510_02148_amd import autotune, pipeline
    p = pi.config("c3", seed=seed)
    say(f"c3 seed={seed} contrast={p.meta.get('contrast')} grid={p.grid}: component vectors, "
        f"float64 and mixed, against the oracle at 1e-12")
    A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    b = dev(p.q)
    xs = {}
    for mode, prec in ((psl.FP64, "f64"), (psl.MIXED, "f32")):
        tile = autotune.tiles_for([p.grid], precision=prec, kind="single")[0]
        s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr),
                           tile_cells=tile, components=True)
        xs[mode] = s
    xr, it_ref, rel_ref, d_ref = references[seed].result(timeout=1500)
    say(f"  oracle: d={d_ref} iters={it_ref} relres={rel_ref:.2e}")
    assert xs[psl.FP64].d == d_ref
    for mode, name in ((psl.FP64, "fp64"), (psl.MIXED, "mixed")):
        _check(psl, xs[mode], b, A, bh, xr, mode, name)
    if seed == 2:
        # one vector per (subdomain, class) region: same solution, other deflation space
        for mode, prec, name in ((psl.FP64, "f64", "fp64-regions"),
                                 (psl.MIXED, "f32", "mixed-regions")):
            tile = autotune.tiles_for([p.grid], precision=prec, kind="single")[0]
            s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr),
                               tile_cells=tile, components=False)
            _check(psl, s, b, A, bh, xr, mode, name)
