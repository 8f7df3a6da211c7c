"""Full-size workloads in the launch configuration the benchmark times (its tuned tile sizes,
its solver entry points), checked through the C-ABI against the oracle.

128x128x64 layered (1.0 M cells): the oracle's own solution and iteration count.
256x256x128 channelized (8.4 M cells): the oracle's DEF1 solves take minutes there, so the
check is a property that holds at any size and fixes the answer: the relative residual of
the GPU x in the oracle's own float64 matrix, <= 1e-8 (with the matrix the oracle assembles
from the same K, so the assembly, labels and solve are all covered), plus the deflation
space size against the oracle's labels.
"""
import numpy as np
import pytest

import psl_inputs as pi
from oracle import psl_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _setup(psl, p, prec, components):
    from paper_1510_02148_amd import autotune, pipeline
    tile = autotune.tiles_for([p.grid], precision=prec, kind="single")[0]
    return pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr),
                          tile_cells=tile, components=components)


def _solve(psl, s, b, solver, mode):
    if solver == "gmres":
        return psl.psl_solve_gmres(s.ctx, b, tol=1e-8, restart=30)
    if solver == "poly":
        return psl.psl_solve_poly(s.ctx, b, tol=1e-8)
    return psl.psl_solve(s.ctx, b, tol=1e-8, mode=psl.MIXED if mode == "mixed" else psl.FP64)


C2_CASES = [("fp64", "dpcg"), ("mixed", "dpcg"), ("fp64", "poly"), ("fp64", "gmres")]


@pytest.mark.parametrize("mode,solver", C2_CASES, ids=[f"{s}-{m}" for m, s in C2_CASES])
def test_layered_full_size(gpu_lib, mode, solver):
    psl = gpu_lib
    p = pi.config("c2")
    say(f"full size c2 {solver} {mode} grid={p.grid}")
    s = _setup(psl, p, "f32" if mode == "mixed" else "f64", False)
    x, st = _solve(psl, s, dev(p.q), solver, mode)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    assert d == s.d == 512
    Z = O.deflation_matrix(lab, d)
    co = O.Coarse(A, Z)
    if solver == "gmres":
        ref = O.pdgmres(A, b, Z, m=30, tol=1e-8, coarse=co)
    elif solver == "poly":
        ref = O.dpcg_poly(A, b, Z, degree=3, ratio=30.0, tol=1e-8, coarse=co)
    else:
        ref = O.dpcg(A, b, Z, tol=1e-8, coarse=co)
    xr = O.dpcg(A, b, Z, tol=1e-12, coarse=co).x
    xg = host(x)
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.iters}) "
        f"relres={O.relres(A, b, xg):.2e}")
    assert st["status"] == 0 and O.relres(A, b, xg) <= 1e-8
    assert np.linalg.norm(xg - xr) / np.linalg.norm(xr) <= 1e-6
    assert abs(st["iters"] - ref.iters) <= max(2, 0.03 * ref.iters)


C3_CASES = [("fp64", "dpcg", False), ("mixed", "dpcg", False), ("mixed", "dpcg", True),
            ("fp64", "poly", True), ("fp64", "poly", False), ("fp64", "gmres", True)]


@pytest.mark.parametrize("mode,solver,components", C3_CASES,
                         ids=[f"{s}-{m}-{'components' if c else 'regions'}"
                              for m, s, c in C3_CASES])
def test_channelized_full_size(gpu_lib, mode, solver, components):
    psl = gpu_lib
    p = pi.config("c3", contrast=1e6)
    say(f"full size c3 {solver} {mode} components={components} grid={p.grid}")
    s = _setup(psl, p, "f32" if mode == "mixed" else "f64", components)
    x, st = _solve(psl, s, dev(p.q), solver, mode)
    xg = host(x)
    del s
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    label_fn = O.levelset_components if components else O.levelset_labels
    _, d = label_fn(p.grid, p.K, p.nsub, p.thr)
    rel = O.relres(A, b, xg)
    say(f"  status={st['status_str']} iters={st['iters']} d={d} relres={rel:.2e} "
        f"(device {st['relres_true']:.2e})")
    assert st["status"] == 0 and rel <= 1e-8
    assert abs(rel - st["relres_true"]) <= 1e-3 * rel + 1e-15
