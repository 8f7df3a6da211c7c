"""Batched solve (many independent systems per launch) on the GPU: every system's float64
answer is the single-system float64 answer bit for bit, the mixed-precision answers meet
the oracle's accuracy bar and do not depend on the rest of the batch, and the per-system
failure paths stay per system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import psl_inputs as pi
from oracle import psl_oracle as O

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _setup_all(problems):
    import torch
    from paper_1510_02148_amd import pipeline
    setups, bs = [], []
    for p in problems:
        K = torch.as_tensor(p.K, dtype=torch.float64, device="cuda")
        setups.append(pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr)))
        bs.append(torch.as_tensor(p.q, dtype=torch.float64, device="cuda"))
    return setups, bs


def _small_batch(nsys=6, seed=3):
    # uneven cubes (sides 12..28) with the full-size recipe otherwise
    return pi.batch(nsys=nsys, side_lo=12, side_hi=28, seed=seed)


def test_batched_equals_single_bitwise(gpu_lib):
    psl = gpu_lib
    probs = _small_batch()
    say("batched vs single, sides " + ",".join(str(p.grid[0]) for p in probs))
    setups, bs = _setup_all(probs)
    xs, stats, rc = psl.psl_solve_batched([s.ctx for s in setups], bs)
    assert rc == 0, [s["status_str"] for s in stats]
    for p, s, b, xb, stb in zip(probs, setups, bs, xs, stats):
        x1, st1 = psl.psl_solve(s.ctx, b, mode=psl.FP64)
        assert st1["status"] == 0
        assert stb["iters"] == st1["iters"], (stb["iters"], st1["iters"])
        assert np.array_equal(xb.cpu().numpy(), x1.cpu().numpy())
        assert stb["relres_true"] == st1["relres_true"]


def test_batched_matches_oracle(gpu_lib):
    psl = gpu_lib
    probs = _small_batch(nsys=8, seed=11)
    setups, bs = _setup_all(probs)
    xs, stats, rc = psl.psl_solve_batched([s.ctx for s in setups], bs)
    assert rc == 0
    for p, xg, st in zip(probs, xs, stats):
        A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
        xh = xg.cpu().numpy()
        res = O.relres(A, b, xh)
        xr = spla.spsolve(A.tocsc(), b)
        err = np.linalg.norm(xh - xr) / np.linalg.norm(xr)
        ref = O.dpcg(A, b, O.deflation_matrix(*O.levelset_labels(p.grid, p.K, p.nsub, p.thr)),
                     tol=1e-8)
        say(f"  side {p.grid[0]} c={p.meta.get('contrast', 0):.1e} iters {st['iters']} "
            f"(oracle {ref.iters}) relres {res:.2e} err {err:.2e}")
        assert res <= 1e-8 and st["relres_true"] <= 1e-8
        assert err <= 1e-6
        assert abs(st["iters"] - ref.iters) <= max(2, 0.02 * ref.iters)


def test_batched_repeat_reuses_plan_and_x0(gpu_lib):
    """A second call on the same contexts reuses the cached plan; starting from the
    converged solutions finishes without CG iterations; a different order rebuilds it."""
    psl = gpu_lib
    probs = _small_batch(nsys=4, seed=5)
    setups, bs = _setup_all(probs)
    ctxs = [s.ctx for s in setups]
    xs, st1, rc = psl.psl_solve_batched(ctxs, bs)
    assert rc == 0
    xs2, st2, rc2 = psl.psl_solve_batched(ctxs, bs, xs=[x.clone() for x in xs], use_x0=True)
    assert rc2 == 0 and all(s["iters"] == 0 for s in st2)
    xs3, st3, rc3 = psl.psl_solve_batched(ctxs[::-1], bs[::-1])
    assert rc3 == 0
    for a, b3 in zip(xs, xs3[::-1]):
        assert np.array_equal(a.cpu().numpy(), b3.cpu().numpy())


def test_batched_per_system_outcomes(gpu_lib):
    """A zero right-hand side, a non-finite one and ordinary systems in one batch: each
    gets its own status; the others are unaffected."""
    import torch
    psl = gpu_lib
    probs = _small_batch(nsys=4, seed=7)
    setups, bs = _setup_all(probs)
    bs[1] = torch.zeros_like(bs[1])
    bs[2] = bs[2].clone()
    bs[2][5] = float("nan")
    xs, stats, rc = psl.psl_solve_batched([s.ctx for s in setups], bs)
    say("statuses " + ",".join(s["status_str"] for s in stats))
    assert rc == psl.ENONFINITE
    assert stats[1]["status"] == 0 and float(xs[1].abs().max()) == 0.0
    assert stats[2]["status"] == psl.ENONFINITE
    for i in (0, 3):
        assert stats[i]["status"] == 0 and stats[i]["relres_true"] <= 1e-8


def test_batched_argument_errors(gpu_lib):
    psl = gpu_lib
    probs = _small_batch(nsys=2, seed=9)
    setups, bs = _setup_all(probs)
    with pytest.raises(psl.PslError) as e:
        psl.psl_solve_batched([setups[0].ctx, setups[0].ctx], [bs[0], bs[0]], check=True)
    assert e.value.status == psl.EINVAL
    o = psl.default_opts()
    o.mode = psl.MIXED
    import ctypes
    handles = (ctypes.c_void_p * 2)(*[s.ctx.handle.value for s in setups])
    bp = (ctypes.c_void_p * 2)(*[b.data_ptr() for b in bs])
    xs = [b.clone() for b in bs]
    xp = (ctypes.c_void_p * 2)(*[x.data_ptr() for x in xs])
    st = (psl.psl_solve_stats * 2)()
    o.tau_inner = 1.5                  # out of (0, 1)
    assert psl._solve_batched(handles, 2, bp, xp, ctypes.byref(o), st, None) == psl.EINVAL
    o.tau_inner = 0.01
    o.mode = 7
    assert psl._solve_batched(handles, 2, bp, xp, ctypes.byref(o), st, None) == psl.EINVAL


def test_batched_mixed_matches_oracle(gpu_lib):
    """PSL_MIXED batched: float32 refinement steps for all systems together, float64 to
    finish. Every x meets 1e-8 in the oracle's matrix and 1e-6 against a direct solve,
    and its float64 residual is the library's own figure."""
    psl = gpu_lib
    probs = _small_batch(nsys=8, seed=11)
    setups, bs = _setup_all(probs)
    xs, stats, rc = psl.psl_solve_batched([s.ctx for s in setups], bs, mode=psl.MIXED)
    assert rc == 0, [s["status_str"] for s in stats]
    for p, s, b, xg, st in zip(probs, setups, bs, xs, stats):
        A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
        xh = xg.cpu().numpy()
        res = O.relres(A, bh, xh)
        xr = spla.spsolve(A.tocsc(), bh)
        err = np.linalg.norm(xh - xr) / np.linalg.norm(xr)
        x1, st1 = psl.psl_solve(s.ctx, b, mode=psl.MIXED)
        say(f"  side {p.grid[0]} c={p.meta.get('contrast', 0):.1e} mixed batched: iters "
            f"{st['iters']} outer {st['outer']} fell_back {st['fell_back']} relres {res:.2e} "
            f"err {err:.2e} (single mixed: iters {st1['iters']} outer {st1['outer']})")
        assert st["status"] == 0 and res <= 1e-8 and st["relres_true"] <= 1e-8
        assert abs(st["relres_true"] - res) <= 2e-2 * res + 1e-12
        assert err <= 1e-6
        assert st["outer"] >= 1


def test_batched_mixed_independent_of_batch(gpu_lib):
    """In PSL_MIXED each system's arithmetic is its own (per-system scalars and step
    decisions, fixed-order sums): its x does not depend on the other systems of the batch,
    on their order, or on a repeat of the call (bit for bit)."""
    psl = gpu_lib
    probs = _small_batch(nsys=5, seed=13)
    setups, bs = _setup_all(probs)
    ctxs = [s.ctx for s in setups]
    xs, st, rc = psl.psl_solve_batched(ctxs, bs, mode=psl.MIXED)
    assert rc == 0
    xs = [x.clone() for x in xs]
    xs2, st2, _ = psl.psl_solve_batched(ctxs, bs, mode=psl.MIXED)
    xs3, st3, _ = psl.psl_solve_batched(ctxs[::-1], bs[::-1], mode=psl.MIXED)
    say("mixed batched iterations " + ",".join(str(s["iters"]) for s in st))
    for i in range(len(probs)):
        xa, sa = psl.psl_solve_batched([ctxs[i]], [bs[i]], mode=psl.MIXED)[:2]
        assert np.array_equal(xs[i].cpu().numpy(), xs2[i].cpu().numpy())
        assert np.array_equal(xs[i].cpu().numpy(), xs3[len(probs) - 1 - i].cpu().numpy())
        assert np.array_equal(xs[i].cpu().numpy(), xa[0].cpu().numpy())
        assert st[i]["iters"] == st2[i]["iters"] == sa[0]["iters"]
