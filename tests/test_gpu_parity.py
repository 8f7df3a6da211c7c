"""HIP path vs the CPU float64 oracle, element by element, through the C-ABI.

Bars: integer labels bit-exact; float64 transmissibilities within 1 ulp; operator products
within a few ulps of |A||p|; solves reach ||b - A x|| / ||b|| <= 1e-8 (residual computed
by the oracle's own matrix from the GPU x) and ||x - x_ref|| / ||x_ref|| <= 1e-6 with
x_ref a direct solve (small) or the oracle at tol 1e-12.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import psl_inputs as pi
from oracle import psl_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dev(a, dtype=None):
    dtype = torch.float64 if dtype is None else dtype
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def lognormal(n, seed, sigma=2.0):
    return np.exp(sigma * np.random.Generator(np.random.PCG64(seed)).standard_normal(n))


# ------------------------------------------------------------------ transmissibilities

TPFA_CASES = [((5, 4, 3), 63), ((64, 64, 1), 1), ((37, 29, 11), 1 | 32), ((1, 1, 1), 63),
              ((128, 1, 1), 3), ((16, 9, 70), 4 | 8 | 16)]


@pytest.mark.parametrize("grid,mask", TPFA_CASES)
def test_tpfa_matches_oracle(gpu_lib, grid, mask):
    psl = gpu_lib
    say(f"tpfa grid={grid} mask={mask}")
    n = grid[0] * grid[1] * grid[2]
    K = lognormal(n, 1 + n)
    K[::11] = 0.0                      # impermeable cells: faces between two of them are 0
    Tx, Ty, Tz = psl.psl_assemble_tpfa(grid, dev(K), mask)
    rx, ry, rz = O.transmissibilities(K, grid, mask)
    for got, ref in ((Tx, rx), (Ty, ry), (Tz, rz)):
        g = host(got)
        ulp = np.abs(g - ref) / np.maximum(np.spacing(np.abs(ref)), np.finfo(float).tiny)
        assert np.all(ulp <= 1.0), f"max ulp {ulp.max()}"


# ------------------------------------------------------------------ labels

LABEL_CASES = [
    ((7, 5, 3), (3, 2, 2), [0.1, 1.0]),
    ((9, 4, 1), (4, 3, 1), [1.0]),
    ((37, 29, 11), (5, 3, 2), [0.05, 0.5, 5.0]),
    ((64, 64, 1), (4, 4, 1), [1e-2]),
    ((40, 40, 40), (1, 1, 1), [1.0]),
    ((33, 17, 9), (33, 17, 9), []),
]


@pytest.mark.parametrize("grid,nsub,thr", LABEL_CASES)
def test_labels_bit_exact(gpu_lib, grid, nsub, thr):
    psl = gpu_lib
    say(f"labels grid={grid} nsub={nsub} thr={thr}")
    n = grid[0] * grid[1] * grid[2]
    K = lognormal(n, 7 + n)
    if thr:
        K[::5] = thr[0]                 # ties on a threshold go to the upper class
    lab, d = psl.psl_build_Z(grid, dev(K), nsub, thr)
    ref, dref = O.levelset_labels(grid, K, nsub, np.array(thr))
    assert d == dref
    assert np.array_equal(host(lab), ref)


def test_labels_manual_classes(gpu_lib):
    psl = gpu_lib
    say("labels manual classes")
    grid = (21, 13, 8)
    n = 21 * 13 * 8
    cls = np.random.Generator(np.random.PCG64(3)).integers(0, 4, size=n).astype(np.int32)
    lab, d = psl.psl_build_Z(grid, None, (3, 2, 2), cls=dev(cls, torch.int32), ncls=4)
    ref, dref = O.levelset_labels(grid, None, (3, 2, 2), None, cls=cls, ncls=4)
    assert d == dref and np.array_equal(host(lab), ref)


@pytest.mark.parametrize("components", [False, True], ids=["regions", "components"])
@pytest.mark.parametrize("bad", [4, -1, 7], ids=["ncls", "negative", "above"])
def test_manual_class_out_of_range_rejected(gpu_lib, components, bad):
    """A manual class outside [0, ncls) gives PSL_EINVAL, also in the first subdomain,
    where the key s * ncls + class would otherwise alias a key of the next subdomain."""
    psl = gpu_lib
    say(f"manual class {bad} with ncls=4 components={components}")
    grid = (21, 13, 8)
    n = 21 * 13 * 8
    cls = np.random.Generator(np.random.PCG64(3)).integers(0, 4, size=n).astype(np.int32)
    cls[5] = bad                     # cell 5 lies in subdomain 0 of the 3x2x2 partition
    with pytest.raises(psl.PslError) as ei:
        psl.psl_build_Z(grid, None, (3, 2, 2), cls=dev(cls, torch.int32), ncls=4,
                        components=components)
    assert ei.value.status == psl.EINVAL


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_labels_full_size(gpu_lib, name):
    psl = gpu_lib
    p = pi.config(name)
    say(f"labels full size {name} grid={p.grid}")
    lab, d = psl.psl_build_Z(p.grid, dev(p.K), p.nsub, list(p.thr))
    ref, dref = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    assert d == dref and np.array_equal(host(lab), ref)
    if name == "c2":
        assert d == 512 and np.all(np.bincount(ref) == 2048)


# connected components (psl_build_Z_cc)

@pytest.mark.parametrize("grid,nsub,thr", LABEL_CASES)
def test_components_bit_exact(gpu_lib, grid, nsub, thr):
    """Union-find labels equal the oracle's connected components exactly, and two runs
    give the same array (the result does not depend on how the atomics interleave)."""
    psl = gpu_lib
    say(f"components grid={grid} nsub={nsub} thr={thr}")
    n = grid[0] * grid[1] * grid[2]
    K = lognormal(n, 11 + n)
    lab, d = psl.psl_build_Z(grid, dev(K), nsub, thr, components=True)
    lab2, d2 = psl.psl_build_Z(grid, dev(K), nsub, thr, components=True)
    ref, dref = O.levelset_components(grid, K, nsub, np.array(thr))
    assert d == dref and np.array_equal(host(lab), ref)
    assert d2 == d and torch.equal(lab, lab2)


def test_components_manual_classes(gpu_lib):
    psl = gpu_lib
    say("components manual classes")
    grid = (21, 13, 8)
    n = 21 * 13 * 8
    cls = np.random.Generator(np.random.PCG64(5)).integers(0, 3, size=n).astype(np.int32)
    lab, d = psl.psl_build_Z(grid, None, (3, 2, 2), cls=dev(cls, torch.int32), ncls=3,
                             components=True)
    ref, dref = O.levelset_components(grid, None, (3, 2, 2), None, cls=cls, ncls=3)
    assert d == dref and np.array_equal(host(lab), ref)


@pytest.mark.parametrize("contrast", [1e4, 1e6])
def test_components_full_size(gpu_lib, contrast):
    """256x256x128 channelized field (8.4 M cells): channels cut into pieces inside many
    subdomains, so the components outnumber the regions."""
    psl = gpu_lib
    p = pi.config("c3", contrast=contrast)
    say(f"components full size c3 contrast {contrast:g}")
    Kd = dev(p.K)
    lab, d = psl.psl_build_Z(p.grid, Kd, p.nsub, list(p.thr), components=True)
    ref, dref = O.levelset_components(p.grid, p.K, p.nsub, p.thr)
    _, dplain = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    assert d == dref and np.array_equal(host(lab), ref)
    assert d > dplain
    for _ in range(3):   # millions of racing unions: the same array every time
        again, d2 = psl.psl_build_Z(p.grid, Kd, p.nsub, list(p.thr), components=True)
        assert d2 == d and torch.equal(again, lab)


def test_components_solve(gpu_lib):
    """The whole path on component labels: same x as the oracle's DEF1-PCG with the same
    deflation space, and about its iteration count."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = pi.channelized(48, 40, 24, contrast=1e5, corr_len=6.0, nsub=(6, 5, 3), seed=8)
    say("components solve chan 48x40x24")
    s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr), components=True)
    x, st = psl.psl_solve(s.ctx, dev(p.q), tol=1e-8)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_components(p.grid, p.K, p.nsub, p.thr)
    assert d == s.d
    Z = O.deflation_matrix(lab, d)
    ref = O.dpcg(A, b, Z, tol=1e-8)
    xr = O.dpcg(A, b, Z, tol=1e-12).x
    assert st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8
    assert np.linalg.norm(host(x) - xr) / np.linalg.norm(xr) <= 1e-6
    assert abs(st["iters"] - ref.iters) <= max(2, 0.02 * ref.iters)


# deflated GMRES (psl_solve_gmres)

GMRES_CASES = [("c1", 1, 30, False, 0), ("c2", 4, 30, False, 0), ("chan", 0, 100, False, 0),
               ("chan", 0, 30, True, 0), ("c2", 4, 30, False, 3), ("chan", 0, 30, True, 3),
               ("chan", 0, 30, False, 3), ("c1", 1, 10, False, 2)]


@pytest.mark.parametrize("name,scale,m,comp,degree", GMRES_CASES,
                         ids=[f"{c[0]}/{c[1]}-m{c[2]}{'-components' if c[3] else ''}"
                              f"{'-cheb%d' % c[4] if c[4] else ''}" for c in GMRES_CASES])
def test_gmres_parity(gpu_lib, name, scale, m, comp, degree):
    """The paper's deflated GMRES(m) on the GPU against the oracle's: same solution, a
    1e-8 true residual, and about the oracle's step count (classical Gram-Schmidt twice on
    the GPU, modified Gram-Schmidt in the oracle). On the contrast-1e6 channel field
    GMRES(30) stagnates with one vector per region (as the paper's GMRES(20) does on its
    sandwich case), so that case runs GMRES(100), and GMRES(30) with component vectors.
    degree >= 2: the Chebyshev polynomial preconditioner in place of diag(A)."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _op_problem(name, scale)
    say(f"gmres {name}/{scale} grid={p.grid} m={m} components={comp} degree={degree}")
    s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr), components=comp)
    x, st = psl.psl_solve_gmres(s.ctx, dev(p.q), restart=m, degree=degree)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    labels = O.levelset_components if comp else O.levelset_labels
    lab, d = labels(p.grid, p.K, p.nsub, p.thr)
    Z = O.deflation_matrix(lab, d)
    ref = O.pdgmres(A, b, Z, m=m, tol=1e-8, degree=degree, ratio=30.0)
    xr = O.dpcg(A, b, Z, tol=1e-12).x
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.iters}) cycles={st['outer']}")
    assert st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8
    assert st["relres_true"] <= 1e-8
    assert np.linalg.norm(host(x) - xr) / np.linalg.norm(xr) <= 1e-6
    assert abs(st["iters"] - ref.iters) <= max(3, 0.05 * ref.iters)


def test_gmres_restarts_cap_and_zero_rhs(gpu_lib):
    """Short and long cycles both converge (short ones take more steps); the step cap
    returns PSL_EMAXIT after exactly that many steps with the projected iterate; b = 0
    gives x = 0; restart lengths outside 1..200 are rejected."""
    psl = gpu_lib
    p = pi.config("c2", scale=4)
    s = _setup(psl, p)
    b = dev(p.q)
    _, st5 = psl.psl_solve_gmres(s.ctx, b, restart=5)
    _, st60 = psl.psl_solve_gmres(s.ctx, b, restart=60)
    assert st5["status"] == 0 and st60["status"] == 0
    assert st5["relres_true"] <= 1e-8 and st60["relres_true"] <= 1e-8
    assert st5["iters"] >= st60["iters"]
    _, stc = psl.psl_solve_gmres(s.ctx, b, restart=30, maxit=7)
    assert stc["status"] == psl.EMAXIT and stc["iters"] == 7 and stc["relres_true"] > 1e-8
    x0, st0 = psl.psl_solve_gmres(s.ctx, torch.zeros_like(b))
    assert st0["status"] == 0 and torch.count_nonzero(x0) == 0
    for bad in (0, 201):
        _, stb = psl.psl_solve_gmres(s.ctx, b, restart=bad)
        assert stb["status_str"] == psl.psl_status_str(psl.EINVAL)
    for bad in (-1, 17):
        _, stb = psl.psl_solve_gmres(s.ctx, b, degree=bad)
        assert stb["status_str"] == psl.psl_status_str(psl.EINVAL)


# deflated CG with the Chebyshev polynomial preconditioner (psl_solve_poly)

POLY_CASES = [("c1", 1, 2, 8.0, False), ("c2", 4, 1, 8.0, False), ("c2", 4, 2, 8.0, False),
              ("c2", 4, 3, 30.0, False), ("chan", 0, 2, 8.0, False), ("chan", 0, 5, 4.0, False),
              ("chan", 0, 2, 8.0, True)]


@pytest.mark.parametrize("name,scale,degree,ratio,comp", POLY_CASES,
                         ids=[f"{c[0]}/{c[1]}-deg{c[2]}-ratio{c[3]:g}{'-comp' if c[4] else ''}"
                              for c in POLY_CASES])
def test_poly_parity(gpu_lib, name, scale, degree, ratio, comp):
    """The polynomial-preconditioned deflated CG against the oracle's: the same solution
    (x_ref = the oracle's Jacobi DPCG at 1e-12), a 1e-8 true residual, and the oracle's
    iteration count for the same degree and interval (degree 1: Jacobi's)."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _op_problem(name, scale)
    say(f"poly {name}/{scale} grid={p.grid} degree={degree} ratio={ratio} components={comp}")
    s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr), components=comp)
    x, st = psl.psl_solve_poly(s.ctx, dev(p.q), degree=degree, ratio=ratio)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    labels = O.levelset_components if comp else O.levelset_labels
    lab, d = labels(p.grid, p.K, p.nsub, p.thr)
    Z = O.deflation_matrix(lab, d)
    co = O.Coarse(A, Z)
    ref = O.dpcg_poly(A, b, Z, degree=degree, ratio=ratio, tol=1e-8, coarse=co)
    xr = O.dpcg(A, b, Z, tol=1e-12, coarse=co).x
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.iters})")
    assert st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8
    assert st["relres_true"] <= 1e-8
    assert np.linalg.norm(host(x) - xr) / np.linalg.norm(xr) <= 1e-6
    assert abs(st["iters"] - ref.iters) <= max(2, 0.03 * ref.iters)
    if degree == 1:
        assert abs(st["iters"] - O.dpcg(A, b, Z, tol=1e-8, coarse=co).iters) <= 2


POLY_MIXED_CASES = [("c1", 1, False), ("c2", 4, False), ("chan", 0, False), ("chan", 0, True)]


@pytest.mark.parametrize("name,scale,comp", POLY_MIXED_CASES,
                         ids=[f"{c[0]}/{c[1]}{'-comp' if c[2] else ''}" for c in POLY_MIXED_CASES])
def test_poly_mixed(gpu_lib, name, scale, comp):
    """The polynomial-preconditioned CG in float32 inside float64 refinement: the oracle's
    accuracy bar (1e-8 true residual in the oracle's matrix, 1e-6 against the 1e-12
    solution) and at most twice the float64 solve's iterations."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _op_problem(name, scale)
    say(f"poly mixed {name}/{scale} grid={p.grid} components={comp}")
    s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr), components=comp)
    x, st = psl.psl_solve_poly(s.ctx, dev(p.q), mixed=True)
    _, st64 = psl.psl_solve_poly(s.ctx, dev(p.q))
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    labels = O.levelset_components if comp else O.levelset_labels
    lab, d = labels(p.grid, p.K, p.nsub, p.thr)
    xr = O.dpcg(A, b, O.deflation_matrix(lab, d), tol=1e-12).x
    say(f"  status={st['status_str']} iters={st['iters']} outer={st['outer']} "
        f"(float64 {st64['iters']})")
    assert st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8 and st["relres_true"] <= 1e-8
    assert np.linalg.norm(host(x) - xr) / np.linalg.norm(xr) <= 1e-6
    assert st["outer"] >= 1 and st["iters"] <= 2 * st64["iters"]


def test_poly_result_independent_of_host_checks(gpu_lib):
    """The host's read interval only changes how many launches run after the stop flag
    (as no-ops): x and the iteration count are bit-identical for 1, 16 and 512."""
    psl = gpu_lib
    p = pi.config("c2", scale=4)
    say("poly host-check independence c2/4")
    s = _setup(psl, p)
    b = dev(p.q)
    runs = [psl.psl_solve_poly(s.ctx, b, check_every=k) for k in (1, 16, 512)]
    for x, st in runs:
        assert st["status"] == 0
    for x, st in runs[1:]:
        assert torch.equal(x, runs[0][0]) and st["iters"] == runs[0][1]["iters"]


def test_poly_cap_zero_rhs_start_and_invalid(gpu_lib):
    """The iteration cap returns PSL_EMAXIT after exactly that many iterations with the
    projected iterate; b = 0 gives x = 0; a start vector gives the same solution; options
    out of range are rejected."""
    psl = gpu_lib
    p = pi.config("c2", scale=4)
    say("poly cap / zero rhs / x0 / invalid c2/4")
    s = _setup(psl, p)
    b = dev(p.q)
    x, st = psl.psl_solve_poly(s.ctx, b)
    assert st["status"] == 0
    _, stc = psl.psl_solve_poly(s.ctx, b, maxit=5)
    assert stc["status"] == psl.EMAXIT and stc["iters"] == 5 and stc["relres_true"] > 1e-8
    x0, st0 = psl.psl_solve_poly(s.ctx, torch.zeros_like(b))
    assert st0["status"] == 0 and torch.count_nonzero(x0) == 0
    xs = x + 1e-3 * torch.randn_like(x)
    xw, stw = psl.psl_solve_poly(s.ctx, b, xs.clone(), use_x0=True)
    assert stw["status"] == 0 and stw["iters"] < st["iters"]
    assert torch.linalg.norm(xw - x) / torch.linalg.norm(x) <= 1e-6
    for kw in ({"degree": 0}, {"degree": 17}, {"ratio": 1.0}, {"lmax": 0.0},
               {"check_every": 0}, {"check_every": 513}):
        _, stb = psl.psl_solve_poly(s.ctx, b, **kw)
        assert stb["status_str"] == psl.psl_status_str(psl.EINVAL), kw


def test_poly_below_the_rounding_floor(gpu_lib):
    """A tolerance under the float64 rounding floor: once the deflated residual has reached
    the floor (about 1e-14 relative here) the CG recursion loses it again and ends with a
    breakdown, in the oracle as on the GPU, at about the same step. The GPU call returns
    (PSL_EBREAKDOWN, or PSL_ESTAGNATION when the residual only stalls) instead of running
    to the iteration cap."""
    psl = gpu_lib
    p = pi.config("c2", scale=4)
    say("poly below the floor c2/4 tol 1e-18")
    s = _setup(psl, p)
    x, st = psl.psl_solve_poly(s.ctx, dev(p.q), tol=1e-18)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    ref = O.dpcg_poly(A, b, O.deflation_matrix(lab, d), degree=3, ratio=30.0, tol=1e-18,
                      maxit=2000)
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.status} {ref.iters})")
    assert st["status"] in (psl.ESTAGNATION, psl.EBREAKDOWN) and st["iters"] < 2000
    if ref.status == "breakdown":
        assert st["status"] == psl.EBREAKDOWN and abs(st["iters"] - ref.iters) <= 5
    assert np.isfinite(host(x)).all()


def test_poly_full_size(gpu_lib):
    """128x128x64 layered (the benchmark workload) with the default degree 3 on [2/30, 2]:
    the oracle's residual of the GPU x, and the oracle's iteration count."""
    psl = gpu_lib
    p = pi.config("c2")
    say(f"poly full size c2 grid={p.grid}")
    s = _setup(psl, p)
    x, st = psl.psl_solve_poly(s.ctx, dev(p.q), degree=3, ratio=30.0)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    Z = O.deflation_matrix(lab, d)
    ref = O.dpcg_poly(A, b, Z, degree=3, ratio=30.0, tol=1e-8)
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.iters})")
    assert st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8
    assert abs(st["iters"] - ref.iters) <= max(2, 0.03 * ref.iters)
    assert np.linalg.norm(host(x) - ref.x) / np.linalg.norm(ref.x) <= 1e-6


# ------------------------------------------------------------------ operators

def _setup(psl, p):
    from paper_1510_02148_amd import pipeline
    return pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr))


OP_CASES = [("c1", 1), ("c2", 4), ("chan", 0)]


def _op_problem(name, scale):
    if name == "chan":
        return pi.channelized(48, 40, 24, contrast=1e6, corr_len=6.0, nsub=(6, 5, 3), seed=8)
    if name == "chan2":
        return pi.channelized(64, 48, 32, contrast=1e4, corr_len=6.0, nsub=(8, 6, 3), seed=9)
    if name == "chan3":
        return pi.channelized(96, 80, 48, contrast=1e4, corr_len=6.0, nsub=(16, 10, 6), seed=10)
    return pi.config(name, scale=scale)


@pytest.mark.parametrize("name,scale", OP_CASES)
def test_apply_A(gpu_lib, name, scale):
    psl = gpu_lib
    p = _op_problem(name, scale)
    say(f"apply_A {name}/{scale} grid={p.grid}")
    s = _setup(psl, p)
    A, _ = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    pv = np.random.Generator(np.random.PCG64(5)).standard_normal(p.n)
    q = host(psl.psl_apply_A(s.ctx, dev(pv)))
    ref = A @ pv
    bound = 1e-13 * (abs(A) @ np.abs(pv)) + 1e-300
    assert np.all(np.abs(q - ref) <= bound)


@pytest.mark.parametrize("name,scale", OP_CASES + [("chan2", 0), ("chan3", 0)])
def test_coarse_matrix_and_inverse(gpu_lib, name, scale):
    """E against the oracle's Z^T A Z, and E^-1 E = I to within the conditioning; the
    cases span one to ~30 64-wide blocks of the blocked factor and inverse (block
    diagonals longer than eight blocks take the split two-launch form), with and without a
    ragged last block."""
    psl = gpu_lib
    p = _op_problem(name, scale)
    say(f"coarse E {name}/{scale}")
    s = _setup(psl, p)
    A, _ = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    Eref = O.coarse_matrix(A, O.deflation_matrix(lab, d))
    E, Einv = psl.psl_get_coarse(s.ctx)
    E, Einv = host(E), host(Einv)
    scale_rows = np.abs(Eref).sum(1)[:, None]
    assert np.max(np.abs(E - Eref) / scale_rows) <= 1e-13
    cond = np.linalg.cond(Eref)
    err = np.linalg.norm(Einv @ Eref - np.eye(d), 2)
    assert err <= max(1e-12, 2e-12 * cond), (err, cond)
    assert np.array_equal(Einv, Einv.T)   # the Gram product writes both triangles


@pytest.mark.parametrize("name,scale", OP_CASES)
def test_deflate_projector(gpu_lib, name, scale):
    psl = gpu_lib
    p = _op_problem(name, scale)
    say(f"deflate P1 {name}/{scale}")
    s = _setup(psl, p)
    A, _ = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    Z = O.deflation_matrix(lab, d)
    C = O.Coarse(A, Z)
    r = np.random.Generator(np.random.PCG64(9)).standard_normal(p.n)
    out, cvec = psl.psl_deflate(s.ctx, dev(r))
    out, cvec = host(out), host(cvec)
    cref = C.solve(Z.T @ r)
    ref = r - A @ (Z @ cref)
    cond = np.linalg.cond(C.E)
    assert np.linalg.norm(cvec - cref) <= 1e-13 * cond * np.linalg.norm(cref)
    assert np.linalg.norm(out - ref) <= 1e-9 * np.linalg.norm(r)
    # Z^T P1 = 0
    assert np.linalg.norm(Z.T @ out) <= 1e-8 * np.linalg.norm(Z.T @ r)


# ------------------------------------------------------------------ solves

def _reference_x(A, b, n):
    if n <= 40000:
        return spla.spsolve(A.tocsc(), b)
    return None


SOLVE_CASES = [
    ("c1", 1, {}),
    ("c2", 4, {}),
    ("c2", 2, {}),
    ("c3", 4, {"contrast": 1e5}),
    ("ragged", 0, {}),
]


def _problem(name, scale, kw):
    if name == "ragged":
        return pi.layered3d(37, 29, 11, nlayers=4, contrast=1e4, nsub=(5, 3, 2), seed=21,
                            wells="columns")
    return pi.config(name, scale=scale, **kw)


@pytest.mark.parametrize("mode", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,scale,kw", SOLVE_CASES, ids=[f"{c[0]}-{c[1]}" for c in SOLVE_CASES])
def test_solve_parity(gpu_lib, name, scale, kw, mode):
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _problem(name, scale, kw)
    say(f"solve {name}/{scale} grid={p.grid} mode={mode}")
    x, st, s = pipeline.solve_problem(p, mode=mode)
    xg = host(x)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    res = O.relres(A, b, xg)
    ref = O.dpcg(A, b, O.deflation_matrix(*O.levelset_labels(p.grid, p.K, p.nsub, p.thr)),
                 tol=1e-8)
    xr = _reference_x(A, b, p.n)
    if xr is None:
        xr = O.dpcg(A, b, O.deflation_matrix(*O.levelset_labels(p.grid, p.K, p.nsub, p.thr)),
                    tol=1e-12).x
    err = np.linalg.norm(xg - xr) / np.linalg.norm(xr)
    r = b - A @ xg
    drift_cpu = np.linalg.norm(O.deflation_matrix(
        *O.levelset_labels(p.grid, p.K, p.nsub, p.thr)).T @ r) / np.linalg.norm(r)
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.iters}) outer={st['outer']}"
        f" relres={res:.2e} (lib {st['relres_true']:.2e}) err={err:.2e} "
        f"zt_r_drift={st['zt_r_drift']:.2e} (of the same x on the CPU {drift_cpu:.2e})")
    # Z^T r of the returned x is rounding-level (both sides compute it from a residual
    # that is itself ~1e-8 of b): the same order as the CPU's figure for the same x
    assert 0.0 <= st["zt_r_drift"] <= max(1e-4, 10.0 * drift_cpu)
    assert st["status"] == 0
    assert res <= 1e-8 and st["relres_true"] <= 1e-8
    assert abs(st["relres_true"] - res) <= 2e-2 * res + 1e-12
    assert err <= 1e-6
    if mode == 0:
        assert abs(st["iters"] - ref.iters) <= max(2, 0.02 * ref.iters)


def test_solve_deterministic(gpu_lib):
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = pi.config("c2", scale=4)
    say("determinism c2/4")
    s = _setup(psl, p)
    b = dev(p.q)
    x1, st1 = psl.psl_solve(s.ctx, b)
    x2, st2 = psl.psl_solve(s.ctx, b)
    assert torch.equal(x1, x2) and st1["iters"] == st2["iters"]
    s2 = _setup(psl, p)
    x3, _ = psl.psl_solve(s2.ctx, b)
    assert torch.equal(x1, x3)


@pytest.mark.parametrize("name,scale", [("c2", 4), ("c2", 1)], ids=["graph-replay", "direct"])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_result_independent_of_host_checks(gpu_lib, name, scale, mode):
    """How many iterations the host enqueues between looks at the device (check_every, the
    rate-based tail, the first-enqueue estimate from an earlier solve) only changes how many
    launches exit at once: x and the iteration count are bit-identical. Covers the graph
    replay (small grids) and the direct launches (large grids)."""
    psl = gpu_lib
    p = pi.config(name, scale=scale)
    say(f"host-check independence {name}/{scale} {mode}")
    md = psl.FP64 if mode == "fp64" else psl.MIXED
    b = dev(p.q)
    runs = []
    # (check_every, fresh context): a reused context starts from its iteration history
    for check, fresh in ((2, True), (16, False), (64, True), (16, False)):
        if fresh:
            s = _setup(psl, p)
        x, st = psl.psl_solve(s.ctx, b, mode=md, check_every=check)
        assert st["status"] == 0
        runs.append((x, st["iters"], st["outer"]))
    for x, it, outer in runs[1:]:
        assert torch.equal(x, runs[0][0]) and it == runs[0][1] and outer == runs[0][2]


def test_x0_independence(gpu_lib):
    psl = gpu_lib
    p = pi.config("c2", scale=4)
    say("x0 independence c2/4")
    s = _setup(psl, p)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    g = np.random.Generator(np.random.PCG64(11))
    x0 = g.standard_normal(p.n) + (O.deflation_matrix(lab, d) @ (50 * g.standard_normal(d)))
    b = dev(p.q)
    xa, sa = psl.psl_solve(s.ctx, b, tol=1e-11)
    xb, sb = psl.psl_solve(s.ctx, b, dev(x0), use_x0=True, tol=1e-11)
    xa, xb = host(xa), host(xb)
    assert sa["status"] == 0 and sb["status"] == 0
    assert np.linalg.norm(xa - xb) / np.linalg.norm(xa) <= 1e-6


# ------------------------------------------------------------------ edge cases

def test_zero_rhs(gpu_lib):
    psl = gpu_lib
    p = pi.config("c1")
    say("edge b = 0")
    s = _setup(psl, p)
    x, st = psl.psl_solve(s.ctx, torch.zeros(p.n, dtype=torch.float64, device="cuda"))
    assert st["status"] == 0 and st["iters"] == 0 and torch.count_nonzero(x).item() == 0


def test_nonfinite_rhs(gpu_lib):
    psl = gpu_lib
    p = pi.config("c1")
    say("edge NaN in b")
    s = _setup(psl, p)
    b = p.q.copy()
    b[100] = np.nan
    _, st = psl.psl_solve(s.ctx, dev(b))
    assert st["status"] == psl.ENONFINITE


def test_maxit_returns_projected_iterate(gpu_lib):
    psl = gpu_lib
    p = pi.config("c1")
    say("edge maxit = 3")
    s = _setup(psl, p)
    x, st = psl.psl_solve(s.ctx, dev(p.q), maxit=3)
    assert st["status"] == psl.EMAXIT and st["iters"] == 3
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    ref = O.dpcg(A, b, O.deflation_matrix(lab, d), tol=1e-8, maxit=3)
    assert np.linalg.norm(host(x) - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_one_label_per_cell(gpu_lib):
    """d = n: E = A, the coarse solve alone is exact, no CG iteration is needed."""
    psl = gpu_lib
    say("edge d = n")
    grid = (6, 5, 4)
    n = 120
    K = lognormal(n, 31)
    Tx, Ty, Tz = psl.psl_assemble_tpfa(grid, dev(K), 1)
    labels = dev(np.arange(n, dtype=np.int32), torch.int32)
    ctx = psl.psl_setup_E(grid, Tx, Ty, Tz, labels, n)
    q = np.random.Generator(np.random.PCG64(2)).standard_normal(n)
    x, st = psl.psl_solve(ctx, dev(q))
    A, b = O.assemble(K, grid, 1, q)
    assert st["status"] == 0 and st["iters"] == 0
    xr = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(host(x) - xr) <= 1e-9 * np.linalg.norm(xr)


def test_single_cell_and_single_label(gpu_lib):
    psl = gpu_lib
    say("edge 1 cell; d = 1")
    grid = (1, 1, 1)
    Tx, Ty, Tz = psl.psl_assemble_tpfa(grid, dev([3.0]), 1)
    lab, d = psl.psl_build_Z(grid, dev([3.0]), (1, 1, 1), [])
    ctx = psl.psl_setup_E(grid, Tx, Ty, Tz, lab, d, nsub=(1, 1, 1))
    x, st = psl.psl_solve(ctx, dev([2.0]))
    assert st["status"] == 0 and abs(host(x)[0] - 2.0 / 6.0) <= 1e-15
    # one region for a whole 3D problem
    p = pi.layered3d(20, 12, 10, contrast=1e3, nsub=(1, 1, 1), seed=4)
    p.thr = np.array([])
    from paper_1510_02148_amd import pipeline
    x, st, s = pipeline.solve_problem(p)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    assert s.d == 1 and st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8


OTHER_SOLVERS = [("gmres", 0), ("gmres", 3), ("poly", 1), ("poly", 3)]


def _other_solve(psl, ctx, b, solver, degree, **kw):
    if solver == "gmres":
        return psl.psl_solve_gmres(ctx, b, degree=degree, **kw)
    return psl.psl_solve_poly(ctx, b, degree=degree, **kw)


@pytest.mark.parametrize("solver,degree", OTHER_SOLVERS,
                         ids=[f"{s}-deg{d}" for s, d in OTHER_SOLVERS])
def test_other_solvers_edge_cases(gpu_lib, solver, degree):
    """Deflated GMRES and the polynomial-preconditioned CG on the degenerate cases: d = n
    (E = A: the projection alone is exact, no step), one cell, one region for a whole 3D
    problem (d = 1), and a ragged grid (37x29x11, uneven subdomains) against the oracle's
    solver with the same options."""
    psl = gpu_lib
    say(f"edge cases {solver} degree {degree}")
    grid, n = (6, 5, 4), 120
    K = lognormal(n, 31)
    Tx, Ty, Tz = psl.psl_assemble_tpfa(grid, dev(K), 1)
    ctx = psl.psl_setup_E(grid, Tx, Ty, Tz, dev(np.arange(n, dtype=np.int32), torch.int32), n)
    q = np.random.Generator(np.random.PCG64(2)).standard_normal(n)
    x, st = _other_solve(psl, ctx, dev(q), solver, degree)
    A, b = O.assemble(K, grid, 1, q)
    xr = np.linalg.solve(A.toarray(), b)
    assert st["status"] == 0 and st["iters"] == 0
    assert np.linalg.norm(host(x) - xr) <= 1e-9 * np.linalg.norm(xr)
    # one cell
    g1 = (1, 1, 1)
    Tx, Ty, Tz = psl.psl_assemble_tpfa(g1, dev([3.0]), 1)
    lab, d = psl.psl_build_Z(g1, dev([3.0]), (1, 1, 1), [])
    ctx1 = psl.psl_setup_E(g1, Tx, Ty, Tz, lab, d, nsub=(1, 1, 1))
    x, st = _other_solve(psl, ctx1, dev([2.0]), solver, degree)
    assert st["status"] == 0 and abs(host(x)[0] - 2.0 / 6.0) <= 1e-15
    from paper_1510_02148_amd import pipeline
    # one region for a whole 3D problem
    p = pi.layered3d(20, 12, 10, contrast=1e3, nsub=(1, 1, 1), seed=4)
    p.thr = np.array([])
    s1 = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr))
    x, st = _other_solve(psl, s1.ctx, dev(p.q), solver, degree)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    assert s1.d == 1 and st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8
    # ragged grid against the oracle
    p = _problem("ragged", 0, {})
    s2 = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr))
    x, st = _other_solve(psl, s2.ctx, dev(p.q), solver, degree)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    Z = O.deflation_matrix(lab, d)
    if solver == "gmres":
        ref = O.pdgmres(A, b, Z, m=30, tol=1e-8, degree=degree, ratio=30.0)
    else:
        ref = O.dpcg_poly(A, b, Z, degree=degree, ratio=30.0, tol=1e-8)
    say(f"  ragged: status={st['status_str']} iters={st['iters']} (oracle {ref.iters})")
    assert st["status"] == 0 and O.relres(A, b, host(x)) <= 1e-8
    assert abs(st["iters"] - ref.iters) <= max(3, 0.05 * ref.iters)


def test_bench_kernel_ids_need_their_solver(gpu_lib):
    """The GMRES pass and the Chebyshev step can only be timed after a solve of that kind
    (and the Chebyshev step's float32 form after a mixed one); afterwards they run."""
    psl = gpu_lib
    say("bench kernel ids")
    s = _setup(psl, pi.config("c2", scale=4))
    for kid, mode in ((psl.KERNEL_GMRES_PASS, psl.FP64), (psl.KERNEL_POLY_STEP, psl.FP64),
                      (psl.KERNEL_POLY_STEP, psl.MIXED)):
        with pytest.raises(psl.PslError) as e:
            psl.psl_bench_kernel(s.ctx, kid, mode, 2)
        assert e.value.status == psl.EINVAL
    b = dev(pi.config("c2", scale=4).q)
    psl.psl_solve_gmres(s.ctx, b)
    psl.psl_solve_poly(s.ctx, b)
    psl.psl_bench_kernel(s.ctx, psl.KERNEL_GMRES_PASS, psl.FP64, 2)
    psl.psl_bench_kernel(s.ctx, psl.KERNEL_POLY_STEP, psl.FP64, 2)
    with pytest.raises(psl.PslError):
        psl.psl_bench_kernel(s.ctx, psl.KERNEL_POLY_STEP, psl.MIXED, 2)
    with pytest.raises(psl.PslError):
        psl.psl_bench_kernel(s.ctx, psl.KERNEL_GMRES_PASS, psl.MIXED, 2)
    psl.psl_solve_poly(s.ctx, b, mixed=True)
    psl.psl_bench_kernel(s.ctx, psl.KERNEL_POLY_STEP, psl.MIXED, 2)
    torch.cuda.synchronize()


def test_setup_errors(gpu_lib):
    psl = gpu_lib
    say("edge setup errors")
    grid = (8, 8, 2)
    n = 128
    K = lognormal(n, 41)
    Tx, Ty, Tz = psl.psl_assemble_tpfa(grid, dev(K), 1)
    bad = np.zeros(n, dtype=np.int32)
    bad[5] = 7                                   # label outside [0, d)
    with pytest.raises(psl.PslError) as e:
        psl.psl_setup_E(grid, Tx, Ty, Tz, dev(bad, torch.int32), 2)
    assert e.value.status == psl.EINVAL
    with pytest.raises(psl.PslError) as e:        # column 1 of Z is empty
        psl.psl_setup_E(grid, Tx, Ty, Tz, dev(np.zeros(n, np.int32), torch.int32), 2)
    assert e.value.status == psl.EINVAL
    K0 = K.copy()
    K0[:] = 1.0
    K0[40] = 0.0                                 # an isolated impermeable interior cell
    K0[[39, 41, 32, 48, 104]] = 0.0
    Tx0, Ty0, Tz0 = psl.psl_assemble_tpfa(grid, dev(K0), 1)
    with pytest.raises(psl.PslError) as e:
        psl.psl_setup_E(grid, Tx0, Ty0, Tz0, dev(np.zeros(n, np.int32), torch.int32), 1)
    assert e.value.status == psl.ENOTSPD


@pytest.mark.parametrize("mode", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("reproject", [0, 1])
def test_reprojection_option(gpu_lib, mode, reproject):
    """The fused re-projection (rhat <- P1 rhat every iteration) of the float64 loop
    changes rounding only; the float32 loop ignores the option (its residual is replaced
    by the projected float64 residual instead) and must converge either way."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = pi.config("c3", scale=4, contrast=1e6)
    say(f"reproject={reproject} mode={mode} c3/4 contrast 1e6")
    x, st, s = pipeline.solve_problem(p, mode=mode, reproject=reproject)
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    res = O.relres(A, b, host(x))
    ref = O.dpcg(A, b, O.deflation_matrix(*O.levelset_labels(p.grid, p.K, p.nsub, p.thr)),
                 tol=1e-8)
    say(f"  status={st['status_str']} iters={st['iters']} (oracle {ref.iters}) "
        f"outer={st['outer']} fell_back={st['fell_back']} relres={res:.2e}")
    assert st["status"] == 0 and res <= 1e-8
    if mode == 0:
        # without re-projection the float64 path follows the oracle's iteration; with it
        # the iterates differ by rounding-level projections
        slack = 0.02 if reproject == 0 else 0.05
        assert abs(st["iters"] - ref.iters) <= max(2, slack * ref.iters)


@pytest.mark.parametrize("floor,tau", [(0.0, None), (1e-7, None), (1e-6, None), (1e-4, 0.1),
                                       (0.5, None)],
                         ids=["stall", "1e-7", "1e-6", "1e-4-tau0.1", "at-once"])
def test_mixed_handover(gpu_lib, floor, tau):
    """Float32 CG with residual replacement hands over to float64 (continuing its search
    direction) at the floor, after its float64 residual detaches, or, with floor 0, only
    when it stalls; every route must end at the float64 accuracy of the plain solve."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = pi.config("c3", scale=4, contrast=1e7)
    say(f"mixed handover floor={floor} tau={tau} c3/4 contrast 1e7")
    A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    Z = O.deflation_matrix(*O.levelset_labels(p.grid, p.K, p.nsub, p.thr))
    xr = O.dpcg(A, b, Z, tol=1e-12).x
    # at contrast 1e7 a 1e-8 residual does not pin the solution to 1e-6 (the float64
    # oracle stopped at 1e-8 is off by ~1e-4 here): the errors at looser tolerances are
    # reported, and the 1e-6 error bar is held by the same solve at the first tolerance of
    # 1e-8 ... 1e-11 that reaches it (a smaller residual does not by itself remove the
    # smooth error component: the routes that keep float32 longest were still off by
    # ~2e-6 at 1e-10, the others reach ~1e-10 there)
    for tol in (1e-8, 1e-9, 1e-10, 1e-11):
        x, st, s = pipeline.solve_problem(p, mode=psl.MIXED, mixed_floor=floor, tau_inner=tau,
                                          tol=tol)
        res = O.relres(A, b, host(x))
        err = np.linalg.norm(host(x) - xr) / np.linalg.norm(xr)
        say(f"  tol={tol:g}: status={st['status_str']} iters={st['iters']} outer={st['outer']} "
            f"fell_back={st['fell_back']} relres={res:.2e} err={err:.2e}")
        assert st["status"] == 0 and res <= tol
        if floor == 0.5:
            assert st["fell_back"] == 1      # reached after the first float32 run
        if err <= 1e-6:
            break
    assert err <= 1e-6


@pytest.mark.parametrize("seed,tol", [(1033, 1e-9), (1071, 1e-9), (1071, 1e-8)])
def test_deep_tolerance_recovers(gpu_lib, seed, tol):
    """Channelized 128x128x64 instances (contrast ~5.6e5) on which the single-reduction
    float64 loop lost its accuracy below 1e-8 (one returned a residual of 4). The solve
    goes back to its best iterate and continues with the two-reduction loop; 1e-9 is at
    the edge of float64's attainable accuracy here (it ends within a few per cent of it,
    possibly with a stagnation or cap status), 1e-8 converges."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = pi.learned_x0_instance(seed)
    say(f"deep tolerance seed={seed} tol={tol} grid={p.grid}")
    x, st, s = pipeline.solve_problem(p, mode=psl.FP64, tol=tol)
    say(f"  status={st['status_str']} iters={st['iters']} outer={st['outer']} "
        f"relres={st['relres_true']:.2e}")
    assert st["relres_true"] <= 1.5 * tol
    if tol >= 1e-8:
        assert st["status"] == 0
    else:
        assert st["status"] in (0, psl.ESTAGNATION, psl.EMAXIT)


FINISH_CASES = [("c2", 4, {}), ("c3", 4, {"contrast": 1e5}), ("ragged", 0, {})]


@pytest.mark.parametrize("mode", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,scale,kw", FINISH_CASES,
                         ids=[f"{c[0]}-{c[1]}" for c in FINISH_CASES])
def test_finish_kernels(gpu_lib, name, scale, kw, mode):
    """Step decisions taken in the one-workgroup finish kernels (the large-grid
    configuration, forced on here for small grids) against the oracle, and against the
    same solve with every pass workgroup summing the partials itself: float64 (the
    single-reduction loop sums the same partials in the same order: identical x) and mixed
    (the update partials are grouped per tile instead of per capped workgroup: the same
    iteration count within one)."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _problem(name, scale, kw)
    say(f"finish kernels {name}/{scale} grid={p.grid} mode={mode}")
    K, b = dev(p.K), dev(p.q)
    out = {}
    for fk in (1, -1):
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr), finish_kernels=fk)
        x, st = psl.psl_solve(s.ctx, b, tol=1e-8, mode=mode)
        out[fk] = (x.clone(), st)
    A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    Z = O.deflation_matrix(*O.levelset_labels(p.grid, p.K, p.nsub, p.thr))
    ref = O.dpcg(A, bh, Z, tol=1e-8)
    xr = _reference_x(A, bh, p.n)
    if xr is None:
        xr = O.dpcg(A, bh, Z, tol=1e-12).x
    (x1, st1), (x0, st0) = out[1], out[-1]
    res = O.relres(A, bh, host(x1))
    err = np.linalg.norm(host(x1) - xr) / np.linalg.norm(xr)
    say(f"  finish kernels: status={st1['status_str']} iters={st1['iters']} outer={st1['outer']} "
        f"relres={res:.2e} err={err:.2e}; in the passes: iters={st0['iters']} "
        f"(oracle {ref.iters})")
    assert st1["status"] == 0 and res <= 1e-8 and err <= 1e-6
    if mode == 0:
        assert torch.equal(x1, x0) and st1["iters"] == st0["iters"]
        assert abs(st1["iters"] - ref.iters) <= max(2, 0.02 * ref.iters)
    else:
        assert abs(st1["iters"] - st0["iters"]) <= 1


SYM_CASES = [("c2", 4, {}, None), ("ragged", 0, {}, None),
             ("c3", 4, {"contrast": 1e5}, (16, 16, 12))]


@pytest.mark.parametrize("name,scale,kw,nsub", SYM_CASES,
                         ids=["c2-4", "ragged-0", "c3-4-d5115"])
def test_coarse_symmetric(gpu_lib, name, scale, kw, nsub):
    """The coarse product over the lower block triangle of the symmetric E^-1 (Def. 3.1;
    the large-d configuration, forced on here) against the dense row-wise product on the
    same context set-up, and both against the oracle: float64 (with and without the
    per-iteration re-projection, which takes the second right-hand side), mixed, the
    polynomial CG and deflated GMRES (Chebyshev-preconditioned). Cases: a single block
    (d < 64), d = 512 (8 x 8 blocks) and d = 5115 (80 x 80 blocks, a ragged last block of
    59; the dense product there sums s in a kernel of its own).
    Both products sum in fixed orders that differ, and the explicit inverse's rounding
    (about cond(E) times the unit roundoff) moves the float64 iteration count by a few per
    cent at d = 5115 (symmetric 268, dense 275, oracle 267): float64 counts within 4 % of
    the oracle's for both products, the other solvers' counts within 5 % of each other.
    Errors within 1e-6 of the solution, except GMRES (see below)."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _problem(name, scale, kw)
    if nsub is not None:
        p = dataclasses.replace(p, nsub=nsub)
    K, b = dev(p.K), dev(p.q)
    A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    lab, d = O.levelset_labels(p.grid, p.K, p.nsub, p.thr)
    say(f"coarse symmetric {name}/{scale} grid={p.grid} nsub={p.nsub} d={d}")
    ref = O.dpcg(A, bh, O.deflation_matrix(lab, d), tol=1e-8)
    xr = _reference_x(A, bh, p.n)
    if xr is None:
        xr = O.dpcg(A, bh, O.deflation_matrix(lab, d), tol=1e-12).x
    runs = [("fp64", dict(mode=0)), ("fp64-reproject", dict(mode=0, reproject=1)),
            ("mixed", dict(mode=1)), ("poly", None), ("gmres", None)]
    out = {}
    for cs in (1, -1):
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr), coarse_sym=cs)
        assert s.d == d
        assert psl.psl_get_info(s.ctx)["coarse_sym"] == (cs > 0)
        for tag, kw_solve in runs:
            if tag == "poly":
                x, st = psl.psl_solve_poly(s.ctx, b, tol=1e-8)
            elif tag == "gmres":
                # GMRES(30) with diag(A) stagnates on the region vectors of the d = 5115
                # case (as the oracle's does); with the Chebyshev preconditioner it converges
                x, st = psl.psl_solve_gmres(s.ctx, b, tol=1e-8, degree=3)
            else:
                x, st = psl.psl_solve(s.ctx, b, tol=1e-8, **kw_solve)
            out[(cs, tag)] = (host(x), st)
        s.ctx.destroy()
    failures = []
    for tag, _ in runs:
        (xs, sts), (xd, std) = out[(1, tag)], out[(-1, tag)]
        res, resd = O.relres(A, bh, xs), O.relres(A, bh, xd)
        err = np.linalg.norm(xs - xr) / np.linalg.norm(xr)
        errd = np.linalg.norm(xd - xr) / np.linalg.norm(xr)
        say(f"  {tag}: symmetric iters={sts['iters']} relres={res:.2e} err={err:.2e}; "
            f"dense iters={std['iters']} relres={resd:.2e} err={errd:.2e} "
            f"(oracle DPCG {ref.iters})")
        ok = sts["status"] == 0 and std["status"] == 0 and res <= 1e-8 and resd <= 1e-8
        if tag == "gmres":
            # GMRES minimises the preconditioned deflated residual, not an energy norm: at
            # a 1e-8 residual its error on the d = 5115 case is 3.7e-6 with either product
            # (its accuracy against the oracle's GMRES is tested elsewhere)
            ok = ok and err <= max(1e-6, 2 * errd)
        else:
            ok = ok and err <= 1e-6 and errd <= 1e-6
        if tag.startswith("fp64"):
            ok = ok and all(abs(k - ref.iters) <= max(2, 0.04 * ref.iters)
                            for k in (sts["iters"], std["iters"]))
        else:
            ok = ok and abs(sts["iters"] - std["iters"]) <= max(3, 0.05 * std["iters"])
        if not ok:
            failures.append(tag)
    assert not failures, failures


@pytest.mark.parametrize("tile", [None, 1024], ids=["default-tiles", "tiles-1024"])
@pytest.mark.parametrize("name,scale,kw", FINISH_CASES,
                         ids=[f"{c[0]}-{c[1]}" for c in FINISH_CASES])
def test_stencil_split(gpu_lib, name, scale, kw, tile):
    """The float32 stencil pass split in two (the direction update p = u + beta p_prev in
    a pass of its own, then the plain stencil q = A p with its partials) against the
    fused pass that recomputes the neighbours' p, both with finish kernels (forced on for
    these small grids), in mixed precision: the same fused multiply-add and the same sums
    in the same order, so x is bit-identical with equal iteration and refinement counts;
    and the oracle's residual of x. With 1024-cell tiles each thread owns four cells,
    which the plain stencil takes two at a time and the fused pass all at once."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _problem(name, scale, kw)
    say(f"stencil split {name}/{scale} grid={p.grid} tile={tile}")
    K, b = dev(p.K), dev(p.q)
    out = {}
    for split in (1, -1):
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr), finish_kernels=1,
                           stencil_split=split, tile_cells=tile)
        x, st = psl.psl_solve(s.ctx, b, tol=1e-8, mode=psl.MIXED)
        out[split] = (x.clone(), st)
        s.ctx.destroy()
    (x1, st1), (x0, st0) = out[1], out[-1]
    A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    res = O.relres(A, bh, host(x1))
    say(f"  split: iters={st1['iters']} outer={st1['outer']} fell_back={st1['fell_back']} "
        f"relres={res:.2e}; fused: iters={st0['iters']} outer={st0['outer']}")
    assert st1["status"] == 0 and res <= 1e-8
    assert (st1["iters"], st1["outer"], st1["fell_back"]) == \
        (st0["iters"], st0["outer"], st0["fell_back"])
    assert torch.equal(x1, x0)


def test_profile_kernel(gpu_lib):
    """psl_profile_kernel / psl_profile_read: events around one kernel's launches inside
    real solves. On a grid of 2^14 cells, float64: every stencil launch of the solve is
    timed (at least one per iteration), and x equals the unprofiled solve bit for bit (the
    same kernels in the same order, launched directly instead of replayed); mixed: the
    float32 stencil steps are timed, x again bit-identical. On
    the 64x64 case (float64, one-workgroup inner solve): one timed launch per inner solve,
    x bit-identical to the unprofiled solve; arming a pass kernel there runs the
    three-launch loop instead, which still meets the oracle. The one-workgroup id is
    float64 only."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    for name, scale, mode in (("c2", 4, psl.FP64), ("c2", 4, psl.MIXED), ("c1", 1, psl.FP64)):
        p = _problem(name, scale, {})
        s = pipeline.setup(p.grid, dev(p.K), p.dirichlet_mask, p.nsub, list(p.thr))
        b = dev(p.q)
        small = bool(psl.psl_get_info(s.ctx)["small_solve"])
        assert small == (name == "c1")
        x0, st0 = psl.psl_solve(s.ctx, b, tol=1e-8, mode=mode)
        kid = psl.KERNEL_SMALL_SOLVE if small else psl.KERNEL_STENCIL
        psl.psl_profile_kernel(s.ctx, kid, mode)
        x1, st1 = psl.psl_solve(s.ctx, b, tol=1e-8, mode=mode)
        dur = psl.psl_profile_read(s.ctx)
        psl.psl_profile_kernel(s.ctx, -1, mode)
        say(f"profile {name}: {len(dur)} launches timed, median {np.median(dur):.1f} us, "
            f"iters {st1['iters']} outer {st1['outer']}")
        assert torch.equal(x0, x1) and st0["iters"] == st1["iters"]
        assert all(v > 0 for v in dur)
        if small:
            assert len(dur) == st1["outer"]
            psl.psl_profile_kernel(s.ctx, psl.KERNEL_STENCIL, mode)
            x2, st2 = psl.psl_solve(s.ctx, b, tol=1e-8, mode=mode)
            n2 = len(psl.psl_profile_read(s.ctx))
            psl.psl_profile_kernel(s.ctx, -1, mode)
            A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
            assert n2 >= st2["iters"] and O.relres(A, bh, host(x2)) <= 1e-8
            with pytest.raises(psl.PslError):
                psl.psl_profile_kernel(s.ctx, psl.KERNEL_SMALL_SOLVE, psl.MIXED)
        elif mode == psl.FP64:
            assert len(dur) >= st1["iters"]
        else:
            assert len(dur) >= 1
        s.ctx.destroy()


FACE_CASES = [("c2", 4, {}, False), ("c3", 4, {"contrast": 1e5}, True), ("ragged", 0, {}, False)]


@pytest.mark.parametrize("finish", [1, -1], ids=["finish", "passes"])
@pytest.mark.parametrize("name,scale,kw,components", FACE_CASES,
                         ids=["c2-4", "c3-4-components", "ragged-0"])
def test_face_tables(gpu_lib, name, scale, kw, components, finish):
    """The float32 update with per-tile coarse tables (each cut face packed into one word of
    local indices, the tile's coarse values gathered once) against the unpacked faces, with
    and without finish kernels, in mixed precision, for the Jacobi CG and the Chebyshev
    polynomial CG (whose update applies the same correction): the same terms summed in the
    same order, so x is bit-identical with equal iteration and refinement counts; and the
    oracle's residual of x."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _problem(name, scale, kw)
    say(f"face tables {name}/{scale} components={components} finish={finish} grid={p.grid}")
    K, b = dev(p.K), dev(p.q)
    out = {}
    for ft in (1, -1):
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr),
                           components=components, finish_kernels=finish, face_tables=ft)
        assert psl.psl_get_info(s.ctx)["face_tables"] == (ft > 0)
        x, st = psl.psl_solve(s.ctx, b, tol=1e-8, mode=psl.MIXED)
        xp, stp = psl.psl_solve_poly(s.ctx, b, tol=1e-8, mixed=True)
        out[ft] = (x.clone(), st)
        out[(ft, "poly")] = (xp.clone(), stp)
        s.ctx.destroy()
    (xp1, stp1), (xp0, stp0) = out[(1, "poly")], out[(-1, "poly")]
    say(f"  polynomial CG: tables iters={stp1['iters']}, unpacked iters={stp0['iters']}")
    assert stp1["iters"] == stp0["iters"] and torch.equal(xp1, xp0)
    (x1, st1), (x0, st0) = out[1], out[-1]
    A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    res = O.relres(A, bh, host(x1))
    say(f"  tables: iters={st1['iters']} outer={st1['outer']} relres={res:.2e}; "
        f"unpacked: iters={st0['iters']} outer={st0['outer']}")
    assert st1["status"] == 0 and res <= 1e-8
    assert (st1["iters"], st1["outer"]) == (st0["iters"], st0["outer"])
    assert torch.equal(x1, x0)


@pytest.mark.parametrize("finish", [1, -1], ids=["finish", "passes"])
@pytest.mark.parametrize("name,scale,kw,components", FACE_CASES,
                         ids=["c2-4", "c3-4-components", "ragged-0"])
def test_wide_tiles(gpu_lib, name, scale, kw, components, finish):
    """Tiles two subdomain boxes wide (whole 128-byte rows of float32) against tiles inside
    one box: the same operator and deflation space, only the per-tile partial sums grouped
    differently, so both solutions meet the oracle's residual bound and take nearly the
    same number of iterations, in float64 and mixed precision."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = _problem(name, scale, kw)
    nx, sx = p.grid[0], p.nsub[0]
    expect = sx >= 2 and nx // sx < 32
    say(f"wide tiles {name}/{scale} grid={p.grid} nsub={p.nsub} expect={expect} finish={finish}")
    K, b = dev(p.K), dev(p.q)
    A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
    its = {}
    for wt in (1, -1):
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr),
                           components=components, finish_kernels=finish, wide_tiles=wt)
        assert psl.psl_get_info(s.ctx)["wide_tiles"] == int(wt > 0 and expect)
        for mode in (psl.FP64, psl.MIXED):
            x, st = psl.psl_solve(s.ctx, b, tol=1e-8, mode=mode)
            res = O.relres(A, bh, host(x))
            say(f"  wide={wt} mode={mode}: iters={st['iters']} outer={st['outer']} "
                f"relres={res:.2e}")
            assert st["status"] == 0 and res <= 1e-8
            its[(wt, mode)] = st["iters"]
        s.ctx.destroy()
    for mode in (psl.FP64, psl.MIXED):
        a, c = its[(1, mode)], its[(-1, mode)]
        assert abs(a - c) <= max(2, 0.03 * c), (mode, a, c)


def _tile_count(grid, nsub, tile_max, span):
    """Tiles of the documented split rule: boxes of the floor partition (pairs of
    x-adjacent boxes when spanning), each cut into the fewest z chunks whose largest part
    holds at most tile_max cells, else whole planes into the fewest y chunks that fit,
    else rows cut in x."""
    def lo(b, n, s):
        return (b * n + s - 1) // s

    def cdiv(a, b):
        return (a + b - 1) // b
    nx, ny, nz = grid
    step = 2 if span else 1
    count = 0
    for bz in range(nsub[2]):
        for by in range(nsub[1]):
            for bx in range(0, nsub[0], step):
                ex = lo(min(bx + step, nsub[0]), nx, nsub[0]) - lo(bx, nx, nsub[0])
                ey = lo(by + 1, ny, nsub[1]) - lo(by, ny, nsub[1])
                ez = lo(bz + 1, nz, nsub[2]) - lo(bz, nz, nsub[2])
                cz = cy = cx = 1
                if ex * ey * ez > tile_max:
                    cz = min(ez, cdiv(ex * ey * ez, tile_max))
                    while cz < ez and ex * ey * cdiv(ez, cz) > tile_max:
                        cz += 1
                    if ex * ey * cdiv(ez, cz) > tile_max:
                        cz = ez
                        cy = min(ey, cdiv(ex * ey, tile_max))
                        while cy < ey and ex * cdiv(ey, cy) > tile_max:
                            cy += 1
                        if ex * cdiv(ey, cy) > tile_max:
                            cy, cx = ey, cdiv(ex, tile_max)
                count += cx * cy * cz
    return count


TILE_RULE_CASES = [((87, 87, 87), (4, 4, 4), 256), ((64, 48, 32), (4, 3, 2), 512),
                   ((37, 29, 11), (5, 3, 2), 128), ((96, 80, 48), (6, 5, 3), 1024)]


@pytest.mark.parametrize("grid,nsub,tile", TILE_RULE_CASES)
def test_tile_split_rule(gpu_lib, grid, nsub, tile):
    """The library's tiling follows the split rule on boxes one and two wide (a box whose
    planes do not fit is cut into the fewest y chunks that fit, not into rows: a rounding
    slip there once made 44-cell tiles on an 87^3 grid), and a solve on it is correct."""
    psl = gpu_lib
    from paper_1510_02148_amd import pipeline
    p = pi.layered3d(*grid, nlayers=4, contrast=1e4, nsub=nsub, seed=5)
    say(f"tile rule grid={grid} nsub={nsub} tile={tile}")
    K = dev(p.K)
    for wt in (1, -1):
        s = pipeline.setup(p.grid, K, p.dirichlet_mask, p.nsub, list(p.thr), tile_cells=tile,
                           wide_tiles=wt)
        info = psl.psl_get_info(s.ctx)
        want = _tile_count(grid, nsub, tile, bool(info["wide_tiles"]))
        say(f"  wide={info['wide_tiles']}: ntiles={info['ntiles']} rule={want}")
        assert info["wide_tiles"] == int(wt > 0 and grid[0] // nsub[0] < 32)
        assert info["ntiles"] == want
        if wt > 0:
            x, st = psl.psl_solve(s.ctx, dev(p.q), tol=1e-8, mode=psl.MIXED)
            A, bh = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
            assert st["status"] == 0 and O.relres(A, bh, host(x)) <= 1e-8
        s.ctx.destroy()
