"""Pins that tie the CPU oracle to facts other than itself.

Each pin takes the oracle module ``O`` and raises AssertionError on failure, so
the same pins run against the real oracle (test_oracle_pins.py) and against
deliberately broken copies of it (test_oracle_mutants.py), which shows that a
plausible slip anywhere in the oracle trips at least one pin.

Sources of truth used (none of them is the oracle's own formula retyped):
  * series-resistance closed forms of 1D Darcy flow (discrete flux balance),
  * second differences of polynomials on homogeneous media,
  * row sums = boundary transmissibility, symmetry, M-matrix sign pattern,
  * brute-force pure-Python labelling on tiny grids (regions and their connected
    components), scipy.ndimage.label per region,
  * brute-force face sums for the coarse matrix E = Z^T A Z,
  * textbook Jacobi-PCG (scipy.sparse.linalg.cg) when no vector is deflated,
  * dense direct solves (numpy.linalg.solve),
  * GMRES's defining property: the minimal residual over an explicitly built Krylov
    space,
  * the projector identities of Definition 3.1 and Section 3.1,
  * Theorem 2.1 (eigenvalue count of the diagonally scaled matrix),
  * jump independence of deflated CG (Section 1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

XLO, XHI, YLO, YHI, ZLO, ZHI = 1, 2, 4, 8, 16, 32


def _lognormal(shape, seed, sigma=2.0):
    g = np.random.Generator(np.random.PCG64(seed))
    return np.exp(sigma * g.standard_normal(shape))


def _close(a, b, rtol, what=""):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.max(np.abs(b)), 1e-300)
    err = np.max(np.abs(a - b)) / scale if a.size else 0.0
    assert err <= rtol, f"{what}: rel err {err:.3e} > {rtol:.1e}"


# --------------------------------------------------------------- discretisation

def pin_row_sums(O):
    """A 1 = boundary transmissibility: 2 K_i per Dirichlet face of cell i, interior rows 0."""
    grid = (5, 4, 3)
    nx, ny, nz = grid
    K = _lognormal(nx * ny * nz, 1)
    mask = XLO | ZHI | YLO
    Tx, Ty, Tz = O.transmissibilities(K, grid, mask)
    A = O.pressure_matrix(grid, Tx, Ty, Tz)
    k = K.reshape(nz, ny, nx)
    expect = np.zeros((nz, ny, nx))
    expect[:, :, 0] += 2 * k[:, :, 0]
    expect[:, 0, :] += 2 * k[:, 0, :]
    expect[nz - 1, :, :] += 2 * k[nz - 1, :, :]
    _close(A @ np.ones(K.size), expect.reshape(-1), 1e-13, "A*1")


def pin_symmetric_mmatrix(O):
    """Symmetric, non-positive off-diagonals, weakly diagonally dominant, positive definite."""
    grid = (4, 3, 3)
    K = _lognormal(36, 2)
    Tx, Ty, Tz = O.transmissibilities(K, grid, XLO)
    A = O.pressure_matrix(grid, Tx, Ty, Tz).toarray()
    assert np.array_equal(A, A.T), "A not symmetric"
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0), "positive off-diagonal"
    assert np.all(np.diag(A) + off.sum(1) >= -1e-14 * np.diag(A)), "not diagonally dominant"
    assert np.linalg.eigvalsh(A).min() > 0, "not positive definite"
    # every cell couples to exactly its grid neighbours
    nnz_off = (off != 0).sum(1).reshape(3, 3, 4)
    assert nnz_off[1, 1, 1] == 6 and nnz_off[0, 0, 0] == 3, "wrong stencil connectivity"


def pin_second_difference(O):
    """Homogeneous K = k: A applied to p = c^2 along one axis gives -2k on interior rows
    (the 7-point Laplacian of a parabola), and 0 for p linear."""
    grid = (7, 6, 5)
    nx, ny, nz = grid
    k = 3.5
    K = np.full(nx * ny * nz, k)
    Tx, Ty, Tz = O.transmissibilities(K, grid, 0)
    A = O.pressure_matrix(grid, Tx, Ty, Tz)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for axis, c, m in ((0, ix, nx), (1, iy, ny), (2, iz, nz)):
        inner = (c > 0) & (c < m - 1)
        r = (A @ (c.astype(float) ** 2).reshape(-1)).reshape(nz, ny, nx)
        _close(r[inner], np.full(inner.sum(), -2 * k), 1e-13, f"parabola axis {axis}")
        r1 = (A @ c.astype(float).reshape(-1)).reshape(nz, ny, nx)
        assert np.max(np.abs(r1[inner])) <= 1e-12 * k * m, f"linear field axis {axis}"


def _series_1d(K, a, b):
    """Pressure of 1D Darcy flow with p = 0 at the left outer face, no-flow at the right,
    unit injection in cell a and unit extraction in cell b > a: zero flux left of a,
    unit flux from a to b, so the drop over face (k-1|k) is 1/(2K_{k-1}) + 1/(2K_k)."""
    n = len(K)
    p = np.zeros(n)
    for i in range(a + 1, n):
        if i <= b:
            p[i] = p[i - 1] - (1.0 / (2 * K[i - 1]) + 1.0 / (2 * K[i]))
        else:
            p[i] = p[i - 1]
    return p


def _single_source_1d(K, s):
    """Unit injection in cell s, drained through the p = 0 left face: unit flux to the
    left of s, so p_0 = 1/(2K_0) and p_i = p_{i-1} + 1/(2K_{i-1}) + 1/(2K_i) up to s."""
    n = len(K)
    p = np.zeros(n)
    p[0] = 1.0 / (2 * K[0])
    for i in range(1, n):
        p[i] = p[i - 1] + ((1.0 / (2 * K[i - 1]) + 1.0 / (2 * K[i])) if i <= s else 0.0)
    return p


def pin_series_resistance(O):
    """Discrete 1D solutions (and 3D with K varying only in x and plane sources)."""
    from scipy.sparse.linalg import spsolve
    nx = 24
    K1 = _lognormal(nx, 3, sigma=3.0)
    for (a, b) in ((0, nx - 1), (5, 17), (3, 4)):
        q = np.zeros(nx)
        q[a] += 1.0
        q[b] -= 1.0
        A, rhs = O.assemble(K1, (nx, 1, 1), XLO, q)
        _close(spsolve(A.tocsc(), rhs), _series_1d(K1, a, b), 1e-10, f"1D pair {a},{b}")
    q = np.zeros(nx)
    q[9] = 1.0
    A, rhs = O.assemble(K1, (nx, 1, 1), XLO, q)
    _close(spsolve(A.tocsc(), rhs), _single_source_1d(K1, 9), 1e-10, "1D single source")
    # 3D: K(x) only, unit source in every cell of plane a, sink in plane b
    ny, nz = 3, 2
    K1 = _lognormal(nx, 4, sigma=1.0)
    K3 = np.tile(K1, ny * nz)
    q3 = np.zeros((nz, ny, nx))
    q3[:, :, 4] = 1.0
    q3[:, :, 19] = -1.0
    A, rhs = O.assemble(K3, (nx, ny, nz), XLO, q3.reshape(-1))
    ref = np.tile(_series_1d(K1, 4, 19), ny * nz)
    _close(spsolve(A.tocsc(), rhs), ref, 1e-10, "3D planes")


# ------------------------------------------------------------------ labels / Z

def _labels_bruteforce(grid, K, nsub, thr, cls=None, ncls=None):
    nx, ny, nz = grid
    sx, sy, sz = nsub
    keys = []
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                c = ix + nx * (iy + ny * iz)
                bx = (ix * sx) // nx
                by = (iy * sy) // ny
                bz = (iz * sz) // nz
                s = bx + sx * (by + sy * bz)
                if cls is None:
                    k = sum(1 for t in thr if K[c] >= t)
                    nc = len(thr) + 1
                else:
                    k = int(cls[c])
                    nc = ncls
                keys.append(s * nc + k)
    order = sorted(set(keys))
    rank = {key: i for i, key in enumerate(order)}
    return np.array([rank[key] for key in keys], dtype=np.int32), len(order)


def pin_labels_bruteforce(O):
    g = np.random.Generator(np.random.PCG64(4))
    for grid, nsub, thr in (((7, 5, 3), (3, 2, 2), [0.1, 1.0]),
                            ((9, 4, 1), (4, 3, 1), [1.0]),
                            ((5, 5, 5), (5, 1, 2), [0.01, 0.5, 2.0]),
                            ((6, 6, 4), (1, 1, 1), [0.3])):
        n = grid[0] * grid[1] * grid[2]
        K = np.exp(1.5 * g.standard_normal(n))
        K[::7] = thr[0]                      # ties sit exactly on a threshold
        lab, d = O.levelset_labels(grid, K, nsub, np.array(thr))
        ref, dref = _labels_bruteforce(grid, K, nsub, thr)
        assert d == dref and np.array_equal(lab, ref), f"labels differ on {grid} {nsub}"
    # manual classes (the paper's hand-made layer indicators)
    grid = (6, 5, 4)
    cls = g.integers(0, 3, size=120)
    lab, d = O.levelset_labels(grid, None, (2, 1, 2), None, cls=cls, ncls=3)
    ref, dref = _labels_bruteforce(grid, None, (2, 1, 2), None, cls=cls, ncls=3)
    assert d == dref and np.array_equal(lab, ref), "manual-class labels differ"


def pin_labels_layered2d(O):
    """64x64, 8-row layers, 4x4 subdomains: each 16x16 subdomain holds two layers of
    8x16 cells, one above and one below the threshold: d = 32 regions of 128 cells,
    Z^T Z = 128 I (disjoint, orthogonal vectors)."""
    nx = ny = 64
    K = np.repeat(np.where((np.arange(ny) // 8) % 2 == 0, 1.0, 1e-4), nx)
    lab, d = O.levelset_labels((nx, ny, 1), K, (4, 4, 1), np.array([1e-2]))
    assert d == 32
    Z = O.deflation_matrix(lab, d)
    ZtZ = (Z.T @ Z).toarray()
    assert np.array_equal(ZtZ, 128 * np.eye(32)), "Z^T Z != 128 I"


def _components_bruteforce(grid, K, nsub, thr, cls=None, ncls=None):
    """Breadth-first search over face neighbours with equal (subdomain, class) key,
    started from each unlabelled cell in natural order: labels come out ordered by the
    smallest cell index of their component."""
    nx, ny, nz = grid
    keys, _ = _labels_bruteforce(grid, K, nsub, thr, cls=cls, ncls=ncls)   # rank of key
    n = nx * ny * nz
    lab = [-1] * n
    d = 0
    for start in range(n):
        if lab[start] >= 0:
            continue
        lab[start] = d
        queue = [start]
        while queue:
            c = queue.pop()
            ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
            for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                jx, jy, jz = ix + dx, iy + dy, iz + dz
                if 0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz:
                    m = jx + nx * (jy + ny * jz)
                    if lab[m] < 0 and keys[m] == keys[c]:
                        lab[m] = d
                        queue.append(m)
        d += 1
    return np.array(lab, dtype=np.int32), d


def pin_components_bruteforce(O):
    """Connected-component labels against a pure-Python search on tiny grids (3D and 2D,
    several partitions and thresholds, manual classes)."""
    g = np.random.Generator(np.random.PCG64(14))
    for grid, nsub, thr in (((7, 5, 4), (2, 2, 2), [0.3, 2.0]),
                            ((9, 7, 1), (3, 2, 1), [1.0]),
                            ((6, 6, 6), (1, 1, 1), [0.2, 1.0, 3.0]),
                            ((8, 3, 5), (4, 3, 1), [0.7])):
        n = grid[0] * grid[1] * grid[2]
        K = np.exp(1.5 * g.standard_normal(n))
        lab, d = O.levelset_components(grid, K, nsub, np.array(thr))
        ref, dref = _components_bruteforce(grid, K, nsub, thr)
        assert d == dref and np.array_equal(lab, ref), f"components differ on {grid} {nsub}"
    grid = (6, 5, 4)
    cls = g.integers(0, 3, size=120)
    lab, d = O.levelset_components(grid, None, (2, 1, 2), None, cls=cls, ncls=3)
    ref, dref = _components_bruteforce(grid, None, (2, 1, 2), None, cls=cls, ncls=3)
    assert d == dref and np.array_equal(lab, ref), "manual-class components differ"


def pin_components_ndimage(O):
    """The same partition as scipy.ndimage.label (face connectivity) applied to each
    (subdomain, class) region separately, on a channel-like field; and on the 64x64
    layered case, where every region is connected, the plain subdomain-levelset
    partition."""
    from scipy import ndimage
    grid = (24, 20, 12)
    nx, ny, nz = grid
    g = np.random.Generator(np.random.PCG64(15))
    field = ndimage.gaussian_filter(g.standard_normal((nz, ny, nx)), 2.0)
    K = np.where(field > 0.1, 1.0, 1e-4).reshape(-1)
    nsub, thr = (3, 2, 2), np.array([1e-2])
    lab, d = O.levelset_components(grid, K, nsub, thr)
    keys, _ = O.levelset_labels(grid, K, nsub, thr)
    keys = keys.reshape(nz, ny, nx)
    structure = ndimage.generate_binary_structure(3, 1)
    parts = set()
    for k in np.unique(keys):
        comp, num = ndimage.label(keys == k, structure=structure)
        for j in range(1, num + 1):
            parts.add(frozenset(np.flatnonzero(comp.reshape(-1) == j).tolist()))
    mine = {frozenset(np.flatnonzero(lab == j).tolist()) for j in range(d)}
    assert d == len(parts) and mine == parts, "partition differs from ndimage.label"
    assert d > len(np.unique(keys)), "the field should split some regions"
    # columns ordered by their first cell
    first = [int(np.flatnonzero(lab == j)[0]) for j in range(d)]
    assert first == sorted(first)
    nx = ny = 64
    K = np.repeat(np.where((np.arange(ny) // 8) % 2 == 0, 1.0, 1e-4), nx)
    lab, d = O.levelset_components((nx, ny, 1), K, (4, 4, 1), np.array([1e-2]))
    lab0, d0 = O.levelset_labels((nx, ny, 1), K, (4, 4, 1), np.array([1e-2]))
    assert d == d0 == 32
    assert {frozenset(np.flatnonzero(lab == j).tolist()) for j in range(d)} == \
        {frozenset(np.flatnonzero(lab0 == j).tolist()) for j in range(d0)}


def _tiny_system(O, seed, grid=(6, 5, 4), nsub=(2, 2, 1), thr=(0.5,)):
    nx, ny, nz = grid
    K = _lognormal(nx * ny * nz, seed)
    q = np.zeros(nx * ny * nz)
    q[0], q[-1] = 1.0, -0.5
    A, b = O.assemble(K, grid, XLO, q)
    lab, d = O.levelset_labels(grid, K, nsub, np.array(thr))
    return A, b, O.deflation_matrix(lab, d)


def pin_gmres_direct(O):
    """Deflated GMRES(m) reaches the dense direct solution, with and without restarts and
    with no deflation vectors at all (d = 0: plain right-preconditioned GMRES)."""
    for seed, m in ((21, 5), (22, 40)):
        A, b, Z = _tiny_system(O, seed)
        xd = np.linalg.solve(A.toarray(), b)
        for ZZ in (Z, Z[:, :0]):
            r = O.pdgmres(A, b, ZZ, m=m, tol=1e-12)
            assert r.status == "ok"
            assert np.linalg.norm(r.x - xd) <= 1e-9 * np.linalg.norm(xd), (seed, m, ZZ.shape)


def pin_chebyshev_closed_form(O):
    """The Chebyshev recurrence against its closed form: with S = D^-1/2 A D^-1/2 = U L U^T,
    k steps from y = 0 give y = D^-1/2 U diag((1 - T_k((theta - l) / delta) / T_k(theta /
    delta)) / l) U^T D^-1/2 r (the error polynomial of the Chebyshev iteration; T_k from
    numpy's Chebyshev basis). Also: the spectrum of D^-1 A lies in (0, 2] (Gershgorin
    for these matrices), so with lmax = 2 the operator is symmetric positive definite."""
    from numpy.polynomial import chebyshev as C
    for seed in (31, 32):
        A, _, _ = _tiny_system(O, seed)
        Ad = A.toarray()
        dg = np.diag(Ad)
        s = 1.0 / np.sqrt(dg)
        lam, U = np.linalg.eigh(Ad * s[:, None] * s[None, :])
        assert lam.min() > 0 and lam.max() <= 2.0 + 1e-12
        for k in (1, 2, 3, 5):
            for lmin, lmax in ((0.25, 2.0), (0.05, 1.9), (0.5, 2.0)):
                th, de = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
                Tk = C.Chebyshev.basis(k)
                q = (1.0 - Tk((th - lam) / de) / Tk(th / de)) / lam
                Qc = (s[:, None] * U) @ np.diag(q) @ (U.T * s[None, :])
                Q = np.column_stack([O.chebyshev_apply(A, e, k, lmin, lmax)
                                     for e in np.eye(Ad.shape[0])])
                assert np.linalg.norm(Q - Qc) <= 1e-10 * np.linalg.norm(Qc), (seed, k, lmin)
                if lmax >= lam.max():
                    assert np.linalg.norm(Q - Q.T) <= 1e-12 * np.linalg.norm(Q)
                    assert np.linalg.eigvalsh(0.5 * (Q + Q.T)).min() > 0


def pin_poly_degree_one_is_jacobi(O):
    """Degree 1 is Jacobi times 1/theta, a scale CG does not see: the same residual
    history as the Jacobi-preconditioned deflated CG, step by step."""
    for seed in (33, 34):
        A, b, Z = _tiny_system(O, seed)
        ref = O.dpcg(A, b, Z, tol=1e-10)
        r = O.dpcg_poly(A, b, Z, degree=1, ratio=8.0, tol=1e-10)
        assert r.iters == ref.iters and r.status == "ok"
        assert np.allclose(r.history, ref.history, rtol=1e-7, atol=1e-12 * ref.history[0])


def pin_poly_direct(O):
    """Deflated CG with the polynomial preconditioner reaches the dense direct solution
    for several degrees and intervals, and with no deflation vectors (d = 0)."""
    for seed in (35, 36):
        A, b, Z = _tiny_system(O, seed)
        xd = np.linalg.solve(A.toarray(), b)
        for k, ratio in ((2, 8.0), (3, 30.0), (5, 4.0)):
            for ZZ in (Z, Z[:, :0]):
                r = O.dpcg_poly(A, b, ZZ, degree=k, ratio=ratio, tol=1e-12)
                assert r.status == "ok"
                assert np.linalg.norm(r.x - xd) <= 1e-9 * np.linalg.norm(xd), (seed, k)


def pin_gmres_poly_direct(O):
    """Deflated GMRES(m) with the Chebyshev polynomial preconditioner (degrees 2, 3, 5)
    reaches the dense direct solution, with restarts, and needs fewer steps than with
    Jacobi on the same system."""
    for seed, m in ((24, 8), (25, 40)):
        A, b, Z = _tiny_system(O, seed)
        xd = np.linalg.solve(A.toarray(), b)
        jac = O.pdgmres(A, b, Z, m=m, tol=1e-12)
        for k in (2, 3, 5):
            r = O.pdgmres(A, b, Z, m=m, tol=1e-12, degree=k, ratio=30.0)
            assert r.status == "ok"
            assert np.linalg.norm(r.x - xd) <= 1e-9 * np.linalg.norm(xd), (seed, m, k)
            assert r.iters < jac.iters, (seed, m, k, r.iters, jac.iters)


def pin_gmres_minimal_residual(O):
    """After k steps of a first cycle the least-squares residual is the smallest
    ||r0 - B K_k y|| over the Krylov space K_k = span{r0, B r0, ..., B^(k-1) r0} of
    B = P1 A M^-1 (computed here from an explicit, QR-orthonormalised Krylov basis), and
    it equals the true deflated residual ||P1 (b - A x_k)|| of the iterate the cycle
    returns (which checks x_k = x0 + M^-1 V u)."""
    A, b, Z = _tiny_system(O, 23)
    Ad = A.toarray()
    dg = np.diag(Ad)
    E = (Z.T @ (A @ Z)).toarray()
    Zd = Z.toarray()
    P1 = np.eye(Ad.shape[0]) - Ad @ Zd @ np.linalg.solve(E, Zd.T)
    B = P1 @ Ad / dg[None, :]
    r0 = P1 @ b
    for k in range(1, 7):
        Kk = np.empty((r0.size, k))
        v = r0.copy()
        for i in range(k):
            Kk[:, i] = v
            v = B @ v
        Q, _ = np.linalg.qr(Kk)
        y = np.linalg.lstsq(B @ Q, r0, rcond=None)[0]
        best = np.linalg.norm(r0 - B @ Q @ y)
        r = O.pdgmres(A, b, Z, m=k, tol=1e-300, maxit=k)
        assert abs(r.history[k] - best) <= 1e-9 * np.linalg.norm(r0), (k, r.history[k], best)
        true_res = np.linalg.norm(P1 @ (b - Ad @ r.xhat))
        assert abs(true_res - r.history[k]) <= 1e-9 * np.linalg.norm(r0), (k, true_res)


def pin_gmres_monotone(O):
    """The residual of GMRES never grows, inside a cycle or across restarts."""
    A, b, Z = _tiny_system(O, 24, grid=(9, 8, 5), nsub=(3, 2, 1))
    r = O.pdgmres(A, b, Z, m=4, tol=1e-10)
    assert r.status == "ok" and np.all(np.diff(r.history) <= 1e-12 * r.history[0])


# ------------------------------------------------------------------ coarse E

def pin_coarse_matrix(O):
    grid = (6, 5, 4)
    nx, ny, nz = grid
    K = _lognormal(nx * ny * nz, 5)
    Tx, Ty, Tz = O.transmissibilities(K, grid, XLO | YHI)
    A = O.pressure_matrix(grid, Tx, Ty, Tz)
    lab, d = O.levelset_labels(grid, K, (2, 2, 2), np.array([1.0]))
    Z = O.deflation_matrix(lab, d)
    E = O.coarse_matrix(A, Z)
    # brute force over faces: off-diagonal = -sum of T over faces joining two regions,
    # row sum = Dirichlet transmissibility of the region
    Eref = np.zeros((d, d))
    bnd = np.zeros(d)
    L = lab.reshape(nz, ny, nx)
    faces = ((Tx.reshape(nz, ny, nx + 1), 2), (Ty.reshape(nz, ny + 1, nx), 1),
             (Tz.reshape(nz + 1, ny, nx), 0))
    for T, ax in faces:
        for idx in np.ndindex(*T.shape):
            t = T[idx]
            m = idx[ax]
            hi = list(idx)
            lo = list(idx)
            lo[ax] = m - 1
            if 0 < m < L.shape[ax]:
                a, b = L[tuple(lo)], L[tuple(hi)]
                if a != b:
                    Eref[a, b] -= t
                    Eref[b, a] -= t
            elif t:
                inside = list(idx)
                inside[ax] = min(m, L.shape[ax] - 1)
                bnd[L[tuple(inside)]] += t
    np.fill_diagonal(Eref, bnd - (Eref.sum(1) - np.diag(Eref)))
    _close(E, Eref, 1e-12, "E vs face sums")
    assert np.linalg.eigvalsh(E).min() > 0, "E not SPD"
    # one region per cell: E = A
    n = nx * ny * nz
    Zid = O.deflation_matrix(np.arange(n, dtype=np.int32), n)
    _close(O.coarse_matrix(A, Zid), A.toarray(), 0.0, "E with d = n")


# ------------------------------------------------------------------ DPCG

def pin_textbook_pcg(O):
    """No deflation vectors: the iteration is textbook Jacobi-PCG; iterates after k steps
    equal scipy's cg with M = diag(A)^-1."""
    grid = (9, 8, 5)
    K = _lognormal(360, 6)
    g = np.random.Generator(np.random.PCG64(7))
    A, _ = O.assemble(K, grid, XLO, np.zeros(360))
    b = g.standard_normal(360)
    Z0 = O.deflation_matrix(np.zeros(360, dtype=np.int32), 0)
    M = spla.LinearOperator(A.shape, matvec=lambda v: v / A.diagonal())
    for k in (1, 2, 7, 25):
        res = O.dpcg(A, b, Z0, tol=0.0, maxit=k)
        assert res.iters == k and res.status == "maxit"
        xs, _ = spla.cg(A, b, x0=np.zeros(360), rtol=1e-300, atol=0.0, maxiter=k, M=M)
        _close(res.x, xs, 1e-9, f"PCG iterate k={k}")


def pin_full_deflation(O):
    """One region per cell: E = A, P1 A = 0, so 0 iterations and x = A^-1 b."""
    grid = (5, 4, 3)
    K = _lognormal(60, 8)
    q = np.random.Generator(np.random.PCG64(9)).standard_normal(60)
    A, b = O.assemble(K, grid, XLO, q)
    Z = O.deflation_matrix(np.arange(60, dtype=np.int32), 60)
    res = O.dpcg(A, b, Z, tol=1e-12)
    assert res.iters == 0, res.iters
    _close(res.x, np.linalg.solve(A.toarray(), b), 1e-10, "x with d = n")


def pin_dense_direct(O):
    """Small heterogeneous problems: x agrees with a dense direct solve."""
    cases = (((8, 6, 4), (2, 2, 2), 1e6, 10), ((12, 12, 1), (3, 3, 1), 1e4, 11),
             ((10, 1, 1), (2, 1, 1), 1e8, 12), ((7, 5, 6), (1, 1, 3), 1e3, 13))
    for grid, nsub, contrast, seed in cases:
        nx, ny, nz = grid
        n = nx * ny * nz
        g = np.random.Generator(np.random.PCG64(seed))
        lay = (np.arange(nz if nz > 1 else ny) * 4) // (nz if nz > 1 else ny)
        mu = np.where(lay % 2 == 0, 1.0, 1.0 / contrast)
        if nz > 1:
            K = (mu[:, None, None] * np.exp(0.5 * g.standard_normal((nz, ny, nx)))).reshape(-1)
        else:
            K = (mu[:, None] * np.exp(0.5 * g.standard_normal((ny, nx)))).reshape(-1)
        q = g.standard_normal(n)
        A, b = O.assemble(K, grid, XLO, q)
        lab, d = O.levelset_labels(grid, K, nsub, np.array([1 / math.sqrt(contrast)]))
        res = O.dpcg(A, b, O.deflation_matrix(lab, d), tol=1e-13)
        xd = np.linalg.solve(A.toarray(), b)
        assert res.status == "ok" and res.relres <= 1e-12, (res.status, res.relres)
        err = np.linalg.norm(res.x - xd) / np.linalg.norm(xd)
        assert err <= 1e-7, f"direct mismatch {grid}: {err:.2e}"


def pin_projectors(O):
    """Definition 3.1 identities on a tiny grid (symmetric A): Z^T P1 = 0, P2 Z = 0,
    P1^2 = P1, P1 A = A P2, P1^T = P2, P1 A Z = 0; and the true residual of the
    projected solution equals the deflated residual P1 (b - A xhat)."""
    grid = (5, 4, 3)
    K = _lognormal(60, 14)
    A, _ = O.assemble(K, grid, XLO, np.zeros(60))
    lab, d = O.levelset_labels(grid, K, (2, 2, 1), np.array([1.0]))
    Z = O.deflation_matrix(lab, d)
    P1, P2, E = O.projectors(A, Z)
    Ad = A.toarray()
    Zd = Z.toarray()
    s = np.abs(Ad).max()
    for name, M, scale in (("Z^T P1", Zd.T @ P1, 1.0), ("P2 Z", P2 @ Zd, 1.0),
                           ("P1^2-P1", P1 @ P1 - P1, 1.0), ("P1A-AP2", P1 @ Ad - Ad @ P2, s),
                           ("P1^T-P2", P1.T - P2, 1.0), ("P1 A Z", P1 @ Ad @ Zd, s)):
        assert np.abs(M).max() <= 1e-9 * scale * 60, f"{name}: {np.abs(M).max():.2e}"
    b = np.random.Generator(np.random.PCG64(15)).standard_normal(60)
    res = O.dpcg(A, b, Z, tol=1e-6, maxit=4)
    _close(b - Ad @ res.x, P1 @ (b - Ad @ res.xhat), 1e-8, "b - A x = P1(b - A xhat)")


def pin_x0_independence(O):
    """P2 xhat is unique (Section 3.1), so x does not depend on the start vector, even one
    with arbitrary components in range(Z)."""
    grid = (8, 8, 4)
    K = _lognormal(256, 16)
    g = np.random.Generator(np.random.PCG64(17))
    A, b = O.assemble(K, grid, XLO, g.standard_normal(256))
    lab, d = O.levelset_labels(grid, K, (2, 2, 2), np.array([1.0]))
    Z = O.deflation_matrix(lab, d)
    x_a = O.dpcg(A, b, Z, tol=1e-12).x
    x0 = g.standard_normal(256) + Z @ (100 * g.standard_normal(d))
    x_b = O.dpcg(A, b, Z, x0=x0, tol=1e-12).x
    _close(x_b, x_a, 1e-8, "x0 independence")


def theorem21_count(O, layers: str, eps: float, nx: int = 6, rows: int = 3) -> int:
    """Number of eigenvalues of D^-1/2 A D^-1/2 below 100 eps for a 2D column of layers
    (bottom first; 'H' = 1, 'L' = eps), Dirichlet on top, Neumann elsewhere."""
    ny = rows * len(layers)
    K = np.repeat(np.array([1.0 if c == "H" else eps for c in layers]).repeat(rows), nx)
    A, _ = O.assemble(K, (nx, ny, 1), YHI, np.zeros(nx * ny))
    A = A.toarray()
    dg = np.sqrt(np.diag(A))
    ev = np.linalg.eigvalsh(A / dg[:, None] / dg[None, :])
    return int(np.sum(ev < 100 * eps))


def pin_theorem21(O):
    """Theorem 2.1: one O(eps) eigenvalue per high-permeability layer cut off from the
    Dirichlet boundary by low-permeability layers, for every small eps."""
    for layers, expect in (("HLH", 1), ("HLHLH", 2), ("LHLHL", 2), ("HLHLHLH", 3), ("LHLH", 1)):
        for eps in (1e-4, 1e-6, 1e-8):
            got = theorem21_count(O, layers, eps)
            assert got == expect, f"{layers} eps={eps}: {got} != {expect}"


def pin_jump_independence(O):
    """Deflated CG with layer-aligned regions needs about the same number of iterations
    at every contrast; plain Jacobi-PCG needs more as the contrast grows (Section 1).
    Set-up of Theorem 2.1 (Dirichlet on top, layers stacked in z), so the two high
    layers float and the undeflated matrix carries two O(1/contrast) eigenvalues."""
    grid = (16, 16, 16)
    it_d, it_p = [], []
    for contrast in (1e2, 1e4, 1e6):
        lay = (np.arange(16) * 4) // 16
        mu = np.where(lay % 2 == 0, 1.0, 1.0 / contrast)
        K = np.repeat(mu, 256)
        q = np.zeros(4096)
        q[0], q[-1] = 1.0, -1.0
        A, b = O.assemble(K, grid, ZHI, q)
        lab, d = O.levelset_labels(grid, K, (2, 2, 2), np.array([1 / math.sqrt(contrast)]))
        it_d.append(O.dpcg(A, b, O.deflation_matrix(lab, d), tol=1e-8).iters)
        Z0 = O.deflation_matrix(np.zeros(4096, dtype=np.int32), 0)
        it_p.append(O.dpcg(A, b, Z0, tol=1e-8, maxit=20000).iters)
    assert max(it_d) <= 1.10 * min(it_d), f"deflated iterations vary: {it_d}"
    assert it_p[-1] >= 1.2 * it_p[0] and min(it_p) >= 2 * max(it_d), f"plain {it_p} vs {it_d}"


ALL_PINS = [
    pin_row_sums, pin_symmetric_mmatrix, pin_second_difference, pin_series_resistance,
    pin_labels_bruteforce, pin_labels_layered2d, pin_components_bruteforce,
    pin_components_ndimage, pin_coarse_matrix, pin_textbook_pcg, pin_gmres_direct,
    pin_gmres_minimal_residual, pin_gmres_monotone, pin_gmres_poly_direct,
    pin_chebyshev_closed_form,
    pin_poly_degree_one_is_jacobi, pin_poly_direct,
    pin_full_deflation, pin_dense_direct, pin_projectors, pin_x0_independence,
    pin_theorem21, pin_jump_independence,
]
