"""CPU FP64 oracle for the subdomain-levelset (PSL) deflated PCG solve.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. The product (the HIP
library and its Python binding) never imports it and shares no code, table or
constant with it.

Everything here is plain NumPy/SciPy in float64, written for a reader to check
against the paper (arXiv 1510.02148, "The parallel subdomain-levelset deflation
method in reservoir simulation") by eye:

  * ``transmissibilities`` / ``pressure_matrix`` -- the finite-volume form of the
    pressure equation -div(lambda grad p) = q (Section 2, eq. "pressure") with
    lambda = K (single phase) and two-point harmonic-mean face transmissibilities.
  * ``levelset_labels`` -- subdomain-levelset deflation vectors: indicator
    vectors (Section 3.2, eq. "domdefl") of every (subdomain, permeability
    class) region (Section 3.2, subdomain-levelset figure; Vuik02 choice of
    vectors on both high and low layers). ``levelset_components`` splits each
    region into its connected components (a reading of the automatic
    construction Section 3.2 defers).
  * ``coarse_matrix`` -- E = Z^T A Z (Definition 3.1, eq. "E").
  * ``dpcg`` -- CG on the deflated system P1 A xhat = P1 b (eq. "defsys") with
    Jacobi preconditioning applied after P1 and E built from A itself
    (Remark 3.1), then the projection back x = Z E^-1 Z^T b + P2 xhat
    (eq. "projectback").
  * ``pdgmres`` -- the paper's own solver: right-preconditioned restarted GMRES
    on P1 A M^-1 with the a priori vectors (Algorithm 1, Section 3.2).
  * ``chebyshev_apply`` / ``dpcg_poly`` -- deflated CG with a Chebyshev polynomial
    preconditioner in place of Jacobi (a stronger preconditioner on the deflated
    system; the paper pairs the deflation with AMG, Section 1 and Section 5).
  * ``projectors`` -- dense P1 = I - A Z E^-1 Z^T and P2 = I - Z E^-1 Z^T A
    (eq. "deflops") for identity checks on tiny grids.

The paper gives no CG listing (its solvers are deflated GMRES); the CG form
used here is the symmetric case the paper builds on (Section 1: deflated CG
converges independently of the jump size; Section 3.1: P1^T = P2 when A is
symmetric). Stopping: ||rhat||_2 <= tol * ||b||_2, checked before every
iteration; one iteration = one product with A inside the loop.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# Dirichlet face-mask bits: p = 0 on the masked outer faces, Neumann elsewhere.
MASK_X_LO, MASK_X_HI, MASK_Y_LO, MASK_Y_HI, MASK_Z_LO, MASK_Z_HI = 1, 2, 4, 8, 16, 32


# ---------------------------------------------------------------------------
# Discretisation: two-point flux finite volumes on a unit-spacing grid
# (Section 2: "upstream finite-volume method"; single phase, lambda = K)
# ---------------------------------------------------------------------------

def _harmonic(Ka: np.ndarray, Kb: np.ndarray) -> np.ndarray:
    """Face transmissibility between two unit cells at unit distance:
    1 / (1/(2 Ka) + 1/(2 Kb)) = 2 Ka Kb / (Ka + Kb); zero when both are zero."""
    s = Ka + Kb
    out = np.zeros(np.broadcast(Ka, Kb).shape)
    nz = s > 0
    out[nz] = 2.0 * Ka[nz] * Kb[nz] / s[nz]
    return out


def transmissibilities(K: np.ndarray, grid, dirichlet_mask: int):
    """Face transmissibilities as three face arrays.

    Tx has shape (nz, ny, nx+1): face ix lies between cells ix-1 and ix.
    Ty has shape (nz, ny+1, nx), Tz has shape (nz+1, ny, nx), likewise.
    Interior faces: harmonic mean. Outer faces: 2 K_cell (half-cell distance to
    a p = 0 Dirichlet boundary) where the mask bit is set, else 0 (Neumann).
    Returned flat, float64.
    """
    nx, ny, nz = grid
    k = np.asarray(K, dtype=np.float64).reshape(nz, ny, nx)
    Tx = np.zeros((nz, ny, nx + 1))
    Ty = np.zeros((nz, ny + 1, nx))
    Tz = np.zeros((nz + 1, ny, nx))
    Tx[:, :, 1:nx] = _harmonic(k[:, :, :-1], k[:, :, 1:])
    Ty[:, 1:ny, :] = _harmonic(k[:, :-1, :], k[:, 1:, :])
    Tz[1:nz, :, :] = _harmonic(k[:-1, :, :], k[1:, :, :])
    if dirichlet_mask & MASK_X_LO:
        Tx[:, :, 0] = 2.0 * k[:, :, 0]
    if dirichlet_mask & MASK_X_HI:
        Tx[:, :, nx] = 2.0 * k[:, :, nx - 1]
    if dirichlet_mask & MASK_Y_LO:
        Ty[:, 0, :] = 2.0 * k[:, 0, :]
    if dirichlet_mask & MASK_Y_HI:
        Ty[:, ny, :] = 2.0 * k[:, ny - 1, :]
    if dirichlet_mask & MASK_Z_LO:
        Tz[0, :, :] = 2.0 * k[0, :, :]
    if dirichlet_mask & MASK_Z_HI:
        Tz[nz, :, :] = 2.0 * k[nz - 1, :, :]
    return Tx.reshape(-1), Ty.reshape(-1), Tz.reshape(-1)


def pressure_matrix(grid, Tx, Ty, Tz) -> sp.csr_matrix:
    """A with (A p)_i = sum over the faces f of cell i of T_f (p_i - p_nbr(f)),
    where p_nbr = 0 across an outer face. So A_ii = sum of the cell's face
    transmissibilities and A_ij = -T_f for the face shared with cell j."""
    nx, ny, nz = grid
    n = nx * ny * nz
    Tx = np.asarray(Tx).reshape(nz, ny, nx + 1)
    Ty = np.asarray(Ty).reshape(nz, ny + 1, nx)
    Tz = np.asarray(Tz).reshape(nz + 1, ny, nx)
    cell = np.arange(n).reshape(nz, ny, nx)
    diag = (Tx[:, :, :-1] + Tx[:, :, 1:] + Ty[:, :-1, :] + Ty[:, 1:, :]
            + Tz[:-1, :, :] + Tz[1:, :, :]).reshape(-1)
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [diag]
    # each interior face couples two cells symmetrically
    for a, b, t in ((cell[:, :, :-1], cell[:, :, 1:], Tx[:, :, 1:nx]),
                    (cell[:, :-1, :], cell[:, 1:, :], Ty[:, 1:ny, :]),
                    (cell[:-1, :, :], cell[1:, :, :], Tz[1:nz, :, :])):
        a, b, t = a.reshape(-1), b.reshape(-1), t.reshape(-1)
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def assemble(K, grid, dirichlet_mask: int, q) -> Tuple[sp.csr_matrix, np.ndarray]:
    """A and b = q (unit cell volume) for the pressure equation."""
    Tx, Ty, Tz = transmissibilities(K, grid, dirichlet_mask)
    return pressure_matrix(grid, Tx, Ty, Tz), np.asarray(q, dtype=np.float64).copy()


# ---------------------------------------------------------------------------
# Deflation space: subdomain-levelset indicator vectors (Section 3.2)
# ---------------------------------------------------------------------------

def subdomain_index(grid, nsub) -> np.ndarray:
    """Floor partition: subdomain coordinate along x is floor(ix * sx / nx), etc.;
    subdomain id = sub_x + sx * (sub_y + sy * sub_z)."""
    nx, ny, nz = grid
    sx, sy, sz = nsub
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    bx = (ix * sx) // nx
    by = (iy * sy) // ny
    bz = (iz * sz) // nz
    return (bx + sx * (by + sy * bz)).reshape(-1).astype(np.int64)


def levelset_class(K, thr) -> np.ndarray:
    """Permeability class = number of thresholds t with K >= t (ties go up)."""
    K = np.asarray(K, dtype=np.float64)
    c = np.zeros(K.shape, dtype=np.int64)
    for t in np.asarray(thr, dtype=np.float64):
        c += (K >= t)
    return c


def levelset_labels(grid, K, nsub, thr, cls=None, ncls=None) -> Tuple[np.ndarray, int]:
    """Column index of Z for every cell, and d = number of columns.

    One deflation vector per non-empty (subdomain, class) region: key =
    subdomain * ncls + class, and the label is the rank of the key among the
    keys that occur, so empty regions get no column and Z has full rank.
    With ``cls`` given the classes are taken from it (manual construction);
    otherwise they come from the permeability thresholds.
    """
    sub = subdomain_index(grid, nsub)
    if cls is None:
        c = levelset_class(K, thr)
        ncls = len(thr) + 1
    else:
        c = np.asarray(cls, dtype=np.int64)
        if ncls is None:
            ncls = int(c.max()) + 1
    key = sub * ncls + c
    present, labels = np.unique(key, return_inverse=True)
    return labels.astype(np.int32), int(present.size)


def levelset_components(grid, K, nsub, thr, cls=None, ncls=None) -> Tuple[np.ndarray, int]:
    """Automatic subdomain-levelset construction, connected-components reading.

    Section 3.2 draws every region as one connected piece and leaves an automatic
    construction for later. Here each non-empty (subdomain, class) region is split into
    its face-connected components (cells sharing a face: 6 neighbours in 3D, 4 in 2D),
    and every component is one deflation vector. Columns are ordered by the smallest
    cell index (c = ix + nx (iy + ny iz)) of their component. The components come from
    ``scipy.sparse.csgraph.connected_components`` on the graph whose edges join
    face neighbours with equal (subdomain, class) key.
    """
    from scipy.sparse.csgraph import connected_components
    nx, ny, nz = grid
    n = nx * ny * nz
    sub = subdomain_index(grid, nsub)
    if cls is None:
        c = levelset_class(K, thr)
        ncls = len(thr) + 1
    else:
        c = np.asarray(cls, dtype=np.int64)
        if ncls is None:
            ncls = int(c.max()) + 1
    key = (sub * ncls + c).reshape(nz, ny, nx)
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    rows, cols = [], []
    for axis in (2, 1, 0):                      # x, y, z neighbours
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[axis] = slice(0, -1)
        b[axis] = slice(1, None)
        same = key[tuple(a)] == key[tuple(b)]
        rows.append(idx[tuple(a)][same])
        cols.append(idx[tuple(b)][same])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    graph = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    ncomp, comp = connected_components(graph, directed=False)
    first = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(n, dtype=np.int64))
    order = np.empty(ncomp, dtype=np.int64)
    order[np.argsort(first, kind="stable")] = np.arange(ncomp)
    return order[comp].astype(np.int32), int(ncomp)


def deflation_matrix(labels, d) -> sp.csr_matrix:
    """Z (n x d): (z_j)_i = 1 if cell i belongs to region j, else 0 (eq. "domdefl")."""
    labels = np.asarray(labels)
    n = labels.size
    if d == 0:
        return sp.csr_matrix((n, 0))
    return sp.csr_matrix((np.ones(n), (np.arange(n), labels)), shape=(n, d))


def coarse_matrix(A, Z) -> np.ndarray:
    """E = Z^T A Z, dense (Definition 3.1)."""
    if Z.shape[1] == 0:
        return np.zeros((0, 0))
    return np.asarray((Z.T @ (A @ Z)).todense())


def projectors(A, Z):
    """Dense P1 = I - A Z E^-1 Z^T and P2 = I - Z E^-1 Z^T A (eq. "deflops")."""
    A = np.asarray(A.todense() if sp.issparse(A) else A)
    Z = np.asarray(Z.todense() if sp.issparse(Z) else Z)
    E = Z.T @ A @ Z
    Einv = np.linalg.inv(E)
    n = A.shape[0]
    P1 = np.eye(n) - A @ Z @ Einv @ Z.T
    P2 = np.eye(n) - Z @ Einv @ Z.T @ A
    return P1, P2, E


# ---------------------------------------------------------------------------
# Deflated preconditioned CG (DEF1 form) and projection back
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    x: np.ndarray            # x = Z E^-1 Z^T b + P2 xhat
    xhat: np.ndarray         # last iterate of the deflated system
    iters: int               # products with A inside the loop
    status: str              # "ok" | "maxit" | "breakdown" | "notspd" | "nonfinite"
    relres: float            # ||b - A x||_2 / ||b||_2 from a fresh product
    history: np.ndarray      # ||rhat_k||_2 for k = 0..iters
    zt_r_drift: float        # max_k ||Z^T rhat_k|| / ||rhat_k||


class Coarse:
    """E = Z^T A Z with its Cholesky factor; ``solve`` returns E^-1 s."""

    def __init__(self, A, Z):
        self.Z = Z
        self.E = coarse_matrix(A, Z)
        self.d = self.E.shape[0]
        self.ok = True
        self.factor = None
        if self.d:
            try:
                self.factor = sla.cho_factor(self.E, lower=True, check_finite=True)
            except (np.linalg.LinAlgError, ValueError):
                self.ok = False

    def solve(self, s):
        if self.d == 0:
            return np.zeros(0)
        return sla.cho_solve(self.factor, s)

    def correction(self, v):
        """Z E^-1 Z^T v (coarse-grid correction, prolongated)."""
        if self.d == 0:
            return np.zeros_like(v)
        return self.Z @ self.solve(self.Z.T @ v)


def dpcg(A, b, Z, x0=None, tol: float = 1e-8, maxit: int = 10000,
         coarse: Optional[Coarse] = None) -> Result:
    """Jacobi-preconditioned CG on P1 A xhat = P1 b, then x = xhat + Z E^-1 Z^T (b - A xhat).

    P1 v = v - A Z E^-1 Z^T v is applied with the factored E; M^-1 = diag(A)^-1
    acts on the deflated residual. E is built from A itself (Remark 3.1).
    """
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    if coarse is None:
        coarse = Coarse(A, Z)
    if not coarse.ok:
        return Result(np.zeros(n), np.zeros(n), 0, "notspd", np.inf, np.zeros(0), 0.0)
    dg = A.diagonal()
    if np.any(dg <= 0):
        return Result(np.zeros(n), np.zeros(n), 0, "notspd", np.inf, np.zeros(0), 0.0)
    bnorm = np.linalg.norm(b)
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)
    if not (np.all(np.isfinite(b)) and np.all(np.isfinite(x0))):
        return Result(np.zeros(n), np.zeros(n), 0, "nonfinite", np.nan, np.zeros(0), 0.0)
    if bnorm == 0.0:
        return Result(np.zeros(n), np.zeros(n), 0, "ok", 0.0, np.zeros(1), 0.0)

    def P1(v):
        return v - A @ coarse.correction(v)

    xhat = x0.copy()
    rhat = P1(b - A @ xhat)
    y = rhat / dg
    p = y.copy()
    rho = rhat @ y
    hist = [np.linalg.norm(rhat)]
    drift = 0.0
    status = "ok"
    it = 0
    while hist[-1] > tol * bnorm:
        if it >= maxit:
            status = "maxit"
            break
        q = A @ p
        w = P1(q)                      # w = P1 A p
        pw = p @ w
        if not pw > 0.0:
            status = "breakdown"
            break
        alpha = rho / pw
        xhat += alpha * p
        rhat -= alpha * w
        it += 1
        hist.append(np.linalg.norm(rhat))
        if coarse.d and hist[-1] > 0:
            drift = max(drift, np.linalg.norm(Z.T @ rhat) / hist[-1])
        y = rhat / dg
        rho_new = rhat @ y
        beta = rho_new / rho
        rho = rho_new
        p = y + beta * p
    x = xhat + coarse.correction(b - A @ xhat)
    relres = np.linalg.norm(b - A @ x) / bnorm
    return Result(x, xhat, it, status, relres, np.array(hist), drift)


def chebyshev_apply(A, r, degree: int, lmin: float, lmax: float):
    """y = q(D^-1 A) D^-1 r with D = diag(A): ``degree`` steps of the Chebyshev
    semi-iteration for A y = r with the Jacobi splitting, started from y = 0 and tuned to
    the interval [lmin, lmax] of the spectrum of D^-1 A (the three-term recurrence of the
    Chebyshev iteration, Saad, Iterative Methods for Sparse Linear Systems, Sec. 12.3).

    With theta, delta the interval's centre and half-width, the error after k steps is
    T_k((theta - lambda) / delta) / T_k(theta / delta) times the initial error on each
    eigenvector of D^-1 A; for lmax at or above the largest eigenvalue the operator
    r -> y is symmetric positive definite (a fixed preconditioner for CG). One step
    costs one product with A, the first none (y = D^-1 r / theta).
    """
    dg = A.diagonal()
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = (r / dg) / theta
    y = d.copy()
    for _ in range(degree - 1):
        res = r - A @ y
        rho_next = 1.0 / (2.0 * sigma - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * (res / dg)
        y = y + d
        rho = rho_next
    return y


def dpcg_poly(A, b, Z, degree: int = 3, ratio: float = 30.0, lmax: float = 2.0, x0=None,
              tol: float = 1e-8, maxit: int = 10000,
              coarse: Optional[Coarse] = None) -> Result:
    """Deflated CG (as ``dpcg``) with the Jacobi preconditioner replaced by the Chebyshev
    polynomial preconditioner ``chebyshev_apply`` on [lmax / ratio, lmax]: a stronger
    preconditioner on the deflated system in place of the paper's AMG (Section 1 and the
    SPE10 experiment pair the deflation with AMG applied to the deflated system).
    lmax = 2 bounds the spectrum of D^-1 A for these diagonally dominant matrices
    (Gershgorin). degree = 1 is Jacobi up to a scale, which CG does not see.
    """
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    if coarse is None:
        coarse = Coarse(A, Z)
    dg = A.diagonal()
    if not coarse.ok or np.any(dg <= 0):
        return Result(np.zeros(n), np.zeros(n), 0, "notspd", np.inf, np.zeros(0), 0.0)
    bnorm = np.linalg.norm(b)
    xhat = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    if bnorm == 0.0:
        return Result(np.zeros(n), np.zeros(n), 0, "ok", 0.0, np.zeros(1), 0.0)

    def P1(v):
        return v - A @ coarse.correction(v)

    def Minv(v):
        return chebyshev_apply(A, v, degree, lmax / ratio, lmax)

    rhat = P1(b - A @ xhat)
    y = Minv(rhat)
    p = y.copy()
    rho = rhat @ y
    hist = [np.linalg.norm(rhat)]
    status = "ok"
    it = 0
    while hist[-1] > tol * bnorm:
        if it >= maxit:
            status = "maxit"
            break
        w = P1(A @ p)
        pw = p @ w
        if not pw > 0.0:
            status = "breakdown"
            break
        alpha = rho / pw
        xhat += alpha * p
        rhat -= alpha * w
        it += 1
        hist.append(np.linalg.norm(rhat))
        y = Minv(rhat)
        rho_new = rhat @ y
        p = y + (rho_new / rho) * p
        rho = rho_new
    x = xhat + coarse.correction(b - A @ xhat)
    relres = np.linalg.norm(b - A @ x) / bnorm
    return Result(x, xhat, it, status, relres, np.array(hist), 0.0)


def pdgmres(A, b, Z, m: int = 30, x0=None, tol: float = 1e-8, maxit: int = 10000,
            coarse: Optional[Coarse] = None, degree: int = 1, ratio: float = 30.0,
            lmax: float = 2.0) -> Result:
    """The paper's deflated GMRES (Algorithm 1) with the subdomain-levelset vectors formed
    a priori (Section 3.2): restarted GMRES(m) with right preconditioning M = diag(A) on
    the deflated operator P1 A, then the projection back (eq. "projectback").

    Within a cycle the iterate minimises ||P1 (b - A x)||_2 over x0 + M^-1 K_j(P1 A M^-1,
    r0). Here the basis is kept orthonormal by classical Gram-Schmidt applied twice, the
    small least-squares problem is triangularised by one Givens rotation per step as the
    basis grows, and the residual norm of the minimiser is read from the rotated
    right-hand side (no solve needed to test convergence). A cycle ends on convergence
    (residual <= tol ||b||), on an invariant subspace (new basis direction of norm 0), or
    after m steps; the cycle's correction is M^-1 V y with y from the triangle.

    ``iters`` counts products with A inside the cycles; ``history`` holds the least-
    squares residual after every step (starting with ||r0||). degree >= 2 replaces
    M^-1 = diag(A)^-1 by the Chebyshev polynomial preconditioner ``chebyshev_apply`` on
    [lmax / ratio, lmax] (a stronger preconditioner on the deflated system, as the paper
    pairs the deflation with AMG).
    """
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    if coarse is None:
        coarse = Coarse(A, Z)
    dg = A.diagonal()
    if not coarse.ok or np.any(dg <= 0):
        return Result(np.zeros(n), np.zeros(n), 0, "notspd", np.inf, np.zeros(0), 0.0)
    bnorm = np.linalg.norm(b)
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)
    if bnorm == 0.0:
        return Result(np.zeros(n), np.zeros(n), 0, "ok", 0.0, np.zeros(1), 0.0)

    def P1(v):
        return v - A @ coarse.correction(v)

    def Minv(v):
        if degree <= 1:
            return v / dg
        return chebyshev_apply(A, v, degree, lmax / ratio, lmax)

    def op(v):                        # the right-preconditioned deflated operator
        return P1(A @ Minv(v))

    xm = x0.copy()
    it = 0
    hist = []
    status = "ok"
    goal = tol * bnorm
    while True:
        r0 = P1(b - A @ xm)
        beta = np.linalg.norm(r0)
        if not hist:
            hist.append(beta)
        if beta <= goal:
            break
        if it >= maxit:
            status = "maxit"
            break
        basis = [r0 / beta]
        R = np.zeros((m, m))          # triangular factor of the rotated Hessenberg matrix
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)           # rotated right-hand side beta e1
        g[0] = beta
        k = 0                         # steps taken in this cycle
        while k < m:
            w = op(basis[k])
            Vk = np.array(basis)      # (k + 1) x n
            h = Vk @ w
            w = w - Vk.T @ h
            h2 = Vk @ w               # second pass: reorthogonalisation
            w = w - Vk.T @ h2
            h = h + h2
            hnext = np.linalg.norm(w)
            it += 1
            # earlier rotations act on the new column; a new one zeroes its last entry
            for i in range(k):
                h[i], h[i + 1] = cs[i] * h[i] + sn[i] * h[i + 1], -sn[i] * h[i] + cs[i] * h[i + 1]
            rad = np.hypot(h[k], hnext)
            cs[k], sn[k] = (h[k] / rad, hnext / rad) if rad > 0.0 else (1.0, 0.0)
            R[:k + 1, k] = h[:k + 1]
            R[k, k] = rad
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            res = abs(g[k + 1])
            hist.append(res)
            k += 1
            if hnext == 0.0 or res <= goal or it >= maxit:
                break
            basis.append(w / hnext)
        y = sla.solve_triangular(R[:k, :k], g[:k], lower=False)
        xm = xm + Minv(np.array(basis[:k]).T @ y)
        if hist[-1] <= goal:
            break
    x = xm + coarse.correction(b - A @ xm)
    relres = np.linalg.norm(b - A @ x) / bnorm
    return Result(x, xm, it, status, relres, np.array(hist), 0.0)


def solve(K, grid, dirichlet_mask, q, nsub, thr, tol=1e-8, maxit=10000, x0=None,
          cls=None, ncls=None):
    """Whole path from the permeability field: A, labels, E, DEF1-PCG, projection back."""
    A, b = assemble(K, grid, dirichlet_mask, q)
    labels, d = levelset_labels(grid, K, nsub, thr, cls=cls, ncls=ncls)
    Z = deflation_matrix(labels, d)
    res = dpcg(A, b, Z, x0=x0, tol=tol, maxit=maxit)
    return res, labels, d, A, b


def relres(A, b, x) -> float:
    """||b - A x||_2 / ||b||_2 in float64."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    r = b - A @ np.asarray(x, dtype=np.float64)
    return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))
