"""Thin ctypes binding of libpsl (include/psl.h): argument marshalling only.

Every function here forwards device pointers of torch tensors, host scalars and the
current HIP stream to the C-ABI entry point of the same name. All arithmetic happens
in the library's HIP kernels; there is no host or CPU fallback. Importing this module
without the built library raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libpsl.so not found at {LIB_PATH}; build it with "
        "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

# ---- status codes and constants (mirrors include/psl.h) ----------------------------------
OK, EINVAL, ENOMEM, EHIP, ENOTSPD, EMAXIT, EBREAKDOWN, ENONFINITE, ESTAGNATION, ENOTSUP = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
DIRICHLET_X_LO, DIRICHLET_X_HI, DIRICHLET_Y_LO, DIRICHLET_Y_HI, DIRICHLET_Z_LO, DIRICHLET_Z_HI = (
    1, 2, 4, 8, 16, 32)
FP64, MIXED = 0, 1
MAX_THRESHOLDS = 15
MAX_DENSE_D = 8192
MAX_TILE_LABELS = 16


class psl_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class psl_setup_opts(ctypes.Structure):
    _fields_ = [("tile_cells", ctypes.c_int32), ("finish_kernels", ctypes.c_int32),
                ("coarse_sym", ctypes.c_int32), ("stencil_split", ctypes.c_int32),
                ("face_tables", ctypes.c_int32), ("wide_tiles", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class psl_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("tau_inner", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("reproject", ctypes.c_int32), ("mixed_floor", ctypes.c_double)]


class psl_ctx_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("ntiles", ctypes.c_int32),
                ("m_faces", ctypes.c_int64), ("nslot_max", ctypes.c_int32),
                ("coarse_sym", ctypes.c_int32), ("small_solve", ctypes.c_int32),
                ("face_tables", ctypes.c_int32), ("wide_tiles", ctypes.c_int32)]


class psl_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer", ctypes.c_int32), ("status", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("relres_true", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("zt_r_drift", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class psl_gmres_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class psl_poly_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("ratio", ctypes.c_double), ("lmax", ctypes.c_double),
                ("degree", ctypes.c_int32), ("maxit", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I32P = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_assemble = _sig("psl_assemble_tpfa", ctypes.c_int,
                 [ctypes.POINTER(psl_grid), _P, ctypes.c_uint32, _P, _P, _P, _P])
_build_z = _sig("psl_build_Z", ctypes.c_int,
                [ctypes.POINTER(psl_grid), _P, _I32P, _DP, _I32, _P, _I32, _P, _I32P, _P])
_build_z_cc = _sig("psl_build_Z_cc", ctypes.c_int,
                   [ctypes.POINTER(psl_grid), _P, _I32P, _DP, _I32, _P, _I32, _P, _I32P, _P])
_build_z_noalloc = _sig("psl_build_Z_noalloc", ctypes.c_int,
                        [ctypes.POINTER(psl_grid), _P, _I32P, _DP, _I32, _P, _I32, _P, _I32P,
                         _P])
_setup_e = _sig("psl_setup_E", ctypes.c_int,
                [ctypes.POINTER(_P), ctypes.POINTER(psl_grid), _P, _P, _P, _P, _I32, _I32P, _P])
_setup_e_ex = _sig("psl_setup_E_ex", ctypes.c_int,
                   [ctypes.POINTER(_P), ctypes.POINTER(psl_grid), _P, _P, _P, _P, _I32, _I32P,
                    ctypes.POINTER(psl_setup_opts), _P])
_default_setup_opts = _sig("psl_default_setup_opts", None, [ctypes.POINTER(psl_setup_opts)])
_solve = _sig("psl_solve", ctypes.c_int,
              [_P, _P, _P, ctypes.POINTER(psl_solve_opts), ctypes.POINTER(psl_solve_stats), _P])
_solve_batched = _sig("psl_solve_batched", ctypes.c_int,
                      [ctypes.POINTER(_P), _I32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                       ctypes.POINTER(psl_solve_opts), ctypes.POINTER(psl_solve_stats), _P])
_apply_a = _sig("psl_apply_A", ctypes.c_int, [_P, _P, _P, _P])
_deflate = _sig("psl_deflate", ctypes.c_int, [_P, _P, _P, _P, _P])
_get_coarse = _sig("psl_get_coarse", ctypes.c_int, [_P, _P, _P, _I32P, _P])
_destroy = _sig("psl_destroy", None, [_P])
_get_info = _sig("psl_get_info", ctypes.c_int, [_P, ctypes.POINTER(psl_ctx_info)])
_bench_kernel = _sig("psl_bench_kernel", ctypes.c_int, [_P, _I32, _I32, _I32, _P])
_bench_copy = _sig("psl_bench_copy", ctypes.c_int, [_P, _P, ctypes.c_int64, _P])
_profile_kernel = _sig("psl_profile_kernel", ctypes.c_int, [_P, _I32, _I32, _I32])
_profile_read = _sig("psl_profile_read", ctypes.c_int,
                     [_P, _I32P, ctypes.POINTER(ctypes.c_float), _I32, _P])
_status_str = _sig("psl_status_str", ctypes.c_char_p, [ctypes.c_int])
_default_opts = _sig("psl_default_opts", None, [ctypes.POINTER(psl_solve_opts)])
_default_gmres_opts = _sig("psl_default_gmres_opts", None, [ctypes.POINTER(psl_gmres_opts)])
_solve_gmres = _sig("psl_solve_gmres", ctypes.c_int,
                    [_P, _P, _P, ctypes.POINTER(psl_gmres_opts), ctypes.POINTER(psl_solve_stats), _P])
_default_poly_opts = _sig("psl_default_poly_opts", None, [ctypes.POINTER(psl_poly_opts)])
_solve_poly = _sig("psl_solve_poly", ctypes.c_int,
                   [_P, _P, _P, ctypes.POINTER(psl_poly_opts), ctypes.POINTER(psl_solve_stats), _P])

EXPORTED = ("psl_assemble_tpfa", "psl_build_Z", "psl_build_Z_cc", "psl_build_Z_noalloc", "psl_setup_E", "psl_setup_E_ex",
            "psl_default_setup_opts", "psl_solve",
            "psl_solve_batched", "psl_apply_A",
            "psl_deflate", "psl_get_coarse", "psl_destroy", "psl_status_str",
            "psl_default_opts", "psl_bench_kernel", "psl_bench_copy", "psl_get_info",
            "psl_profile_kernel", "psl_profile_read",
            "psl_solve_gmres", "psl_default_gmres_opts", "psl_solve_poly",
            "psl_default_poly_opts")
(KERNEL_STENCIL, KERNEL_COARSE, KERNEL_UPDATE, KERNEL_DIRECTION, KERNEL_OUTER_RESIDUAL,
 KERNEL_GMRES_PASS, KERNEL_POLY_STEP, KERNEL_SMALL_SOLVE) = range(8)


class PslError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {psl_status_str(status)} ({status})")


def psl_status_str(status: int) -> str:
    return _status_str(int(status)).decode()


def _check(status: int, where: str):
    if status != OK:
        raise PslError(status, where)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, n: Optional[int] = None, name: str = "") -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous {dtype} tensor, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _grid(grid: Sequence[int]) -> psl_grid:
    nx, ny, nz = (int(v) for v in grid)
    return psl_grid(nx, ny, nz)


def face_counts(grid: Sequence[int]) -> Tuple[int, int, int]:
    nx, ny, nz = (int(v) for v in grid)
    return (nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)


def psl_assemble_tpfa(grid, K: torch.Tensor, dirichlet_mask: int,
                      Tx: Optional[torch.Tensor] = None, Ty: Optional[torch.Tensor] = None,
                      Tz: Optional[torch.Tensor] = None):
    """Face transmissibilities (float64 device tensors), allocated when not given."""
    n = int(grid[0]) * int(grid[1]) * int(grid[2])
    fx, fy, fz = face_counts(grid)
    dev = K.device
    Tx = torch.empty(fx, dtype=torch.float64, device=dev) if Tx is None else Tx
    Ty = torch.empty(fy, dtype=torch.float64, device=dev) if Ty is None else Ty
    Tz = torch.empty(fz, dtype=torch.float64, device=dev) if Tz is None else Tz
    g = _grid(grid)
    _check(_assemble(ctypes.byref(g), _dev(K, torch.float64, n, "K"), int(dirichlet_mask),
                     _dev(Tx, torch.float64, fx, "Tx"), _dev(Ty, torch.float64, fy, "Ty"),
                     _dev(Tz, torch.float64, fz, "Tz"), _stream()), "psl_assemble_tpfa")
    return Tx, Ty, Tz


def psl_build_Z(grid, K: Optional[torch.Tensor], nsub, thr=None, cls: Optional[torch.Tensor] = None,
                ncls: int = 0, labels: Optional[torch.Tensor] = None, components: bool = False,
                noalloc: bool = False):
    """Subdomain-levelset labels (int32 device tensor) and d; components=True splits every
    region into its connected components (psl_build_Z_cc); noalloc=True calls
    psl_build_Z_noalloc (no device allocation inside the library; pass `labels` to keep the
    call free of allocation on the Python side too)."""
    if components and noalloc:
        raise ValueError("psl_build_Z: noalloc has no connected-components form")
    n = int(grid[0]) * int(grid[1]) * int(grid[2])
    dev = (K if K is not None else cls).device
    labels = torch.empty(n, dtype=torch.int32, device=dev) if labels is None else labels
    g = _grid(grid)
    ns = (ctypes.c_int32 * 3)(*[int(v) for v in nsub])
    thr = [] if thr is None else [float(t) for t in thr]
    th = (ctypes.c_double * max(1, len(thr)))(*thr)
    d = ctypes.c_int32(0)
    kp = _dev(K, torch.float64, n, "K") if K is not None else ctypes.c_void_p(0)
    cp = _dev(cls, torch.int32, n, "cls") if cls is not None else ctypes.c_void_p(0)
    fn, name = ((_build_z_cc, "psl_build_Z_cc") if components else
                (_build_z_noalloc, "psl_build_Z_noalloc") if noalloc else
                (_build_z, "psl_build_Z"))
    _check(fn(ctypes.byref(g), kp, ns, th, len(thr), cp, int(ncls),
              _dev(labels, torch.int32, n, "labels"), ctypes.byref(d), _stream()), name)
    return labels, int(d.value)


class Context:
    """Owns a psl_ctx (E, its factor and inverse, work space); freed with the object."""

    def __init__(self, ptr: int, grid, d: int):
        self._ptr = ctypes.c_void_p(ptr)
        self.grid = tuple(int(v) for v in grid)
        self.n = self.grid[0] * self.grid[1] * self.grid[2]
        self.d = d

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._ptr:
            raise RuntimeError("context already destroyed")
        return self._ptr

    def destroy(self):
        if self._ptr:
            _destroy(self._ptr)
            self._ptr = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def psl_setup_E(grid, Tx: torch.Tensor, Ty: torch.Tensor, Tz: torch.Tensor,
                labels: torch.Tensor, d: int, nsub=None, tile_cells: Optional[int] = None,
                finish_kernels: int = 0, coarse_sym: int = 0,
                stencil_split: int = 0, face_tables: int = 0,
                wide_tiles: int = 0) -> Context:
    """psl_setup_E, or psl_setup_E_ex when a tile size, the finish-kernel, coarse-product,
    stencil-split, face-table or wide-tile choice is given."""
    n = int(grid[0]) * int(grid[1]) * int(grid[2])
    fx, fy, fz = face_counts(grid)
    g = _grid(grid)
    out = ctypes.c_void_p(0)
    ns = (ctypes.c_int32 * 3)(*[int(v) for v in nsub]) if nsub is not None else None
    args = (ctypes.byref(out), ctypes.byref(g), _dev(Tx, torch.float64, fx, "Tx"),
            _dev(Ty, torch.float64, fy, "Ty"), _dev(Tz, torch.float64, fz, "Tz"),
            _dev(labels, torch.int32, n, "labels"), int(d),
            ns if ns is not None else ctypes.cast(None, _I32P))
    if (tile_cells is None and not finish_kernels and not coarse_sym and not stencil_split
            and not face_tables and not wide_tiles):
        _check(_setup_e(*args, _stream()), "psl_setup_E")
    else:
        so = psl_setup_opts()
        _default_setup_opts(ctypes.byref(so))
        so.tile_cells = int(tile_cells or 0)
        so.finish_kernels = int(finish_kernels)
        so.coarse_sym = int(coarse_sym)
        so.stencil_split = int(stencil_split)
        so.face_tables = int(face_tables)
        so.wide_tiles = int(wide_tiles)
        _check(_setup_e_ex(*args, ctypes.byref(so), _stream()), "psl_setup_E_ex")
    return Context(out.value, grid, int(d))


def default_opts() -> psl_solve_opts:
    o = psl_solve_opts()
    _default_opts(ctypes.byref(o))
    return o


def psl_solve(ctx: Context, b: torch.Tensor, x: Optional[torch.Tensor] = None, *,
              tol: Optional[float] = None, maxit: Optional[int] = None, mode: int = FP64,
              use_x0: bool = False, max_outer: Optional[int] = None,
              tau_inner: Optional[float] = None, check_every: Optional[int] = None,
              reproject: Optional[int] = None, mixed_floor: Optional[float] = None,
              check: bool = False):
    """Solve A x = b; returns (x, stats dict). Non-zero status raises only if check=True."""
    o = default_opts()
    if tol is not None:
        o.tol = tol
    if maxit is not None:
        o.maxit = maxit
    o.mode = int(mode)
    o.use_x0 = 1 if use_x0 else 0
    if max_outer is not None:
        o.max_outer = max_outer
    if tau_inner is not None:
        o.tau_inner = tau_inner
    if check_every is not None:
        o.check_every = check_every
    if reproject is not None:
        o.reproject = int(reproject)
    if mixed_floor is not None:
        o.mixed_floor = float(mixed_floor)
    if x is None:
        if use_x0:
            raise ValueError("use_x0 needs x")
        x = torch.empty_like(b)
    st = psl_solve_stats()
    rc = _solve(ctx.handle, _dev(b, torch.float64, ctx.n, "b"), _dev(x, torch.float64, ctx.n, "x"),
                ctypes.byref(o), ctypes.byref(st), _stream())
    if check:
        _check(rc, "psl_solve")
    stats = st.as_dict()
    stats["status_str"] = psl_status_str(rc)
    return x, stats


def psl_solve_gmres(ctx: Context, b: torch.Tensor, x: Optional[torch.Tensor] = None, *,
                    tol: Optional[float] = None, maxit: Optional[int] = None,
                    restart: Optional[int] = None, use_x0: bool = False, degree: int = 0,
                    check: bool = False):
    """The paper's deflated right-preconditioned GMRES(m) (degree >= 2: with the Chebyshev
    polynomial preconditioner); returns (x, stats dict)."""
    o = psl_gmres_opts()
    _default_gmres_opts(ctypes.byref(o))
    if tol is not None:
        o.tol = tol
    if maxit is not None:
        o.maxit = maxit
    if restart is not None:
        o.restart = restart
    o.degree = int(degree)
    o.use_x0 = 1 if use_x0 else 0
    if x is None:
        if use_x0:
            raise ValueError("use_x0 needs x")
        x = torch.empty_like(b)
    st = psl_solve_stats()
    rc = _solve_gmres(ctx.handle, _dev(b, torch.float64, ctx.n, "b"),
                      _dev(x, torch.float64, ctx.n, "x"), ctypes.byref(o), ctypes.byref(st),
                      _stream())
    if check:
        _check(rc, "psl_solve_gmres")
    stats = st.as_dict()
    stats["status_str"] = psl_status_str(rc)
    return x, stats


def psl_solve_poly(ctx: Context, b: torch.Tensor, x: Optional[torch.Tensor] = None, *,
                   tol: Optional[float] = None, degree: Optional[int] = None,
                   ratio: Optional[float] = None, lmax: Optional[float] = None,
                   maxit: Optional[int] = None, check_every: Optional[int] = None,
                   use_x0: bool = False, mixed: bool = False, check: bool = False):
    """Deflated CG with the Chebyshev polynomial preconditioner (mixed: float32 inner
    solves in float64 refinement); returns (x, stats dict)."""
    o = psl_poly_opts()
    _default_poly_opts(ctypes.byref(o))
    for name, val in (("tol", tol), ("degree", degree), ("ratio", ratio), ("lmax", lmax),
                      ("maxit", maxit), ("check_every", check_every)):
        if val is not None:
            setattr(o, name, val)
    o.use_x0 = 1 if use_x0 else 0
    o.mixed = 1 if mixed else 0
    if x is None:
        if use_x0:
            raise ValueError("use_x0 needs x")
        x = torch.empty_like(b)
    st = psl_solve_stats()
    rc = _solve_poly(ctx.handle, _dev(b, torch.float64, ctx.n, "b"),
                     _dev(x, torch.float64, ctx.n, "x"), ctypes.byref(o), ctypes.byref(st),
                     _stream())
    if check:
        _check(rc, "psl_solve_poly")
    stats = st.as_dict()
    stats["status_str"] = psl_status_str(rc)
    return x, stats


def psl_solve_batched(ctxs, bs, xs=None, *, tol: Optional[float] = None,
                      maxit: Optional[int] = None, use_x0: bool = False,
                      check_every: Optional[int] = None, check: bool = False,
                      mode: int = FP64):
    """Solve independent systems A_i x_i = b_i together (float64 CG, or float32 refinement
    steps then float64 with mode=MIXED; one launch per kernel for all systems). Returns
    (xs, [stats dict per system], overall status)."""
    n = len(ctxs)
    if n < 1 or len(bs) != n or (xs is not None and len(xs) != n):
        raise ValueError("need one b (and x) per context")
    o = default_opts()
    o.mode = int(mode)
    if tol is not None:
        o.tol = tol
    if maxit is not None:
        o.maxit = maxit
    o.use_x0 = 1 if use_x0 else 0
    if check_every is not None:
        o.check_every = check_every
    if xs is None:
        if use_x0:
            raise ValueError("use_x0 needs xs")
        xs = [torch.empty_like(b) for b in bs]
    handles = (_P * n)(*[c.handle.value for c in ctxs])
    bp = (_P * n)(*[_dev(b, torch.float64, c.n, "b") for b, c in zip(bs, ctxs)])
    xp = (_P * n)(*[_dev(x, torch.float64, c.n, "x") for x, c in zip(xs, ctxs)])
    st = (psl_solve_stats * n)()
    rc = _solve_batched(handles, n, bp, xp, ctypes.byref(o), st, _stream())
    if check:
        _check(rc, "psl_solve_batched")
    stats = []
    for i in range(n):
        d = st[i].as_dict()
        d["status_str"] = psl_status_str(d["status"])
        stats.append(d)
    return xs, stats, rc


def psl_apply_A(ctx: Context, p: torch.Tensor, q: Optional[torch.Tensor] = None) -> torch.Tensor:
    q = torch.empty_like(p) if q is None else q
    _check(_apply_a(ctx.handle, _dev(p, torch.float64, ctx.n, "p"),
                    _dev(q, torch.float64, ctx.n, "q"), _stream()), "psl_apply_A")
    return q


def psl_deflate(ctx: Context, r: torch.Tensor, out: Optional[torch.Tensor] = None,
                c: Optional[torch.Tensor] = None):
    """out = P1 r and c = E^-1 Z^T r."""
    out = torch.empty_like(r) if out is None else out
    c = torch.empty(ctx.d, dtype=torch.float64, device=r.device) if c is None else c
    _check(_deflate(ctx.handle, _dev(r, torch.float64, ctx.n, "r"),
                    _dev(out, torch.float64, ctx.n, "out"), _dev(c, torch.float64, ctx.d, "c"),
                    _stream()), "psl_deflate")
    return out, c


def psl_get_coarse(ctx: Context, device="cuda"):
    """(E, E^-1) as d x d float64 device tensors."""
    d = ctx.d
    E = torch.empty((d, d), dtype=torch.float64, device=device)
    Einv = torch.empty((d, d), dtype=torch.float64, device=device)
    dd = ctypes.c_int32(0)
    _check(_get_coarse(ctx.handle, _dev(E, torch.float64, d * d, "E"),
                       _dev(Einv, torch.float64, d * d, "Einv"), ctypes.byref(dd), _stream()),
           "psl_get_coarse")
    return E, Einv


def psl_get_info(ctx: Context) -> dict:
    info = psl_ctx_info()
    _check(_get_info(ctx.handle, ctypes.byref(info)), "psl_get_info")
    return {k: getattr(info, k) for k, _ in info._fields_ if k != "reserved"}


def psl_bench_kernel(ctx: Context, kernel: int, mode: int, reps: int):
    _check(_bench_kernel(ctx.handle, int(kernel), int(mode), int(reps), _stream()),
           "psl_bench_kernel")


def psl_bench_copy(src: torch.Tensor, dst: torch.Tensor):
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("psl_bench_copy: src and dst must be device tensors of equal size")
    _check(_bench_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                       nbytes, _stream()), "psl_bench_copy")


def psl_destroy(ctx: Context):
    ctx.destroy()


def psl_profile_kernel(ctx, kernel: int, mode: int, max_launches: int = 4096):
    """Arm per-launch event timing of one CG kernel (KERNEL_STENCIL, KERNEL_COARSE,
    KERNEL_UPDATE, or KERNEL_SMALL_SOLVE in FP64) in the precision of `mode` for the
    following solves; kernel < 0 disarms."""
    _check(_profile_kernel(ctx.handle, int(kernel), int(mode), int(max_launches)),
           "psl_profile_kernel")


def psl_profile_read(ctx, max_launches: int = 4096):
    """Durations (microseconds, launch order) of the launches timed since arming or the last
    read, as a list of floats."""
    n = ctypes.c_int32(0)
    buf = (ctypes.c_float * max(1, int(max_launches)))()
    _check(_profile_read(ctx.handle, ctypes.byref(n), buf, int(max_launches), _stream()),
           "psl_profile_read")
    return [float(buf[i]) for i in range(min(n.value, int(max_launches)))]
