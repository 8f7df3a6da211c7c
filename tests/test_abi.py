"""The C-ABI library loads on a machine without a GPU and exports every entry point that
include/psl.h declares; the ctypes structs match the C layout (checked with gcc)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psl.h")
LIB = os.path.join(ROOT, "paper_1510_02148_amd", "libpsl.so")


def declared_functions():
    import glob
    src = "\n".join(open(h).read() for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(psl_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("psl_build_Z", "psl_setup_E", "psl_solve", "psl_solve_batched",
                 "psl_assemble_tpfa", "psl_destroy", "psl_status_str"):
        assert must in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpsl.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu(lib):
    lib.psl_status_str.restype = ctypes.c_char_p
    assert lib.psl_status_str(0) == b"ok"
    assert b"positive definite" in lib.psl_status_str(-4)
    assert lib.psl_status_str(12345) == b"unknown status"


def test_binding_struct_layout_matches_c(tmp_path):
    from paper_1510_02148_amd import psl
    prog = tmp_path / "sz.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "psl.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(psl_solve_opts),"
        " sizeof(psl_solve_stats), offsetof(psl_solve_opts, tau_inner),"
        " offsetof(psl_solve_opts, check_every), offsetof(psl_solve_opts, mixed_floor),"
        " offsetof(psl_solve_stats, relres_true), sizeof(psl_grid), sizeof(psl_setup_opts),"
        " sizeof(psl_gmres_opts), offsetof(psl_gmres_opts, use_x0), sizeof(psl_poly_opts),"
        " offsetof(psl_poly_opts, degree), offsetof(psl_poly_opts, check_every),"
        " offsetof(psl_poly_opts, mixed), offsetof(psl_gmres_opts, degree));"
        "printf(\"%zu\\n\", offsetof(psl_solve_stats, zt_r_drift));"
        "printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(psl_ctx_info), offsetof(psl_ctx_info, coarse_sym),"
        " offsetof(psl_ctx_info, small_solve), offsetof(psl_ctx_info, face_tables),"
        " offsetof(psl_ctx_info, wide_tiles));"
        "printf(\"%zu\\n\", offsetof(psl_setup_opts, wide_tiles));"
        "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(psl.psl_solve_opts), ctypes.sizeof(psl.psl_solve_stats),
            psl.psl_solve_opts.tau_inner.offset, psl.psl_solve_opts.check_every.offset,
            psl.psl_solve_opts.mixed_floor.offset, psl.psl_solve_stats.relres_true.offset,
            ctypes.sizeof(psl.psl_grid), ctypes.sizeof(psl.psl_setup_opts),
            ctypes.sizeof(psl.psl_gmres_opts), psl.psl_gmres_opts.use_x0.offset,
            ctypes.sizeof(psl.psl_poly_opts), psl.psl_poly_opts.degree.offset,
            psl.psl_poly_opts.check_every.offset, psl.psl_poly_opts.mixed.offset,
            psl.psl_gmres_opts.degree.offset, psl.psl_solve_stats.zt_r_drift.offset,
            ctypes.sizeof(psl.psl_ctx_info), psl.psl_ctx_info.coarse_sym.offset,
            psl.psl_ctx_info.small_solve.offset, psl.psl_ctx_info.face_tables.offset,
            psl.psl_ctx_info.wide_tiles.offset, psl.psl_setup_opts.wide_tiles.offset]
    assert got == want


def test_default_opts(lib):
    from paper_1510_02148_amd import psl
    o = psl.default_opts()
    assert o.tol == 1e-8 and o.maxit == 10000 and o.mode == psl.FP64 and o.check_every == 16
    assert o.tau_inner == 0.01 and o.reproject == -1 and o.mixed_floor == 1e-7


def test_default_gmres_opts(lib):
    from paper_1510_02148_amd import psl
    o = psl.psl_gmres_opts()
    psl._default_gmres_opts(ctypes.byref(o))
    assert o.tol == 1e-8 and o.maxit == 10000 and o.restart == 30 and o.use_x0 == 0
    assert o.degree == 0 and list(o.reserved) == [0, 0]


def test_default_poly_opts(lib):
    from paper_1510_02148_amd import psl
    o = psl.psl_poly_opts()
    psl._default_poly_opts(ctypes.byref(o))
    assert o.tol == 1e-8 and o.ratio == 30.0 and o.lmax == 2.0 and o.degree == 3
    assert o.maxit == 10000 and o.use_x0 == 0 and o.check_every == 16 and o.mixed == 0
    assert list(o.reserved) == [0]


def test_invalid_arguments_rejected_before_any_device_work(lib):
    from paper_1510_02148_amd import psl
    # null pointers and bad sizes return PSL_EINVAL without touching the device
    g = psl.psl_grid(0, 4, 4)
    rc = psl._assemble(ctypes.byref(g), None, 1, None, None, None, None)
    assert rc == psl.EINVAL
    out = ctypes.c_void_p(0)
    g = psl.psl_grid(4, 4, 4)
    rc = psl._setup_e(ctypes.byref(out), ctypes.byref(g), None, None, None, None, 3, None, None)
    assert rc == psl.EINVAL and not out.value
    d = ctypes.c_int32(0)
    ns = (ctypes.c_int32 * 3)(9, 1, 1)  # more subdomains than cells along x
    rc = psl._build_z(ctypes.byref(g), ctypes.c_void_p(16), ns, None, 0, None, 0,
                      ctypes.c_void_p(16), ctypes.byref(d), None)
    assert rc == psl.EINVAL
    assert psl._solve(None, None, None, None, None, None) == psl.EINVAL
    assert psl._solve_gmres(None, None, None, None, None, None) == psl.EINVAL
    assert psl._solve_poly(None, None, None, None, None, None) == psl.EINVAL
    rc = psl._build_z_cc(ctypes.byref(g), ctypes.c_void_p(16), ns, None, 0, None, 0,
                         ctypes.c_void_p(16), ctypes.byref(d), None)
    assert rc == psl.EINVAL


def test_batched_rejects_bad_arguments_without_device_work(lib):
    from paper_1510_02148_amd import psl
    st = (psl.psl_solve_stats * 1)()
    assert psl._solve_batched(None, 1, None, None, None, st, None) == psl.EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert psl._solve_batched(arr, 0, arr, arr, None, st, None) == psl.EINVAL
    assert psl._solve_batched(arr, 1, arr, arr, None, st, None) == psl.EINVAL


def test_grids_above_the_cell_limit_refused_before_device_work(lib):
    """Grids whose cell count or a face-array length exceeds PSL_MAX_CELLS (2^29 - 1) are
    refused with PSL_ENOTSUP by every entry point that takes a grid, before any device
    work (the solve kernels form float64 byte offsets in 32 bits)."""
    from paper_1510_02148_amd import psl
    src = open(HEADER).read()
    lim = int(re.search(r"#define PSL_MAX_CELLS\s+(\d+)", src).group(1))
    assert lim == 2**29 - 1
    fake = ctypes.c_void_p(16)   # never dereferenced: the size check comes first
    d = ctypes.c_int32(0)
    ns = (ctypes.c_int32 * 3)(1, 1, 1)
    out = ctypes.c_void_p(0)
    for g in (psl.psl_grid(1024, 1024, 512),        # 2^29 cells
              psl.psl_grid(2**29 - 1, 1, 1),        # cells at the limit, x faces above it
              psl.psl_grid(1, 2**29 - 1, 1),        # y faces above the limit
              psl.psl_grid(1, 1, 2**29 - 1)):       # z faces above the limit
        assert psl._assemble(ctypes.byref(g), fake, 1, fake, fake, fake, None) == psl.ENOTSUP
        assert psl._build_z(ctypes.byref(g), fake, ns, None, 0, None, 0, fake,
                            ctypes.byref(d), None) == psl.ENOTSUP
        assert psl._build_z_cc(ctypes.byref(g), fake, ns, None, 0, None, 0, fake,
                               ctypes.byref(d), None) == psl.ENOTSUP
        rc = psl._setup_e(ctypes.byref(out), ctypes.byref(g), fake, fake, fake, fake, 3, None,
                          None)
        assert rc == psl.ENOTSUP and not out.value
