"""psl_build_Z_noalloc (labels without device allocation, scratch in a fixed device array)
against psl_build_Z on the same inputs, through the C-ABI: bit-exact labels and equal d,
on two calls in a row with the second on a smaller input (the shared scratch keeps the
first call's contents and must not leak into the second), and its size limit."""
import ctypes

import numpy as np
import pytest

import psl_inputs as pi

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.gpu
def test_noalloc_labels_match_allocating_entry_point(gpu_lib):
    psl = gpu_lib
    big = pi.config("c2")                              # 128x128x64, 8x8x4 subdomains, d = 512
    small = pi.layered3d(37, 29, 11, nlayers=4, contrast=1e4, nsub=(5, 3, 2), seed=21,
                         wells="columns")              # ragged, fewer keys than the first call
    cases = [(big, None), (small, None)]
    g = np.random.Generator(np.random.PCG64(9))
    cls = g.integers(0, 3, size=small.n).astype(np.int32)
    cases.append((small, cls))                         # manual classes after threshold classes
    for p, c in cases:
        say(f"noalloc labels grid={p.grid} nsub={p.nsub} manual={c is not None}")
        K = dev(p.K)
        kw = dict(cls=dev(c, torch.int32), ncls=3) if c is not None else {}
        thr = None if c is not None else list(p.thr)
        ref, dref = psl.psl_build_Z(p.grid, K if c is None else None, p.nsub, thr, **kw)
        lab = torch.full((p.n,), -7, dtype=torch.int32, device="cuda")
        got, d = psl.psl_build_Z(p.grid, K if c is None else None, p.nsub, thr, labels=lab,
                                 noalloc=True, **kw)
        torch.cuda.synchronize()
        assert d == dref and torch.equal(got, ref)
    # a bad manual class is still reported after calls that left the scratch flag clear
    bad = cls.copy()
    bad[3] = 5
    with pytest.raises(psl.PslError) as ei:
        psl.psl_build_Z(small.grid, None, small.nsub, cls=dev(bad, torch.int32), ncls=3,
                        noalloc=True)
    assert ei.value.status == psl.EINVAL
    # and the next good call is not affected by the flag that call raised
    got, d = psl.psl_build_Z(small.grid, None, small.nsub, cls=dev(cls, torch.int32), ncls=3,
                             noalloc=True)
    ref, dref = psl.psl_build_Z(small.grid, None, small.nsub, cls=dev(cls, torch.int32), ncls=3)
    assert d == dref and torch.equal(got, ref)


def test_noalloc_key_limit_refused_before_device_work():
    """More (subdomain, class) keys than PSL_NOALLOC_MAX_KEYS: PSL_ENOTSUP, checked before
    any device work (runs without a GPU)."""
    from paper_1510_02148_amd import psl
    g = psl.psl_grid(1024, 1024, 2)
    ns = (ctypes.c_int32 * 3)(1024, 1024, 1)           # 2^20 subdomains x 1 class
    d = ctypes.c_int32(0)
    fake = ctypes.c_void_p(16)
    rc = psl._build_z_noalloc(ctypes.byref(g), fake, ns, None, 0, None, 0, fake, ctypes.byref(d),
                              None)
    assert rc == psl.ENOTSUP
