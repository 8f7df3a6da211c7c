"""Seeded synthetic workloads: reproducible, and with the structure each config names."""
import math

import numpy as np

import psl_inputs as pi


def test_reproducible():
    a = pi.config("c2", seed=3, scale=4)
    b = pi.config("c2", seed=3, scale=4)
    assert np.array_equal(a.K, b.K) and np.array_equal(a.q, b.q)
    c = pi.config("c2", seed=4, scale=4)
    assert not np.array_equal(a.K, c.K)


def test_layered2d_structure():
    p = pi.config("c1")
    assert p.grid == (64, 64, 1) and p.nsub == (4, 4, 1)
    k = p.K.reshape(64, 64)
    assert np.all(k[0:8] == 1.0) and np.all(k[8:16] == 1e-4) and np.all(k[56:64] == 1e-4)
    assert p.q[0] == 1.0 and p.q[-1] == -1.0 and abs(p.q.sum()) == 0.0


def test_layered3d_statistics():
    p = pi.layered3d(32, 32, 16, contrast=1e6, sigma_ln=1.0, seed=0)
    lnk = np.log(p.K).reshape(16, 32, 32)
    even = lnk[0:2].ravel()
    odd = lnk[2:4].ravel()
    assert abs(even.mean()) < 0.1 and abs(even.std() - 1) < 0.05
    assert abs(odd.mean() + math.log(1e6)) < 0.1


def test_channelized_fraction_and_contrast():
    p = pi.channelized(64, 64, 32, contrast=1e5, corr_len=8.0, seed=1)
    frac = np.mean(p.K >= p.thr[0])
    assert abs(frac - 0.30) < 0.01
    assert abs(p.meta["channel_frac"] - 0.30) < 0.01


def test_batch_sizes_and_wells():
    sys = pi.batch(nsys=16, seed=0)
    sides = [s.grid[0] for s in sys]
    assert all(32 <= s <= 96 for s in sides) and len(set(sides)) > 4
    for s in sys:
        assert abs(s.q.sum()) < 1e-12 and s.q.max() > 0 and s.q.min() < 0
        assert s.nsub == (4, 4, 4)
