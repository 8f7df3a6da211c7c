"""Pins of the start-vector network's float64 reference against independent facts:
library correlation and bfloat16 conversion, adjoint identities, finite differences, the
closed-form optimum of the energy loss, and the documented behaviour of Adam. Each pin
takes the module under test (the oracle, or a planted-mistake copy of it)."""
import numpy as np
import scipy.ndimage as ndi

from oracle import psl_oracle as O


def rng(s):
    return np.random.Generator(np.random.PCG64(s))


def pin_bf16_round_known_values_and_torch(N):
    import torch
    one = 1.0
    assert N.bf16_round(np.array([one]))[0] == 1.0
    assert N.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0                 # tie -> even
    assert N.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6     # tie -> even
    assert N.bf16_round(np.array([1 + 2 ** -8 + 2 ** -20]))[0] == 1 + 2 ** -7
    x = rng(1).normal(0, 10, 4096) * np.exp(rng(2).normal(0, 5, 4096))
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16_round(x), ref)


def pin_conv3d_matches_library_correlation(N):
    g = rng(3)
    x = g.normal(size=(5, 6, 7, 3))
    w = g.normal(size=(4, 27, 3))
    b = g.normal(size=4)
    out = N.conv3d(x, w, b)
    for co in range(4):
        ref = b[co] + sum(ndi.correlate(x[..., ci], w[co, :, ci].reshape(3, 3, 3),
                                        mode="constant", cval=0.0) for ci in range(3))
        assert np.allclose(out[..., co], ref, rtol=1e-12, atol=1e-12)


def pin_conv3d_backward_is_the_adjoint_and_matches_differences(N):
    g = rng(4)
    x = g.normal(size=(4, 5, 6, 3))
    w = g.normal(size=(2, 27, 3))
    b = g.normal(size=2)
    gout = g.normal(size=(4, 5, 6, 2))
    gx, gw, gb = N.conv3d_backward(x, w, gout)
    # linear in x (bias fixed): <conv(x + d) - conv(x), gout> = <d, gx>
    d = g.normal(size=x.shape)
    lhs = np.sum((N.conv3d(x + d, w, b) - N.conv3d(x, w, b)) * gout)
    assert np.isclose(lhs, np.sum(d * gx), rtol=1e-11)
    # weights and bias: central differences of <conv, gout>
    f = lambda ww, bb: np.sum(N.conv3d(x, ww, bb) * gout)
    for idx in [(0, 0, 0), (1, 13, 2), (0, 26, 1)]:
        e = np.zeros_like(w); e[idx] = 1e-6
        fd = (f(w + e, b) - f(w - e, b)) / 2e-6
        assert np.isclose(gw[idx], fd, rtol=1e-7, atol=1e-7)
    e = np.zeros_like(b); e[1] = 1e-6
    assert np.isclose(gb[1], (f(w, b + e) - f(w, b - e)) / 2e-6, rtol=1e-7)
    # 1x1x1 layer is a per-cell matrix product
    w1 = g.normal(size=(2, 1, 3))
    assert np.allclose(N.conv3d(x, w1, b), x @ w1[:, 0, :].T + b)


def pin_pool_and_upsample_adjoints(N):
    g = rng(5)
    a = g.normal(size=(2, 3, 4, 2))
    c = g.normal(size=(4, 6, 8, 2))
    assert np.isclose(np.sum(N.upsample2(a) * c), np.sum(a * N.upsample2_backward(c)))
    assert np.allclose(N.pool2(N.upsample2(a)), a)
    assert np.isclose(np.sum(N.pool2(c) * a), np.sum(c * N.pool2_backward(a)))
    # pooling a constant field keeps it; the block mean of an explicit block
    assert np.allclose(N.pool2(np.full((4, 4, 4, 1), 3.0)), 3.0)
    assert np.isclose(N.pool2(c)[1, 2, 3, 1], c[2:4, 4:6, 6:8, 1].mean())


def pin_layer_shapes_chain(N):
    shapes = N.layer_shapes()
    assert [s[0] for s in shapes] == ["e0a", "e0b", "e1a", "e1b", "e2a", "e2b", "e3a", "e3b",
                                      "d2", "d1", "d0", "out"]
    assert dict((s[0], s[3]) for s in shapes)["d2"] == 64 + 48
    assert dict((s[0], s[3]) for s in shapes)["d0"] == 32 + 16


def pin_network_gradient_finite_differences(N, bf16):
    arch = N.Arch(cin=2, widths=(3, 4, 4, 5))
    params = N.init_params(arch, seed=7)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng(8).normal(0, 0.1, params[k].shape)
    x = rng(9).normal(size=(8, 8, 8, 2))
    r = rng(10).normal(size=(8, 8, 8, 1))
    y, cache = N.forward(params, x, arch)
    grads = N.backward(params, cache, r, arch)
    f = lambda p: np.sum(N.forward(p, x, arch)[0] * r)
    picks = [("e0a.w", (1, 5, 0)), ("e1b.w", (2, 13, 3)), ("e3a.w", (4, 26, 1)),
             ("d2.w", (0, 4, 7)), ("d0.w", (2, 20, 5)), ("out.w", (0, 0, 2)), ("d1.b", (1,)),
             ("e2b.b", (3,))]
    for name, idx in picks:
        p1 = {k: v.copy() for k, v in params.items()}
        p2 = {k: v.copy() for k, v in params.items()}
        p1[name][idx] += 1e-6
        p2[name][idx] -= 1e-6
        fd = (f(p1) - f(p2)) / 2e-6
        assert np.isclose(grads[name][idx], fd, rtol=2e-5, atol=1e-8), (name, grads[name][idx], fd)
    if bf16:
        # with bf16 operands the forward differs from float64 at bf16 resolution only
        yb, _ = N.forward(params, x, arch, bf16=True)
        assert np.linalg.norm(yb - y) <= 0.05 * np.linalg.norm(y)


def _tiny_system():
    import psl_inputs as pi
    prob = pi.layered3d(8, 8, 8, nlayers=4, contrast=1e3, sigma_ln=0.5, nsub=(2, 2, 2),
                        seed=3, wells="columns")
    A, b = O.assemble(prob.K, prob.grid, prob.dirichlet_mask, prob.q)
    Z = O.deflation_matrix(*O.levelset_labels(prob.grid, prob.K, prob.nsub, prob.thr))
    return prob, A, b, Z


def pin_energy_loss_closed_form_and_gradient(N):
    prob, A, b, Z = _tiny_system()
    P1 = O.projectors(A, Z)[0]
    P1A = lambda v: P1 @ (A @ v)
    xs = np.linalg.solve(A.toarray(), b)
    P1b = P1 @ b
    c = float(xs @ P1b)
    y = rng(11).normal(size=(8, 8, 8, 1))
    L, gL, alpha = N.energy_loss(y, P1b, P1A, c)
    # definition: ||P2 (alpha y - x*)||_A^2 / ||P2 x*||_A^2 with P2 = I - Z E^-1 Z^T A
    P2 = np.eye(A.shape[0]) - Z.toarray() @ np.linalg.solve((Z.T @ A @ Z).toarray(),
                                                             (Z.T @ A).toarray())
    e = P2 @ (alpha * y.reshape(-1) - xs)
    ref = (e @ (A @ e)) / ((P2 @ xs) @ (A @ (P2 @ xs)))
    assert np.isclose(L, ref, rtol=1e-9)
    # alpha is optimal: any other scale is worse
    for s in (0.5, 0.9, 1.1, 2.0):
        e2 = P2 @ (s * alpha * y.reshape(-1) - xs)
        assert e2 @ (A @ e2) >= e @ (A @ e) - 1e-12
    # scale-free, zero at the solution, gradient by central differences
    assert np.isclose(N.energy_loss(3.7 * y, P1b, P1A, c)[0], L, rtol=1e-12)
    assert abs(N.energy_loss(xs.reshape(y.shape), P1b, P1A, c)[0]) < 1e-10
    for idx in [(0, 0, 0, 0), (3, 4, 5, 0), (7, 7, 7, 0)]:
        d = np.zeros_like(y); d[idx] = 1e-6
        fd = (N.energy_loss(y + d, P1b, P1A, c)[0] - N.energy_loss(y - d, P1b, P1A, c)[0]) / 2e-6
        assert np.isclose(gL[idx], fd, rtol=1e-5, atol=1e-10)
    # fixed-scale regression on t = x* / sigma: definition, zero at t, differences
    sigma = 3.0
    Ls, gs, _ = N.energy_loss(y, P1b, P1A, c, sigma=sigma)
    t = xs / sigma
    e = P2 @ (y.reshape(-1) - t)
    assert np.isclose(Ls, (e @ (A @ e)) / ((P2 @ t) @ (A @ (P2 @ t))), rtol=1e-9)
    assert abs(N.energy_loss(t.reshape(y.shape), P1b, P1A, c, sigma=sigma)[0]) < 1e-10
    assert np.isclose(N.energy_loss(0 * y, P1b, P1A, c, sigma=sigma)[0], 1.0)
    assert Ls >= L - 1e-12            # the best multiple is never worse
    for idx in [(1, 2, 3, 0), (6, 0, 5, 0)]:
        # the loss is quadratic in y: central differences are exact for any step
        d = np.zeros_like(y); d[idx] = 1e-2
        fd = (N.energy_loss(y + d, P1b, P1A, c, sigma=sigma)[0]
              - N.energy_loss(y - d, P1b, P1A, c, sigma=sigma)[0]) / 2e-2
        assert np.isclose(gs[idx], fd, rtol=1e-8, atol=1e-12)


def pin_adam_first_step_and_convergence(N):
    g = np.array([3.0, -0.002, 40.0])
    p, m, v = N.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # first bias-corrected step has magnitude lr (up to eps) in the direction of -g
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-4)
    # minimises a convex quadratic
    q = np.array([1.0, -2.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = N.adam_step(p, 2 * (p - q), m, v, t, lr=0.01)
    assert np.allclose(p, q, atol=1e-3)


def pin_make_input_normalisation(N):
    import psl_inputs as pi
    prob = pi.layered3d(8, 8, 4, nlayers=2, contrast=1e4, nsub=(2, 2, 2), seed=1, wells="columns")
    x = N.make_input(prob.K, prob.q, prob.grid)
    assert x.shape == (4, 8, 8, 2)
    assert abs(x[..., 0].mean()) < 1e-12 and abs(x[..., 0].std() - 1) < 1e-12
    assert np.isclose(np.abs(x[..., 1]).max(), 1.0)
    assert np.array_equal(x[..., 1].reshape(-1), prob.q / np.abs(prob.q).max())


def pin_weighted_l2_and_cell_diag(N):
    prob, A, b, Z = _tiny_system()
    Tx, Ty, Tz = O.transmissibilities(prob.K, prob.grid, prob.dirichlet_mask)
    assert np.allclose(N.cell_diag(Tx, Ty, Tz, prob.grid), A.diagonal(), rtol=1e-14)
    g = rng(21)
    y, t = g.normal(size=(4, 5, 6, 1)), g.normal(size=(4, 5, 6, 1))
    d = np.exp(g.normal(size=120))
    L, gL = N.weighted_l2_loss(y, t, d)
    assert np.isclose(L, np.sum(d * (y - t).reshape(-1) ** 2) / np.sum(d * t.reshape(-1) ** 2))
    assert N.weighted_l2_loss(t, t, d)[0] == 0.0
    assert np.isclose(N.weighted_l2_loss(0 * y, t, d)[0], 1.0)
    for idx in [(0, 0, 0, 0), (3, 4, 5, 0)]:
        e = np.zeros_like(y); e[idx] = 1e-2            # quadratic: central differences exact
        fd = (N.weighted_l2_loss(y + e, t, d)[0] - N.weighted_l2_loss(y - e, t, d)[0]) / 2e-2
        assert np.isclose(gL[idx], fd, rtol=1e-8)
