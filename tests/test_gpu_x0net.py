"""Start-vector network on the GPU against its float64 reference (oracle/x0net_oracle.py).

Kernel tests feed both sides the same bf16-rounded operands, so only float32 summation
order separates them (bounds stated per test). The whole-network test differs also in
where bf16 rounding happens around pooling (the GPU rounds each conv output before the
next layer reads it), so its bound is looser."""
import numpy as np
import pytest

import psl_inputs as pi
from oracle import psl_oracle as O
from oracle import x0net_oracle as N

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def rng(s):
    return np.random.Generator(np.random.PCG64(s))


def to_bf16_bits(a):
    """Bit patterns of bf16(a) (round to nearest even) as an int16 device tensor."""
    import torch
    r = N.bf16_round(np.asarray(a, dtype=np.float64)).astype(np.float32)
    bits = (r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(bits)).cuda()


def from_bf16_bits(t):
    b = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def dev32(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


GRID = (16, 6, 5)   # nx multiple of 8, ragged y/z


def _grid_arr(shape, c, seed):
    nx, ny, nz = shape
    return N.bf16_round(rng(seed).normal(size=(nz, ny, nx, c)))


def _pack_weights(w3):
    """Master weights (Cout, 27, Cin) -> GPU operands via the Adam kernel's repack (t=0)."""
    import torch
    from paper_1510_02148_amd import nn
    cout, _, cin = w3.shape
    p = dev32(w3.reshape(cout, -1))
    z = torch.zeros_like(p)
    pb = torch.zeros(cout, dtype=torch.float32, device="cuda")
    w = nn.bf16_empty(cout, nn.kp(cin), zero=True)
    wt = nn.bf16_empty(cin, nn.kp(cout), zero=True)
    nn.adam_conv(cout, cin, p, z.clone(), z.clone(), pb, pb.clone(), pb.clone(), None, 0, 0.0, w, wt)
    return w, wt


@pytest.mark.parametrize("cin,cout,relu", [(8, 16, True), (16, 32, False), (48, 16, True),
                                           (112, 48, True)])
def test_conv3_forward(gpu_lib, cin, cout, relu):
    import torch
    from paper_1510_02148_amd import nn
    say(f"conv3 forward cin={cin} cout={cout} relu={relu} grid={GRID}")
    x = _grid_arr(GRID, cin, 1)
    w3 = N.bf16_round(rng(2).normal(size=(cout, 27, cin)) / np.sqrt(27 * cin))
    b = rng(3).normal(size=cout).astype(np.float32).astype(np.float64)
    w, _ = _pack_weights(w3)
    n = int(np.prod(GRID))
    y = nn.bf16_empty(n, cout)
    yf = torch.empty(n, cout, dtype=torch.float32, device="cuda")
    nn.conv3(GRID, to_bf16_bits(x.reshape(n, cin)), cin, w, cout, dev32(b), relu, y, yf)
    ref = N.conv3d(x, w3, b)
    ref = N.relu(ref) if relu else ref
    got = yf.cpu().numpy().astype(np.float64).reshape(ref.shape)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  max rel err {err:.2e}")
    assert err <= 2e-6
    # the bf16 output is the rounding of the float32 one
    assert np.array_equal(from_bf16_bits(y).reshape(-1), N.bf16_round(yf.cpu().numpy()).reshape(-1))


# (24, 20, 19) has 9120 cells: the weight gradient's split over 4096-cell chunks then has
# two full chunks and a ragged third, whose partial sums the finishing pass adds
BACKWARD_CASES = [(GRID, 16, 16), (GRID, 48, 16), (GRID, 32, 48), (GRID, 112, 48),
                  (GRID, 48, 64), ((24, 20, 19), 16, 32), ((24, 20, 19), 48, 16)]


@pytest.mark.parametrize("grid,cin,cout", BACKWARD_CASES,
                         ids=[f"{g[0]}x{g[1]}x{g[2]}-{a}-{b}" for g, a, b in BACKWARD_CASES])
def test_conv3_input_and_weight_gradients(gpu_lib, grid, cin, cout):
    import torch
    from paper_1510_02148_amd import nn
    GRID = grid
    say(f"conv3 backward cin={cin} cout={cout} grid={GRID}")
    n = int(np.prod(GRID))
    x = _grid_arr(GRID, cin, 4)
    g = _grid_arr(GRID, cout, 5)
    w3 = N.bf16_round(rng(6).normal(size=(cout, 27, cin)) / np.sqrt(27 * cin))
    w, wt = _pack_weights(w3)
    gx_ref, gw_ref, gb_ref = N.conv3d_backward(x, w3, g)
    gq = to_bf16_bits(g.reshape(n, cout))
    gx = torch.empty(n, cin, dtype=torch.float32, device="cuda")
    nn.conv3(GRID, gq, cout, wt, cin, None, False, None, gx)
    e1 = np.abs(gx.cpu().numpy().reshape(gx_ref.shape) - gx_ref).max() / np.abs(gx_ref).max()
    kp = nn.kp(cin)
    dw = torch.empty(cout, kp + 16, dtype=torch.float32, device="cuda")
    work = torch.empty(nn.wgrad_work(GRID, cin, cout), dtype=torch.float32, device="cuda")
    nn.conv3_wgrad(GRID, gq, cout, to_bf16_bits(x.reshape(n, cin)), cin, dw, work)
    d = dw.cpu().numpy().astype(np.float64)
    gw = d[:, :27 * cin].reshape(cout, 27, cin)
    e2 = np.abs(gw - gw_ref).max() / np.abs(gw_ref).max()
    e3 = np.abs(d[:, kp] - gb_ref).max() / np.abs(gb_ref).max()
    say(f"  input grad {e1:.2e}  weight grad {e2:.2e}  bias grad {e3:.2e}")
    assert e1 <= 2e-6 and e2 <= 2e-6 and e3 <= 2e-6
    assert np.all(d[:, 27 * cin:kp] == 0) and np.all(d[:, kp + 1:] == 0)


def test_resampling_and_mask(gpu_lib):
    import torch
    from paper_1510_02148_amd import nn
    fine = (16, 6, 4)
    n = int(np.prod(fine))
    c = 16
    x = _grid_arr(fine, c, 7)
    y = nn.bf16_empty(n // 8, c)
    nn.pool2(fine, to_bf16_bits(x.reshape(n, c)), c, y)
    assert rel(from_bf16_bits(y).reshape(-1), N.bf16_round(N.pool2(x)).reshape(-1)) <= 4e-3
    gy = rng(8).normal(size=(fine[2] // 2, fine[1] // 2, fine[0] // 2, c))
    gx = dev32(np.ones((n, c)))
    nn.pool2_grad_add(fine, dev32(gy.reshape(-1, c)), c, gx)
    assert rel(gx.cpu().numpy(), (1.0 + N.pool2_backward(gy)).reshape(n, c)) <= 1e-6
    # decoder input and its adjoint
    ca, cb = 32, 16
    h = _grid_arr((8, 3, 2), ca, 9)
    s = _grid_arr(fine, cb, 10)
    cat = nn.bf16_empty(n, ca + cb)
    nn.upcat(fine, to_bf16_bits(h.reshape(-1, ca)), ca, to_bf16_bits(s.reshape(n, cb)), cb, cat)
    ref = np.concatenate([N.upsample2(h), s], axis=3)
    assert np.array_equal(from_bf16_bits(cat).reshape(-1), ref.reshape(-1))
    gcat = rng(11).normal(size=(n, ca + cb))
    gh = torch.empty(n // 8 * ca, dtype=torch.float32, device="cuda")
    gs = torch.empty(n * cb, dtype=torch.float32, device="cuda")
    nn.upcat_grad(fine, dev32(gcat), ca, cb, gh, gs)
    g4 = gcat.reshape(fine[2], fine[1], fine[0], ca + cb)
    assert rel(gh.cpu().numpy(), N.upsample2_backward(g4[..., :ca]).reshape(-1)) <= 1e-6
    assert rel(gs.cpu().numpy(), g4[..., ca:].reshape(-1)) <= 1e-7
    # ReLU mask with bf16 rounding of the kept gradient
    yv = _grid_arr(fine, c, 12)
    gyv = rng(13).normal(size=yv.shape)
    gq = nn.bf16_empty(n * c)
    nn.relu_grad(dev32(gyv.reshape(-1)), to_bf16_bits(yv.reshape(-1)), gq, relu=True)
    assert np.array_equal(from_bf16_bits(gq).reshape(-1),
                          N.bf16_round(N.relu_backward(yv, gyv)).reshape(-1))


def test_output_layer(gpu_lib):
    import torch
    from paper_1510_02148_amd import nn
    n, cin = int(np.prod(GRID)), 16
    h = _grid_arr(GRID, cin, 14)
    w1 = N.bf16_round(rng(15).normal(size=(1, 1, cin)))
    b = np.array([0.25])
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    nn.conv1(n, to_bf16_bits(h.reshape(n, cin)), cin, to_bf16_bits(w1.reshape(-1)), dev32(b), y)
    ref = N.conv3d(h, w1, b)
    assert rel(y.cpu().numpy(), ref.reshape(-1)) <= 1e-6
    gy = rng(16).normal(size=(n,))
    gh = torch.empty(n * cin, dtype=torch.float32, device="cuda")
    dw = torch.empty(cin + 1, dtype=torch.float32, device="cuda")
    work = torch.empty(nn.conv1_work(n, cin), dtype=torch.float32, device="cuda")
    nn.conv1_grad(n, dev32(gy), to_bf16_bits(h.reshape(n, cin)), cin, to_bf16_bits(w1.reshape(-1)),
                  gh, dw, work)
    gq = N.bf16_round(gy).reshape(h.shape[:3] + (1,))
    gx_ref, gw_ref, gb_ref = N.conv3d_backward(h, w1, gq)
    assert rel(gh.cpu().numpy(), gx_ref.reshape(-1)) <= 1e-6
    assert rel(dw.cpu().numpy()[:cin], gw_ref.reshape(-1)) <= 1e-5
    assert abs(dw.cpu().numpy()[cin] - gb_ref[0]) <= 1e-5 * max(1.0, abs(gb_ref[0]))


def test_input_energy_and_adam(gpu_lib):
    import torch
    from paper_1510_02148_amd import nn, pipeline
    psl = gpu_lib
    prob = pi.layered3d(16, 8, 8, nlayers=4, contrast=1e4, sigma_ln=1.0, nsub=(2, 2, 2), seed=2,
                        wells="columns")
    n = prob.n
    K = torch.tensor(prob.K, device="cuda")
    b = torch.tensor(prob.q, device="cuda")
    x = nn.bf16_empty(n, 8, zero=True)
    work = torch.empty(max(nn.input_work(n), nn.energy_work(n)), dtype=torch.float64, device="cuda")
    nn.make_input(K, b, x, work)
    ref = N.make_input(prob.K, prob.q, prob.grid).reshape(n, 2)
    got = from_bf16_bits(x).reshape(n, 8)
    assert np.all(got[:, 2:] == 0)
    assert np.abs(got[:, :2] - N.bf16_round(ref)).max() <= 2 ** -7 * max(1.0, np.abs(ref).max())
    # energy loss through the solver's own operators
    s = pipeline.setup(prob.grid, K, prob.dirichlet_mask, prob.nsub, list(prob.thr))
    A, bh = O.assemble(prob.K, prob.grid, prob.dirichlet_mask, prob.q)
    Z = O.deflation_matrix(*O.levelset_labels(prob.grid, prob.K, prob.nsub, prob.thr))
    P1 = O.projectors(A, Z)[0]
    xs = np.linalg.solve(A.toarray(), bh)
    c = float(xs @ (P1 @ bh))
    # a direction correlated with the solution, so that alpha and L are well conditioned
    y = (xs + 0.3 * np.abs(xs).mean() * rng(17).normal(size=n)).astype(np.float32)
    L_ref, g_ref, a_ref = N.energy_loss(y.astype(np.float64), P1 @ bh, lambda v: P1 @ (A @ v), c)
    P1b = torch.empty_like(b)
    psl.psl_deflate(s.ctx, b, P1b)
    y64 = torch.empty_like(b)
    Ay = torch.empty_like(b)
    yd = dev32(y)
    nn.widen(yd, y64)
    psl.psl_apply_A(s.ctx, y64, Ay)
    psl.psl_deflate(s.ctx, Ay, Ay)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    gy = torch.empty(n, dtype=torch.float32, device="cuda")
    x0 = torch.empty_like(b)
    nn.energy(yd, P1b, Ay, c, out, work, gy=gy, x0=x0)
    o = out.cpu().numpy()
    say(f"energy L={o[0]:.6f} (oracle {L_ref:.6f}) alpha={o[1]:.4e} (oracle {a_ref:.4e})")
    assert abs(o[0] - L_ref) <= 1e-9 and abs(o[1] - a_ref) <= 1e-9 * abs(a_ref)
    assert rel(gy.cpu().numpy(), g_ref) <= 1e-6
    assert 0.0 < o[0] < 1.0
    assert rel(x0.cpu().numpy(), a_ref * y.astype(np.float64)) <= 1e-12
    # training form: regression on x* / sigma
    sigma = float(np.sqrt(np.mean(xs ** 2)))
    Ls_ref, gs_ref, _ = N.energy_loss(y.astype(np.float64), P1 @ bh, lambda v: P1 @ (A @ v), c,
                                      sigma=sigma)
    nn.energy(yd, P1b, Ay, c, out, work, gy=gy, sigma=sigma)
    say(f"regression L={out[0].item():.6f} (oracle {Ls_ref:.6f})")
    assert abs(out[0].item() - Ls_ref) <= 1e-9 * max(1.0, abs(Ls_ref))
    assert rel(gy.cpu().numpy(), gs_ref) <= 1e-6
    # Adam against the reference update, three steps
    shape = (16, 27, 8)
    p = rng(18).normal(size=shape)
    pg = [rng(19 + t).normal(size=shape) for t in range(3)]
    bias_g = [rng(29 + t).normal(size=16) for t in range(3)]
    pt, mt, vt = dev32(p.reshape(16, -1)), *[torch.zeros(16, 27 * 8, device="cuda") for _ in range(2)]
    pb, mb, vb = [torch.zeros(16, device="cuda") for _ in range(3)]
    w = nn.bf16_empty(16, nn.kp(8), zero=True)
    kp = nn.kp(8)
    pr, mr, vr = p.copy(), np.zeros(shape), np.zeros(shape)
    br, bm, bv = np.zeros(16), np.zeros(16), np.zeros(16)
    for t in range(1, 4):
        dw = np.zeros((16, kp + 16))
        dw[:, :27 * 8] = pg[t - 1].reshape(16, -1)
        dw[:, kp] = bias_g[t - 1]
        nn.adam_conv(16, 8, pt, mt, vt, pb, mb, vb, dev32(dw), t, 1e-2, w, None)
        pr, mr, vr = N.adam_step(pr, pg[t - 1], mr, vr, t, lr=1e-2)
        br, bm, bv = N.adam_step(br, bias_g[t - 1], bm, bv, t, lr=1e-2)
    assert rel(pt.cpu().numpy().reshape(shape), pr) <= 1e-6
    assert rel(pb.cpu().numpy(), br) <= 1e-5
    assert np.array_equal(from_bf16_bits(w).reshape(16, kp)[:, :27 * 8],
                          N.bf16_round(pt.cpu().numpy()).reshape(16, -1))


def test_network_forward_backward(gpu_lib):
    """Whole network on a 64x16x16 grid.

    Forward: against the reference with bf16 operands and bf16-stored activations. The
    first layer matches bit for bit; later layers differ where float32 and float64 sums
    round to neighbouring bf16 values, and those 1-ulp differences propagate (measured:
    ~2e-3 relative at the output, 78 of 262144 ReLU masks flipped in the last layer).
    Backward: the reference backward runs on the GPU's own stored activations (same
    masks, same operands), so every parameter gradient checks the backward kernels alone;
    the last layers agree to ~1e-7 and the error grows to a few 1e-3 towards the first
    layers as the bf16 rounding of the gradients passed between layers meets the same
    1-ulp ties."""
    import torch
    from paper_1510_02148_amd import x0net
    grid = (64, 16, 16)
    n = int(np.prod(grid))
    net = x0net.X0Net(grid, seed=3)
    params = net.export_params()
    for k in params:                                     # non-zero biases exercise the sums
        if k.endswith(".b"):
            params[k] = rng(40).normal(0, 0.05, params[k].shape).astype(np.float32).astype(np.float64)
    net.load_params(params)
    prob = pi.layered3d(*grid, nlayers=4, contrast=1e4, nsub=(4, 2, 2), seed=5, wells="columns")
    K = torch.tensor(prob.K, device="cuda")
    b = torch.tensor(prob.q, device="cuda")
    net.set_input(K, b)
    y = net.forward().cpu().numpy().astype(np.float64)
    xin = N.make_input(prob.K, prob.q, prob.grid)
    yr, _ = N.forward(params, xin, bf16=True, store_bf16=True)
    e = rel(y, yr.reshape(-1))
    say(f"network output rel err {e:.2e}")
    assert e <= 5e-3
    # the GPU's activations as the reference's cache
    def act(name, lvl):
        gx, gyd, gz = net.grids[lvl]
        return from_bf16_bits(net.A[name]).reshape(gz, gyd, gx, -1)
    cache = {"in": {}, "out": {}}
    cache["in"]["e0a"] = act("x", 0)[..., :2]
    for i in range(net.nl):
        cache["in"][f"e{i}b"] = act(f"e{i}a", i)
        if i > 0:
            cache["in"][f"e{i}a"] = act(f"pool{i}", i)
        cache["out"][f"e{i}a"] = act(f"e{i}a", i)
        cache["out"][f"e{i}b"] = act(f"e{i}b", i)
    for i in range(net.nl - 1):
        cache["in"][f"d{i}"] = act(f"cat{i}", i)
        cache["out"][f"d{i}"] = act(f"d{i}", i)
    cache["in"]["out"] = act("d0", 0)
    gy = rng(41).normal(size=n)
    net.backward(torch.tensor(gy, dtype=torch.float32, device="cuda"))
    gref = N.backward(params, cache, gy.reshape(yr.shape), bf16=True)
    worst = 0.0
    for name, L in net.P.items():
        d = L["dw"].cpu().numpy().astype(np.float64)
        if L["taps"] == 27:
            cin = L["cin"] if name != "e0a" else 2
            gw = d[:, :27 * L["cin"]].reshape(L["cout"], 27, L["cin"])[:, :, :cin]
            gb = d[:, nnkp(L["cin"])]
        else:
            gw, gb = d[:-1].reshape(1, 1, -1), d[-1:]
        ew, eb = rel(gw, gref[name + ".w"]), rel(gb, gref[name + ".b"])
        worst = max(worst, ew, eb)
        say(f"  {name}: weight grad {ew:.2e} bias grad {eb:.2e}")
    assert worst <= 1e-2


def nnkp(cin):
    from paper_1510_02148_amd import nn
    return nn.kp(cin)


def test_training_gain_on_held_out_instances(gpu_lib):
    """What the trained network gains over the method without it, measured: the network is
    trained on the GPU (its own forward, backward and Adam kernels, the energy loss through
    the solver's P1 A) on 24 instances of the learned-start workload at 64x64x32, then
    every one of 8 held-out instances is solved to 1e-8 from x0 = 0 and from the scaled
    network start (inference included in its time). Asserted: training lowers the loss
    from its initial value; the scaled start is never worse than x0 = 0 in the energy norm
    of the deflated error (the scale is energy-optimal, zero among its candidates); both
    solves converge; the learned start costs at most 2 % more iterations in total. The
    measured gain (iterations and time, which may be none) is printed."""
    from paper_1510_02148_amd import x0net, x0train
    shape = (64, 64, 32)
    tr = [pi.learned_x0_instance(1000 + i, shape=shape, nsub=(4, 4, 2)) for i in range(24)]
    te = [pi.learned_x0_instance(5000 + i, shape=shape, nsub=(4, 4, 2)) for i in range(8)]
    say(f"x0 training: {len(tr)} train, {len(te)} held-out instances of {shape}")
    dtr, dte = x0train.prepare(tr), x0train.prepare(te)
    net = x0net.X0Net(shape, seed=0)
    losses = x0train.train(net, dtr, 240, lr=1e-3, loss="energy")
    first, last = float(np.mean(losses[:24])), float(np.mean(losses[-24:]))
    ev = x0train.evaluate(net, dte, repeats=2)
    it0 = sum(r["iters_zero"] for r in ev)
    it1 = sum(r["iters_net"] for r in ev)
    t0 = sum(r["t_zero"] for r in ev)
    t1 = sum(r["t_net"] for r in ev)
    say(f"  training loss {first:.4f} -> {last:.4f}; held-out iterations {it0} (x0 = 0) vs "
        f"{it1} (learned), gain {it0 - it1} ({(it0 - it1) / it0:+.1%}); time "
        f"{t0 * 1e3:.1f} vs {t1 * 1e3:.1f} ms (inference included); start energy loss "
        + " ".join(f"{r['loss_net']:.4f}" for r in ev))
    assert last < first
    assert all(r["loss_net"] <= 1.0 + 1e-9 for r in ev)
    assert all(r["relres_zero"] <= 1e-8 and r["relres_net"] <= 1e-8 for r in ev)
    assert it1 <= 1.02 * it0
