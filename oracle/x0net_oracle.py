"""Plain float64 reference of the start-vector network (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU leg may import this module; the
product path runs the HIP kernels of libpsl and never calls it.

The network maps two input channels on the pressure grid (normalised log10 K and the
normalised right-hand side) to one output channel y; the start vector is x0 = alpha y
with alpha the energy-optimal scale below. The paper has no learned component: this is
a project addition, and these routines define what the GPU kernels must compute.

Tensors are channels-last arrays of shape (nz, ny, nx, C) (cell c = ix + nx (iy + ny iz)
is index [iz, iy, ix]). Convolutions are 3x3x3 cross-correlations with zero padding and
stride 1 (plus one 1x1x1 output layer); weights have shape (Cout, 27, Cin) with the tap
index t = (dz+1)*9 + (dy+1)*3 + (dx+1). Pooling averages 2x2x2 blocks; upsampling copies
each cell into its 2x2x2 children. Rounding to bfloat16 is round-to-nearest-even on the
float32 bit pattern.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# ---------------------------------------------------------------------------------------
# bfloat16
# ---------------------------------------------------------------------------------------
def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) and return the value as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


# ---------------------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------------------
def _shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[z, y, x] = x[z + dz, y + dy, x + dx], zero outside the grid."""
    nz, ny, nx = x.shape[:3]
    out = np.zeros_like(x)
    zs, zd = slice(max(0, dz), nz + min(0, dz)), slice(max(0, -dz), nz - max(0, dz))
    ys, yd = slice(max(0, dy), ny + min(0, dy)), slice(max(0, -dy), ny - max(0, dy))
    xs, xd = slice(max(0, dx), nx + min(0, dx)), slice(max(0, -dx), nx - max(0, dx))
    out[zd, yd, xd] = x[zs, ys, xs]
    return out


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[v, co] = b[co] + sum_t sum_ci w[co, t, ci] x[v + tap_t, ci] (3x3x3 or 1x1x1)."""
    cout, ntap, cin = w.shape
    assert x.shape[3] == cin and ntap in (1, 27)
    out = np.broadcast_to(b, x.shape[:3] + (cout,)).astype(np.float64).copy()
    taps = TAPS if ntap == 27 else [(0, 0, 0)]
    for t, (dz, dy, dx) in enumerate(taps):
        out += _shift(x, dz, dy, dx) @ w[:, t, :].T
    return out


def conv3d_backward(x: np.ndarray, w: np.ndarray, gout: np.ndarray
                    ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Gradients of conv3d with respect to x, w and b for the output gradient gout."""
    cout, ntap, cin = w.shape
    taps = TAPS if ntap == 27 else [(0, 0, 0)]
    gx = np.zeros_like(x, dtype=np.float64)
    gw = np.zeros_like(w, dtype=np.float64)
    flat_g = gout.reshape(-1, cout)
    for t, (dz, dy, dx) in enumerate(taps):
        xs = _shift(x, dz, dy, dx)
        gw[:, t, :] = flat_g.T @ xs.reshape(-1, cin)
        # out[v] uses x[v + tap]: the adjoint moves gout back by -tap
        gx += _shift(gout @ w[:, t, :], -dz, -dy, -dx)
    gb = flat_g.sum(axis=0)
    return gx, gw, gb


def relu(x: np.ndarray) -> np.ndarray:
    return np.maximum(x, 0.0)


def relu_backward(y: np.ndarray, gy: np.ndarray) -> np.ndarray:
    """Gradient through relu given its output y (the derivative is taken 0 at 0)."""
    return np.where(y > 0.0, gy, 0.0)


def pool2(x: np.ndarray) -> np.ndarray:
    """Average over 2x2x2 blocks (even extents)."""
    nz, ny, nx, c = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def pool2_backward(g: np.ndarray) -> np.ndarray:
    return upsample2(g) / 8.0


def upsample2(x: np.ndarray) -> np.ndarray:
    """Each cell copied into its 2x2x2 children."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=0), 2, axis=1), 2, axis=2)


def upsample2_backward(g: np.ndarray) -> np.ndarray:
    nz, ny, nx, c = g.shape
    return g.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).sum(axis=(1, 3, 5))


# ---------------------------------------------------------------------------------------
# network: 4-level encoder/decoder with skip connections
# ---------------------------------------------------------------------------------------
@dataclass
class Arch:
    cin: int = 2
    widths: Tuple[int, ...] = (16, 32, 48, 64)


def layer_shapes(arch: Arch = Arch()) -> List[Tuple[str, int, int, int]]:
    """(name, Cout, taps, Cin) of every convolution in evaluation order."""
    w = arch.widths
    shapes = [("e0a", w[0], 27, arch.cin), ("e0b", w[0], 27, w[0])]
    for i in range(1, len(w)):
        shapes += [(f"e{i}a", w[i], 27, w[i - 1]), (f"e{i}b", w[i], 27, w[i])]
    for i in range(len(w) - 2, -1, -1):
        shapes += [(f"d{i}", w[i], 27, w[i + 1] + w[i])]   # input: upsampled + skip
    shapes += [("out", 1, 1, w[0])]
    return shapes


def init_params(arch: Arch = Arch(), seed: int = 0) -> Dict[str, np.ndarray]:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, from a seeded PCG64."""
    g = np.random.Generator(np.random.PCG64(seed))
    params = {}
    for name, cout, ntap, cin in layer_shapes(arch):
        params[name + ".w"] = g.normal(0.0, np.sqrt(2.0 / (ntap * cin)), (cout, ntap, cin))
        params[name + ".b"] = np.zeros(cout)
    return params


def forward(params: Dict[str, np.ndarray], x: np.ndarray, arch: Arch = Arch(),
            bf16: bool = False, store_bf16: bool = False) -> Tuple[np.ndarray, dict]:
    """Network output y (nz, ny, nx, 1) and the activations the backward pass needs.
    bf16=True rounds every convolution's weight and input to bfloat16 (the GPU operands);
    sums stay in float64 here. store_bf16=True also keeps every hidden activation as
    bfloat16 (each convolution output and each pooled field rounded when stored), the
    storage precision of the GPU network; the output layer stays unrounded."""
    rd = bf16_round if bf16 else (lambda a: a)
    st = bf16_round if store_bf16 else (lambda a: a)
    nl = len(arch.widths)
    cache = {"in": {}, "out": {}}

    def conv(name, inp, act=True):
        w = rd(params[name + ".w"])
        xi = rd(inp)
        cache["in"][name] = xi
        o = conv3d(xi, w, params[name + ".b"])
        o = relu(o) if act else o
        if act:
            o = st(o)
        cache["out"][name] = o
        return o

    h = x
    skips = []
    for i in range(nl):
        if i > 0:
            h = st(pool2(h))
        h = conv(f"e{i}a", h)
        h = conv(f"e{i}b", h)
        skips.append(h)
    for i in range(nl - 2, -1, -1):
        h = np.concatenate([upsample2(h), skips[i]], axis=3)
        h = conv(f"d{i}", h)
    y = conv("out", h, act=False)
    return y, cache


def backward(params: Dict[str, np.ndarray], cache: dict, gy: np.ndarray,
             arch: Arch = Arch(), bf16: bool = False) -> Dict[str, np.ndarray]:
    """Parameter gradients for the output gradient gy. bf16=True rounds the operands of
    both backward products (weights, cached inputs, masked output gradients) as the GPU
    does; the gradient passed between layers stays unrounded."""
    rd = bf16_round if bf16 else (lambda a: a)
    nl = len(arch.widths)
    grads = {}

    def conv_back(name, g, act=True):
        if act:
            g = relu_backward(cache["out"][name], g)
        g = rd(g)   # the masked output gradient is an operand of both products
        gx, gw, gb = conv3d_backward(cache["in"][name], rd(params[name + ".w"]), g)
        grads[name + ".w"] = gw
        grads[name + ".b"] = gb
        return gx

    # decoder: forward order was d_{nl-2}, ..., d_0, out
    g = conv_back("out", gy, act=False)
    gskip = [None] * nl
    for i in range(0, nl - 1):
        gcat = conv_back(f"d{i}", g)
        cup = gcat.shape[3] - arch.widths[i]
        gskip[i] = gcat[..., cup:]
        g = upsample2_backward(gcat[..., :cup])
    # g is now the gradient of the deepest encoder output
    for i in range(nl - 1, -1, -1):
        if gskip[i] is not None:
            g = g + gskip[i]
        g = conv_back(f"e{i}b", g)
        g = conv_back(f"e{i}a", g)
        if i > 0:
            g = pool2_backward(g)
    return grads


# ---------------------------------------------------------------------------------------
# energy loss of the projected start-vector error, scale-free in y
# ---------------------------------------------------------------------------------------
def energy_loss(y: np.ndarray, P1b: np.ndarray, P1A, c: float, sigma: float = 0.0
                ) -> Tuple[float, np.ndarray, float]:
    """Energy-norm error of the projected start vector, relative to ||P2 x*||_A^2 = c with
    c = (x*, P1 b). (P1 A = A P2 is symmetric and P2^T A P2 = P1 A, so ||P2 e||_A^2 =
    (e, P1 A e); with A x* = b, P1 A x* = P1 b.) With u = (y, P1 b), v = (y, P1 A y):
      sigma > 0: regression of y on the scaled solution t = x* / sigma,
        L = ||P2 (y - t)||_A^2 / ||P2 t||_A^2 = (sigma^2 v - 2 sigma u + c) / c,
        dL/dy = 2 (sigma^2 P1 A y - sigma P1 b) / c;
      sigma = 0: the same error for the best multiple alpha y,
        L = 1 - u^2 / (v c),  dL/dy = (2u / (v c)) ((u / v) P1 A y - P1 b).
    Returns L, dL/dy and the best scale alpha = u / v (0, the zero start, when v = 0).
    P1A is a callable v -> P1 A v."""
    yv = y.reshape(-1)
    u = float(yv @ P1b)
    Ay = P1A(yv)
    v = float(yv @ Ay)
    if sigma > 0.0:
        L = (sigma * sigma * v - 2.0 * sigma * u + c) / c
        grad = (2.0 / c) * (sigma * sigma * Ay - sigma * P1b)
    elif v > 0.0:
        L = 1.0 - u * u / (v * c)
        grad = (2.0 * u / (v * c)) * ((u / v) * Ay - P1b)
    else:                       # no direction: the zero start
        L, grad = 1.0, np.zeros_like(yv)
    return L, grad.reshape(y.shape), (u / v if v > 0.0 else 0.0)


def weighted_l2_loss(y: np.ndarray, t: np.ndarray, d: np.ndarray) -> Tuple[float, np.ndarray]:
    """Training regression of the output y on the target t with cell weights d > 0:
    L = sum d (y - t)^2 / sum d t^2, dL/dy = 2 d (y - t) / sum d t^2 (all cells)."""
    yv, tv, dv = y.reshape(-1), t.reshape(-1), d.reshape(-1)
    den = float(np.sum(dv * tv * tv))
    e = yv - tv
    return float(np.sum(dv * e * e)) / den, (2.0 * dv * e / den).reshape(y.shape)


def cell_diag(Tx: np.ndarray, Ty: np.ndarray, Tz: np.ndarray, grid) -> np.ndarray:
    """diag(A) of the two-point flux matrix: the sum of the six face transmissibilities
    of each cell (face arrays in the (nx+1) ny nz, nx (ny+1) nz, nx ny (nz+1) layouts)."""
    nx, ny, nz = grid
    tx = Tx.reshape(nz, ny, nx + 1)
    ty = Ty.reshape(nz, ny + 1, nx)
    tz = Tz.reshape(nz + 1, ny, nx)
    d = tx[:, :, :-1] + tx[:, :, 1:] + ty[:, :-1, :] + ty[:, 1:, :] + tz[:-1] + tz[1:]
    return d.reshape(-1)


# ---------------------------------------------------------------------------------------
# Adam (Kingma & Ba), bias-corrected
# ---------------------------------------------------------------------------------------
def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One update at step t >= 1; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------------------
# network inputs
# ---------------------------------------------------------------------------------------
def make_input(K: np.ndarray, b: np.ndarray, grid) -> np.ndarray:
    """Two channels: log10 K standardised over the grid, and b divided by max |b|."""
    nx, ny, nz = grid
    lk = np.log10(K)
    lk = (lk - lk.mean()) / max(lk.std(), 1e-12)
    bm = np.abs(b).max()
    bb = b / bm if bm > 0 else b * 0.0
    return np.stack([lk.reshape(nz, ny, nx), bb.reshape(nz, ny, nx)], axis=3)
