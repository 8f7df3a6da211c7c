"""ctypes binding of the start-vector network kernels (include/psl_nn.h): argument
marshalling only; every operation runs in libpsl's HIP kernels."""
from __future__ import annotations

import ctypes

import torch

from .psl import _lib, _check, _stream, psl_grid, _grid

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F = ctypes.c_float
_D = ctypes.c_double
_G = ctypes.POINTER(psl_grid)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_kp = _sig("psl_nn_kp", _I32, [_I32])
_conv3 = _sig("psl_nn_conv3", ctypes.c_int, [_G, _P, _I32, _P, _I32, _P, _I32, _P, _P, _P])
_wgrad_work = _sig("psl_nn_wgrad_work", _I64, [_G, _I32, _I32])
_wgrad = _sig("psl_nn_conv3_wgrad", ctypes.c_int, [_G, _P, _I32, _P, _I32, _P, _P, _P])
_relu_grad = _sig("psl_nn_relu_grad", ctypes.c_int, [_I64, _P, _P, _I32, _P, _P])
_pool2 = _sig("psl_nn_pool2", ctypes.c_int, [_G, _P, _I32, _P, _P])
_pool2_grad_add = _sig("psl_nn_pool2_grad_add", ctypes.c_int, [_G, _P, _I32, _P, _P])
_upcat = _sig("psl_nn_upcat", ctypes.c_int, [_G, _P, _I32, _P, _I32, _P, _P])
_upcat_grad = _sig("psl_nn_upcat_grad", ctypes.c_int, [_G, _P, _I32, _I32, _P, _P, _P])
_conv1 = _sig("psl_nn_conv1", ctypes.c_int, [_I64, _P, _I32, _P, _P, _P, _P])
_conv1_work = _sig("psl_nn_conv1_work", _I64, [_I64, _I32])
_conv1_grad = _sig("psl_nn_conv1_grad", ctypes.c_int, [_I64, _P, _P, _I32, _P, _P, _P, _P, _P])
_input_work = _sig("psl_nn_input_work", _I64, [_I64])
_make_input = _sig("psl_nn_make_input", ctypes.c_int, [_I64, _P, _P, _P, _P, _P])
_energy_work = _sig("psl_nn_energy_work", _I64, [_I64])
_energy = _sig("psl_nn_energy", ctypes.c_int, [_I64, _P, _P, _P, _D, _D, _P, _P, _P, _P, _P])
_widen = _sig("psl_nn_widen", ctypes.c_int, [_I64, _P, _P, _P])
_wl2_work = _sig("psl_nn_wl2_work", _I64, [_I64])
_wl2 = _sig("psl_nn_wl2", ctypes.c_int, [_I64, _P, _P, _P, _P, _P, _P, _P])
_cell_diag = _sig("psl_nn_cell_diag", ctypes.c_int, [_G, _P, _P, _P, _P, _P])
_adam_conv = _sig("psl_nn_adam_conv", ctypes.c_int,
                  [_I32, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _F, _F, _F, _F, _P, _P, _P])
_adam_vec = _sig("psl_nn_adam_vec", ctypes.c_int, [_I32, _P, _P, _P, _P, _I32, _F, _F, _F, _F,
                                                   _P, _P])

EXPORTED = tuple(f.__name__ for f in (_kp, _conv3, _wgrad_work, _wgrad, _relu_grad, _pool2,
                                      _pool2_grad_add, _upcat, _upcat_grad, _conv1, _conv1_work,
                                      _conv1_grad, _input_work, _make_input, _energy_work,
                                      _energy, _widen, _adam_conv, _adam_vec, _wl2_work, _wl2,
                                      _cell_diag))


def _p(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return t.data_ptr()


def kp(cin: int) -> int:
    return int(_kp(int(cin)))


def bf16_empty(*shape, zero=False):
    """Device buffer of bfloat16 bit patterns (held as int16: same bits, full torch support)."""
    f = torch.zeros if zero else torch.empty
    return f(*shape, dtype=torch.int16, device="cuda")


def conv3(grid, x, cin, w, cout, bias=None, relu=True, y=None, yf=None):
    g = _grid(grid)
    _check(_conv3(ctypes.byref(g), _p(x), cin, _p(w), cout, _p(bias), 1 if relu else 0, _p(y),
                  _p(yf), _stream()), "psl_nn_conv3")


def wgrad_work(grid, cin, cout) -> int:
    g = _grid(grid)
    return int(_wgrad_work(ctypes.byref(g), cin, cout))


def conv3_wgrad(grid, gy, cout, x, cin, dw, work):
    g = _grid(grid)
    _check(_wgrad(ctypes.byref(g), _p(gy), cout, _p(x), cin, _p(dw), _p(work), _stream()),
           "psl_nn_conv3_wgrad")


def relu_grad(gy, y, gq, relu=True):
    _check(_relu_grad(gy.numel(), _p(gy), _p(y), 1 if relu else 0, _p(gq), _stream()),
           "psl_nn_relu_grad")


def pool2(grid, x, c, y):
    g = _grid(grid)
    _check(_pool2(ctypes.byref(g), _p(x), c, _p(y), _stream()), "psl_nn_pool2")


def pool2_grad_add(grid, gy, c, gx):
    g = _grid(grid)
    _check(_pool2_grad_add(ctypes.byref(g), _p(gy), c, _p(gx), _stream()), "psl_nn_pool2_grad_add")


def upcat(grid, h, ca, s, cb, y):
    g = _grid(grid)
    _check(_upcat(ctypes.byref(g), _p(h), ca, _p(s), cb, _p(y), _stream()), "psl_nn_upcat")


def upcat_grad(grid, gy, ca, cb, gh, gs):
    g = _grid(grid)
    _check(_upcat_grad(ctypes.byref(g), _p(gy), ca, cb, _p(gh), _p(gs), _stream()),
           "psl_nn_upcat_grad")


def conv1(n, h, cin, w, bias, y):
    _check(_conv1(n, _p(h), cin, _p(w), _p(bias), _p(y), _stream()), "psl_nn_conv1")


def conv1_work(n, cin) -> int:
    return int(_conv1_work(n, cin))


def conv1_grad(n, gy, h, cin, w, gh, dw, work):
    _check(_conv1_grad(n, _p(gy), _p(h), cin, _p(w), _p(gh), _p(dw), _p(work), _stream()),
           "psl_nn_conv1_grad")


def make_input(K, b, x, work):
    _check(_make_input(K.numel(), _p(K), _p(b), _p(x), _p(work), _stream()), "psl_nn_make_input")


def input_work(n) -> int:
    return int(_input_work(n))


def energy(y, P1b, P1Ay, c, out, work, gy=None, x0=None, sigma=0.0):
    _check(_energy(y.numel(), _p(y), _p(P1b), _p(P1Ay), float(c), float(sigma), _p(out), _p(gy),
                   _p(x0), _p(work), _stream()), "psl_nn_energy")


def energy_work(n) -> int:
    return int(_energy_work(n))


def widen(y, y64):
    _check(_widen(y.numel(), _p(y), _p(y64), _stream()), "psl_nn_widen")


def adam_conv(cout, cin, p, m, v, pb, mb, vb, dw, t, lr, w, wt, b1=0.9, b2=0.999, eps=1e-8):
    _check(_adam_conv(cout, cin, _p(p), _p(m), _p(v), _p(pb), _p(mb), _p(vb), _p(dw), int(t),
                      float(lr), float(b1), float(b2), float(eps), _p(w), _p(wt), _stream()),
           "psl_nn_adam_conv")


def adam_vec(p, m, v, dw, t, lr, w, b1=0.9, b2=0.999, eps=1e-8):
    _check(_adam_vec(p.numel(), _p(p), _p(m), _p(v), _p(dw), int(t), float(lr), float(b1),
                     float(b2), float(eps), _p(w), _stream()), "psl_nn_adam_vec")


def wl2_work(n) -> int:
    return int(_wl2_work(n))


def wl2(y, t, d, out, work, gy=None):
    _check(_wl2(y.numel(), _p(y), _p(t), _p(d), _p(out), _p(gy), _p(work), _stream()), "psl_nn_wl2")


def cell_diag(grid, Tx, Ty, Tz, d):
    g = _grid(grid)
    _check(_cell_diag(ctypes.byref(g), _p(Tx), _p(Ty), _p(Tz), _p(d), _stream()),
           "psl_nn_cell_diag")
