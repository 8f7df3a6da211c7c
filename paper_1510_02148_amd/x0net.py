"""Learned start vector: a 4-level 3D encoder/decoder run on libpsl's bf16 matrix-core
kernels, trained on solutions of the plain solver, predicting x0 for psl_solve.

Inputs (8 channels, 2 used): log10 K standardised over the grid and b / max |b|. The
network output y gives the start vector x0 = alpha y with the energy-optimal scale
alpha = (y, P1 b) / (y, P1 A y): it minimises ||P2 (alpha y - x*)||_A over alpha, and
alpha = 0 (the zero start) is among the candidates, so the scaled start is never worse
than x0 = 0 in that norm. Training minimises the same kind of error relative to ||P2 x*||_A^2
(energy-norm regression on x* / rms(x*), whose gradient needs only P1 A y, P1 b and
(x*, P1 b); the scale-free form 1 - cos^2 of the angle has no gradient at a random
start, where the output is almost orthogonal to x*).

Layout: activations channels-last bf16 (operands of the matrix products), gradients
float32; master weights float32 [Cout][27 Cin] with Adam moments, packed bf16 operands
for the forward product and a flipped, transposed copy for the input gradient.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import nn, psl

WIDTHS = (16, 32, 48, 64)
CIN = 8          # input channels as stored (2 used, zero-padded to the operand width)
CIN_USED = 2


def layer_table(widths: Sequence[int] = WIDTHS) -> List[Tuple[str, int, int, int, int]]:
    """(name, Cout, taps, Cin, level) of every convolution in evaluation order."""
    w = widths
    out = [("e0a", w[0], 27, CIN, 0), ("e0b", w[0], 27, w[0], 0)]
    for i in range(1, len(w)):
        out += [(f"e{i}a", w[i], 27, w[i - 1], i), (f"e{i}b", w[i], 27, w[i], i)]
    for i in range(len(w) - 2, -1, -1):
        out += [(f"d{i}", w[i], 27, w[i + 1] + w[i], i)]
    out += [("out", 1, 1, w[0], 0)]
    return out


class X0Net:
    """Parameters, activations and workspaces of the network for one grid shape."""

    def __init__(self, grid: Sequence[int], widths: Sequence[int] = WIDTHS, seed: int = 0):
        nx, ny, nz = (int(v) for v in grid)
        nl = len(widths)
        if nx % (8 << (nl - 1)) or ny % (1 << (nl - 1)) or nz % (1 << (nl - 1)):
            raise ValueError("grid extents must halve evenly at every level (nx a multiple "
                             f"of {8 << (nl - 1)} for the weight gradient)")
        self.widths = tuple(int(v) for v in widths)
        self.nl = nl
        self.grids = [(nx >> i, ny >> i, nz >> i) for i in range(nl)]
        self.ns = [a * b * c for a, b, c in self.grids]
        self.layers = layer_table(self.widths)
        self.step = 0
        dev = "cuda"
        f32 = dict(dtype=torch.float32, device=dev)
        g = np.random.Generator(np.random.PCG64(seed))
        self.P: Dict[str, dict] = {}
        for name, cout, taps, cin, lvl in self.layers:
            fan_in = taps * (CIN_USED if name == "e0a" else cin)
            if taps == 27:
                p = g.normal(0.0, math.sqrt(2.0 / fan_in), (cout, 27, cin))
                if name == "e0a":
                    p[:, :, CIN_USED:] = 0.0            # padding channels carry no input
                L = dict(p=torch.tensor(p.reshape(cout, -1), **f32), pb=torch.zeros(cout, **f32))
                L["w"] = nn.bf16_empty(cout, nn.kp(cin), zero=True)
                L["wt"] = (nn.bf16_empty(cin, nn.kp(cout), zero=True) if name != "e0a" else None)
                L["dw"] = torch.zeros(cout, nn.kp(cin) + 16, **f32)
            else:
                # the output layer starts at zero: the untrained network predicts the zero
                # start (loss 1) and training moves away from it only where that helps
                p = np.zeros(cin)
                L = dict(p=torch.tensor(np.concatenate([p, [0.0]]), **f32))   # bias last
                L["w"] = nn.bf16_empty(cin, zero=True)
                L["dw"] = torch.zeros(cin + 1, **f32)
            for k in ("p", "pb"):
                if k in L:
                    L["m" + k[1:]] = torch.zeros_like(L[k])
                    L["v" + k[1:]] = torch.zeros_like(L[k])
            L.update(cout=cout, cin=cin, taps=taps, level=lvl)
            self.P[name] = L
        self._pack()
        # activations (bf16) and gradients (float32)
        A = {}
        for i in range(nl):
            n, c = self.ns[i], self.widths[i]
            if i > 0:
                A[f"pool{i}"] = nn.bf16_empty(n, self.widths[i - 1])
            A[f"e{i}a"] = nn.bf16_empty(n, c)
            A[f"e{i}b"] = nn.bf16_empty(n, c)
        for i in range(nl - 2, -1, -1):
            n, c = self.ns[i], self.widths[i]
            A[f"cat{i}"] = nn.bf16_empty(n, self.widths[i + 1] + c)
            A[f"d{i}"] = nn.bf16_empty(n, c)
        A["x"] = nn.bf16_empty(self.ns[0], CIN, zero=True)
        A["y"] = torch.empty(self.ns[0], **f32)
        self.A = A
        wmax = max(nn.wgrad_work(self.grids[L["level"]], L["cin"], L["cout"])
                   for L in self.P.values() if L["taps"] == 27)
        self.work = torch.empty(max(wmax, nn.conv1_work(self.ns[0], self.widths[0])), **f32)
        self.dwork = torch.empty(max(nn.input_work(self.ns[0]), nn.energy_work(self.ns[0]),
                                     nn.wl2_work(self.ns[0])), dtype=torch.float64, device=dev)
        self.eout = torch.zeros(4, dtype=torch.float64, device=dev)
        cmax = max(self.widths[i + 1] + self.widths[i] for i in range(nl - 1))
        self.g_a = torch.empty(self.ns[0] * cmax, **f32)       # gradient scratch
        self.g_b = torch.empty(self.ns[0] * cmax, **f32)
        self.gq = nn.bf16_empty(self.ns[0] * cmax)
        self.gskip = [torch.empty(self.ns[i] * self.widths[i], **f32) for i in range(nl)]
        self.gy = torch.empty(self.ns[0], **f32)
        self.y64 = torch.empty(self.ns[0], dtype=torch.float64, device=dev)
        self.Ay = torch.empty_like(self.y64)

    # ---------------------------------------------------------------- parameters
    def _pack(self):
        for name, L in self.P.items():
            if L["taps"] == 27:
                nn.adam_conv(L["cout"], L["cin"], L["p"], L["m"], L["v"], L["pb"], L["mb"],
                             L["vb"], None, 0, 0.0, L["w"], L["wt"])
            else:
                nn.adam_vec(L["p"], L["m"], L["v"], None, 0, 0.0, L["w"])

    def export_params(self) -> Dict[str, np.ndarray]:
        """Float32 master parameters in the (Cout, taps, Cin) layout, float64 copies; the
        first layer keeps only its used input channels."""
        out = {}
        for name, L in self.P.items():
            if L["taps"] == 27:
                w = L["p"].double().cpu().numpy().reshape(L["cout"], 27, L["cin"])
                if name == "e0a":
                    w = w[:, :, :CIN_USED]
                out[name + ".w"] = w
                out[name + ".b"] = L["pb"].double().cpu().numpy()
            else:
                p = L["p"].double().cpu().numpy()
                out[name + ".w"] = p[:-1].reshape(1, 1, -1)
                out[name + ".b"] = p[-1:]
        return out

    def load_params(self, params: Dict[str, np.ndarray]):
        for name, L in self.P.items():
            w = np.asarray(params[name + ".w"], dtype=np.float64)
            if L["taps"] == 27:
                if name == "e0a" and w.shape[2] != L["cin"]:
                    full = np.zeros((L["cout"], 27, L["cin"]))
                    full[:, :, :w.shape[2]] = w
                    w = full
                L["p"].copy_(torch.tensor(w.reshape(L["cout"], -1), dtype=torch.float32))
                L["pb"].copy_(torch.tensor(params[name + ".b"], dtype=torch.float32))
            else:
                L["p"].copy_(torch.tensor(np.concatenate([w.reshape(-1), params[name + ".b"]]),
                                          dtype=torch.float32))
        self._pack()

    def state_dict(self) -> Dict[str, torch.Tensor]:
        sd = {}
        for name, L in self.P.items():
            for k in ("p", "pb", "m", "v", "mb", "vb"):
                if k in L:
                    sd[f"{name}.{k}"] = L[k].detach().cpu()
        sd["step"] = torch.tensor(self.step)
        return sd

    def load_state_dict(self, sd: Dict[str, torch.Tensor]):
        for name, L in self.P.items():
            for k in ("p", "pb", "m", "v", "mb", "vb"):
                if k in L:
                    L[k].copy_(sd[f"{name}.{k}"].to(L[k].device))
        self.step = int(sd["step"])
        self._pack()

    # ---------------------------------------------------------------- forward / backward
    def set_input(self, K: torch.Tensor, b: torch.Tensor):
        nn.make_input(K, b, self.A["x"], self.dwork)

    def forward(self) -> torch.Tensor:
        """Runs the network on the current input; returns y (float32 [n], a view)."""
        A, P = self.A, self.P
        h = A["x"]
        for i in range(self.nl):
            grid = self.grids[i]
            if i > 0:
                nn.pool2(self.grids[i - 1], A[f"e{i - 1}b"], self.widths[i - 1], A[f"pool{i}"])
                h = A[f"pool{i}"]
            for s in ("a", "b"):
                L = P[f"e{i}{s}"]
                nn.conv3(grid, h, L["cin"], L["w"], L["cout"], L["pb"], True, A[f"e{i}{s}"])
                h = A[f"e{i}{s}"]
        for i in range(self.nl - 2, -1, -1):
            L = P[f"d{i}"]
            nn.upcat(self.grids[i], h, self.widths[i + 1], A[f"e{i}b"], self.widths[i],
                     A[f"cat{i}"])
            nn.conv3(self.grids[i], A[f"cat{i}"], L["cin"], L["w"], L["cout"], L["pb"], True,
                     A[f"d{i}"])
            h = A[f"d{i}"]
        L = P["out"]
        nn.conv1(self.ns[0], h, L["cin"], L["w"], L["p"][-1:], A["y"])
        return A["y"]

    def _conv_back(self, name: str, g: torch.Tensor, x_in: torch.Tensor,
                   gx: Optional[torch.Tensor]):
        """Layer `name` with output gradient g (float32): weight gradient into dw, input
        gradient into gx (float32) unless gx is None."""
        L = self.P[name]
        grid = self.grids[L["level"]]
        n = self.ns[L["level"]]
        gq = self.gq[: n * L["cout"]]
        nn.relu_grad(g[: n * L["cout"]], self.A[name], gq, relu=True)
        nn.conv3_wgrad(grid, gq, L["cout"], x_in, L["cin"], L["dw"], self.work)
        if gx is not None:
            nn.conv3(grid, gq, L["cout"], L["wt"], L["cin"], None, False, None, gx[: n * L["cin"]])

    def backward(self, gy: torch.Tensor):
        """Parameter gradients (into each layer's dw) for the output gradient gy [n].

        Buffers: g_a holds the gradient of the current layer's output, g_b receives input
        gradients, gskip[i] collects level i's encoder-output gradient (skip part from
        the decoder, plus the pooled path from level i + 1)."""
        A, P, w, nl = self.A, self.P, self.widths, self.nl
        g_a, g_b = self.g_a, self.g_b
        L = P["out"]
        n0 = self.ns[0]
        nn.conv1_grad(n0, gy, A["d0"], L["cin"], L["w"], g_a[: n0 * L["cin"]], L["dw"], self.work)
        for i in range(0, nl - 1):                       # decoder, last applied first
            ncat = self.ns[i] * (w[i + 1] + w[i])
            self._conv_back(f"d{i}", g_a, A[f"cat{i}"], g_b)
            nn.upcat_grad(self.grids[i], g_b[:ncat], w[i + 1], w[i],
                          g_a[: self.ns[i + 1] * w[i + 1]], self.gskip[i])
        for i in range(nl - 1, -1, -1):                  # encoder, deepest level first
            g_out = g_a if i == nl - 1 else self.gskip[i]
            self._conv_back(f"e{i}b", g_out, A[f"e{i}a"], g_b)
            self._conv_back(f"e{i}a", g_b, A["x"] if i == 0 else A[f"pool{i}"],
                            g_a if i > 0 else None)
            if i > 0:
                nn.pool2_grad_add(self.grids[i - 1], g_a[: self.ns[i] * w[i - 1]], w[i - 1],
                                  self.gskip[i - 1])

    def adam(self, lr: float = 1e-3):
        self.step += 1
        for L in self.P.values():
            if L["taps"] == 27:
                nn.adam_conv(L["cout"], L["cin"], L["p"], L["m"], L["v"], L["pb"], L["mb"],
                             L["vb"], L["dw"], self.step, lr, L["w"], L["wt"])
            else:
                nn.adam_vec(L["p"], L["m"], L["v"], L["dw"], self.step, lr, L["w"])

    # ---------------------------------------------------------------- loss and start vector
    def energy(self, ctx: psl.Context, P1b: torch.Tensor, c: float, grad: bool,
               x0: Optional[torch.Tensor] = None, sigma: float = 0.0):
        """Energy loss of alpha y for the current output (P1 A y through the solver's own
        operators; c = (x*, P1 b), 0 when unknown): the regression on x* / sigma when
        sigma > 0, else the error of the best multiple. Fills self.gy when grad; x0
        (float64) receives alpha y when given. Returns the device tensor {L, alpha, u, v}."""
        y = self.A["y"]
        nn.widen(y, self.y64)
        psl.psl_apply_A(ctx, self.y64, self.Ay)
        psl.psl_deflate(ctx, self.Ay, self.Ay)
        nn.energy(y, P1b, self.Ay, c, self.eout, self.dwork, gy=self.gy if grad else None,
                  x0=x0, sigma=sigma)
        return self.eout

    def train_step(self, K, b, lr=1e-3, *, target=None, weight=None, ctx=None, P1b=None,
                   c=0.0, sigma=0.0) -> torch.Tensor:
        """One Adam step. With target/weight: the weighted regression on target (float32
        [n]); otherwise the energy-norm regression toward x* / sigma through ctx. Returns
        the device tensor whose entry 0 is the loss before the step."""
        self.set_input(K, b)
        self.forward()
        if target is not None:
            nn.wl2(self.A["y"], target, weight, self.eout, self.dwork, gy=self.gy)
            out = self.eout
        else:
            out = self.energy(ctx, P1b, c, grad=True, sigma=sigma)
        self.backward(self.gy)
        self.adam(lr)
        return out

    def predict_x0(self, K, b, ctx, P1b: Optional[torch.Tensor] = None,
                   x0: Optional[torch.Tensor] = None) -> torch.Tensor:
        """x0 = alpha y for psl_solve(use_x0=1)."""
        if P1b is None:
            P1b = torch.empty_like(b)
            psl.psl_deflate(ctx, b, P1b)
        x0 = torch.empty_like(b) if x0 is None else x0
        self.set_input(K, b)
        self.forward()
        self.energy(ctx, P1b, 0.0, grad=False, x0=x0)
        return x0
