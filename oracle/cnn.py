"""FP64 reference of the convolutional coarse propagator G (Section 3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network of Section 3.2 maps U_n to an approximation of U_{n+1}: 3x3
convolutions with "circular" (periodic) padding of 1, an activation after
every convolution except the last, no pooling and no dense layers, and
optionally a uniform shift that restores the mass of the input (the mass
fix of the conservative model) followed by a bound limiter (the maximum
principle).  The workloads fix the stack as a plain chain of convolutions
1 -> C -> ... -> C -> 1 with GELU (the exact erf form) and a global
residual, G(u) = u + net(u).

Weights follow torch.nn.Conv2d: W[l] has shape [C_out, C_in, 3, 3], the
operation is a cross-correlation, out[co, y, x] = b[co] +
sum_{ci, ky, kx} W[co, ci, ky, kx] * in[ci, y + ky - 1, x + kx - 1] with
indices taken modulo N.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch
import torch.nn.functional as Fnn


@dataclass
class CnnSpec:
    """Layer widths, activation and output options of the coarse network."""
    n_layers: int
    channels: int
    act: str = "gelu"           # "gelu" (exact erf) or "tanh"
    residual: bool = True       # G(u) = u + net(u)
    mass_fix: bool = False      # add mean(u) - mean(G(u)) uniformly
    limiter: Optional[tuple] = None   # (lo, hi) clamp after the mass fix

    def widths(self) -> List[int]:
        return [1] + [self.channels] * (self.n_layers - 1) + [1]


def init_weights(spec: CnnSpec, seed: int, scale: float = 1.0):
    """torch.nn.Conv2d default initialisation under torch.manual_seed(seed),
    in float64; returns ([W_l], [b_l]).  `scale` multiplies the last layer
    (a small last layer makes the untrained G close to the identity)."""
    g = torch.Generator().manual_seed(seed)
    ws, bs = [], []
    w = spec.widths()
    for l in range(spec.n_layers):
        cin, cout = w[l], w[l + 1]
        bound = 1.0 / math.sqrt(cin * 9)
        W = (torch.rand((cout, cin, 3, 3), generator=g, dtype=torch.float64) * 2 - 1) * bound
        b = (torch.rand((cout,), generator=g, dtype=torch.float64) * 2 - 1) * bound
        if l == spec.n_layers - 1:
            W = W * scale
            b = b * scale
        ws.append(W)
        bs.append(b)
    return ws, bs


def gelu_exact(x: torch.Tensor) -> torch.Tensor:
    """GELU in its exact form x * Phi(x) = x/2 (1 + erf(x / sqrt 2))."""
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def _act(x, name):
    return gelu_exact(x) if name == "gelu" else torch.tanh(x)


def conv3x3_periodic(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """3x3 cross-correlation with circular padding 1 (library conv2d)."""
    return Fnn.conv2d(Fnn.pad(x, (1, 1, 1, 1), mode="circular"), W, b)


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (round to nearest even) and back to float64."""
    return x.to(torch.bfloat16).to(torch.float64)


def forward(u, weights: Sequence[torch.Tensor], biases: Sequence[torch.Tensor],
            spec: CnnSpec, emulate_bf16=False) -> np.ndarray:
    """G(u) for u [B, N, N] (numpy or torch); returns float64 numpy.

    emulate_bf16 = True (or "all"): the activations after every layer but
    the last, and the weights of the hidden (C -> C) layers, are rounded to
    bfloat16 where a bfloat16 kernel stores them (the first and last layers
    keep their weights and the first reads the state unrounded);
    "weights": only those weights are rounded.
    All sums stay float64."""
    round_w = emulate_bf16 in (True, "all", "weights")
    round_a = emulate_bf16 in (True, "all")
    ut = torch.as_tensor(np.asarray(u, dtype=np.float64))
    x = ut[:, None]
    L = spec.n_layers
    for l in range(L):
        W, b = weights[l].to(torch.float64), biases[l].to(torch.float64)
        if round_w and 0 < l < L - 1:
            W = bf16(W)
        x = conv3x3_periodic(x, W, b)
        if l < L - 1:
            x = _act(x, spec.act)
            if round_a:
                x = bf16(x)
    net = x[:, 0]
    out = ut + net if spec.residual else net
    if spec.mass_fix:
        out = out + (ut.mean(dim=(-2, -1), keepdim=True) - out.mean(dim=(-2, -1), keepdim=True))
    if spec.limiter is not None:
        out = out.clamp(spec.limiter[0], spec.limiter[1])
    return out.numpy()


def conv3x3_periodic_loops(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The same cross-correlation written out with shifts, for pinning."""
    cin = x.shape[1]
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for co in range(W.shape[0]):
        acc = np.full((x.shape[0],) + x.shape[2:], b[co])
        for ci in range(cin):
            for ky in range(3):
                for kx in range(3):
                    # in[y + ky - 1, x + kx - 1] = roll by -(ky - 1)
                    shifted = np.roll(x[:, ci], shift=(1 - ky, 1 - kx), axis=(-2, -1))
                    acc = acc + W[co, ci, ky, kx] * shifted
        out[:, co] = acc
    return out
