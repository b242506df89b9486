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
    """Each value rounded to the nearest bfloat16 number (8 significant
    bits), ties to the one with an even last bit, in a single rounding from
    float64; returned as float64.  Normal-range values only (weights and
    activations of the network).  Gradients pass straight through."""
    xd = x.detach().to(torch.float64)
    m, e = torch.frexp(xd)                  # xd = m 2^e, 1/2 <= |m| < 1
    r = torch.ldexp(torch.round(m * 256.0), (e - 8).to(torch.float64))
    return x + (r - xd)


PRECISIONS = ("exact", "bf16", "bf16x2")


def rounding_plan(prec: str, n_layers: int):
    """Which numbers a network of the given number format rounds to bfloat16.

    Section 3.2's network is a chain of 3x3 convolutions; the workloads run
    it on the bfloat16 matrix cores with FP32 accumulation.  The dense
    contractions are the hidden convolutions C -> C, and those are what
    take bfloat16 operands:

      "exact"   nothing is rounded (float64 throughout);
      "bf16"    the weights of every hidden layer (0 < l < L-1) and every
                activation a layer hands on (the output of layers
                0 .. L-2, after the activation function) are rounded to
                bfloat16; the first layer (1 -> C, nine taps per output)
                keeps its weights and reads the state unrounded, and the
                last layer (C -> 1) keeps its weights;
      "bf16x2"  the split form: the same bfloat16 hidden weights, with each
                activation carried as a pair hi + lo of bfloat16 numbers
                (16 significant bits or more), taken here as unrounded.

    Returns (round_weights[l], round_activation[l]) for l = 0 .. L-1.
    All sums stay float64; the GPU's FP32 accumulation and its hi + lo
    pairs differ from this by FP32-level roundings, well inside the test
    tolerances derived from them."""
    if prec not in PRECISIONS:
        raise ValueError(f"unknown network precision {prec!r}")
    L = n_layers
    rw = [prec != "exact" and 0 < l < L - 1 for l in range(L)]
    ra = [prec == "bf16" and l < L - 1 for l in range(L)]
    return rw, ra


def forward(u, weights: Sequence[torch.Tensor], biases: Sequence[torch.Tensor],
            spec: CnnSpec, prec: str = "exact") -> np.ndarray:
    """G(u) for u [B, N, N] (numpy or torch); returns float64 numpy.

    `prec` is the network's number format, as `rounding_plan` defines it;
    "exact" is the network itself in float64."""
    rw, ra = rounding_plan(prec, spec.n_layers)
    ut = torch.as_tensor(np.asarray(u, dtype=np.float64))
    x = ut[:, None]
    L = spec.n_layers
    for l in range(L):
        W, b = weights[l].to(torch.float64), biases[l].to(torch.float64)
        if rw[l]:
            W = bf16(W)
        x = conv3x3_periodic(x, W, b)
        if l < L - 1:
            x = _act(x, spec.act)
        if ra[l]:
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
