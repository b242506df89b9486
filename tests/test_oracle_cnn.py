"""Pins of the FP64 coarse-network oracle (Section 3.2)."""

import math

import numpy as np
import pytest
import torch

from oracle import cnn
from paper_2510_07672_amd import synth


def _spec(**kw):
    d = dict(n_layers=4, channels=8)
    d.update(kw)
    return cnn.CnnSpec(**d)


def test_conv_matches_shift_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 9, 7))
    W = rng.standard_normal((5, 3, 3, 3))
    b = rng.standard_normal(5)
    lib = cnn.conv3x3_periodic(torch.from_numpy(x), torch.from_numpy(W), torch.from_numpy(b)).numpy()
    ref = cnn.conv3x3_periodic_loops(x, W, b)
    assert np.abs(lib - ref).max() <= 1e-13


def test_conv_of_a_delta_is_the_flipped_kernel():
    # a unit impulse at (y0, x0): out[y, x] = W[y0 - y + 1, x0 - x + 1]
    x = np.zeros((1, 1, 8, 8))
    x[0, 0, 3, 5] = 1.0
    W = np.arange(9, dtype=float).reshape(1, 1, 3, 3)
    out = cnn.conv3x3_periodic(torch.from_numpy(x), torch.from_numpy(W), torch.zeros(1, dtype=torch.float64)).numpy()[0, 0]
    for ky in range(3):
        for kx in range(3):
            assert out[3 - ky + 1, 5 - kx + 1] == W[0, 0, ky, kx]
    assert np.count_nonzero(out) == 8  # W[0,0,0,0] = 0


def test_gelu_identities():
    x = torch.linspace(-6, 6, 101, dtype=torch.float64)
    g = cnn.gelu_exact(x)
    assert torch.allclose(g - cnn.gelu_exact(-x), x, atol=1e-15, rtol=0)   # Phi(x)+Phi(-x)=1
    assert cnn.gelu_exact(torch.zeros(1)).item() == 0.0
    # x Phi(x) at x = 1: Phi(1) = 0.8413447460685429 (standard normal table)
    assert abs(cnn.gelu_exact(torch.ones(1, dtype=torch.float64)).item() - 0.8413447460685429) <= 1e-15


def test_constant_input_follows_scalar_chain():
    spec = _spec(residual=True)
    ws, bs = cnn.init_weights(spec, seed=3)
    c = 0.37
    u = np.full((1, 16, 16), c)
    out = cnn.forward(u, ws, bs, spec)
    # by hand: each layer maps per-channel constants v to b + (sum_kernel W) v
    v = np.array([c])
    for l in range(spec.n_layers):
        Wsum = ws[l].numpy().sum(axis=(2, 3))         # [cout, cin]
        v = bs[l].numpy() + Wsum @ v
        if l < spec.n_layers - 1:
            v = 0.5 * v * (1 + np.vectorize(math.erf)(v / math.sqrt(2)))
    assert np.abs(out - (c + v[0])).max() <= 1e-14


@pytest.mark.parametrize("act", ["gelu", "tanh"])
def test_shift_equivariance(act):
    spec = _spec(act=act)
    ws, bs = cnn.init_weights(spec, seed=1)
    u = synth.random_ic(16, [4])
    a = cnn.forward(np.roll(u, (3, -5), axis=(1, 2)), ws, bs, spec)
    b = np.roll(cnn.forward(u, ws, bs, spec), (3, -5), axis=(1, 2))
    assert np.abs(a - b).max() <= 1e-13


def test_mass_fix_and_limiter():
    spec = _spec(mass_fix=True)
    ws, bs = cnn.init_weights(spec, seed=2)
    u = synth.random_ic(16, [5, 6])
    out = cnn.forward(u, ws, bs, spec)
    assert np.abs(out.mean(axis=(1, 2)) - u.mean(axis=(1, 2))).max() <= 1e-15
    spec_l = _spec(limiter=(-0.5, 0.5))
    out = cnn.forward(u, ws, bs, spec_l)
    assert out.min() >= -0.5 and out.max() <= 0.5


def test_zero_output_layer_gives_identity():
    spec = _spec()
    ws, bs = cnn.init_weights(spec, seed=7, scale=0.0)
    u = synth.random_ic(16, [8])
    assert np.array_equal(cnn.forward(u, ws, bs, spec), u)


def test_bf16_emulation_is_close_and_not_equal():
    spec = _spec(channels=16)
    ws, bs = cnn.init_weights(spec, seed=9)
    u = synth.random_ic(32, [1])
    a = cnn.forward(u, ws, bs, spec)
    b = cnn.forward(u, ws, bs, spec, emulate_bf16=True)
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 1e-6 < rel < 1e-2


def test_pins_catch_zero_padding(monkeypatch):
    def zero_pad(x, W, b):
        return torch.nn.functional.conv2d(x, W, b, padding=1)
    monkeypatch.setattr(cnn, "conv3x3_periodic", zero_pad)
    with pytest.raises(AssertionError):
        test_shift_equivariance("gelu")
