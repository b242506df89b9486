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


# ---------------------------------------------------------------- bfloat16
# The network in bfloat16 (oracle.cnn.rounding_plan): hidden-layer weights
# and every activation rounded ("bf16"), or the hidden-layer weights only,
# activations carried as hi + lo pairs ("bf16x2").  Pinned against the
# same network written out with the shift-definition convolution and an
# integer-bit rounding, so that moving any one rounding fails.

def _rne_bf16_bits(x):
    """Round-to-nearest-even to 8 significant bits on the float64 bit
    pattern: add half an ulp of the kept part (minus one, plus the kept
    part's last bit) and clear the 45 dropped bits."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    keep_lsb = (b >> np.uint64(45)) & np.uint64(1)
    b = (b + np.uint64((1 << 44) - 1) + keep_lsb) & ~np.uint64((1 << 45) - 1)
    return b.view(np.float64)


def test_bf16_rounding_literals():
    one = 1.0
    cases = [
        (one + 2.0 ** -8, 1.0),                       # tie -> even (1.0000000)
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),       # tie -> even (1.0000010)
        (one + 2.0 ** -8 + 2.0 ** -40, one + 2.0 ** -7),  # above the tie
        (255.5, 256.0), (254.5, 254.0),               # ties at exponent 7
        (-(one + 2.0 ** -8), -1.0),
        (0.1, 0.10009765625),                         # 0x3DCD
        (1.0 / 3.0, 0.333984375),                     # 0x3EAB
        (0.0, 0.0),
    ]
    x = torch.tensor([c[0] for c in cases], dtype=torch.float64)
    want = [c[1] for c in cases]
    assert cnn.bf16(x).tolist() == want


def test_bf16_rounding_matches_bits_and_library():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))
    got = cnn.bf16(torch.from_numpy(x)).numpy()
    assert np.array_equal(got, _rne_bf16_bits(x))
    # float32 inputs: torch's own float -> bfloat16 conversion rounds once
    x32 = x.astype(np.float32)
    lib = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(torch.from_numpy(x32.astype(np.float64))).numpy(), lib)


def _gelu_np(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def _written_out(u, ws, bs, L, prec):
    """The bfloat16 network by hand: shift-definition convolutions, GELU
    from math.erf, integer-bit rounding of the hidden weights and (bf16)
    of each activation a layer hands on."""
    x = u[:, None]
    for l in range(L):
        W, b = ws[l].numpy(), bs[l].numpy()
        if prec in ("bf16", "bf16x2") and 0 < l < L - 1:
            W = _rne_bf16_bits(W)
        x = cnn.conv3x3_periodic_loops(x, W, b)
        if l < L - 1:
            x = _gelu_np(x)
            if prec == "bf16":
                x = _rne_bf16_bits(x)
    return u + x[:, 0]


@pytest.mark.parametrize("prec", ["bf16", "bf16x2", "exact"])
@pytest.mark.parametrize("L", [3, 4])
def test_bf16_network_is_the_written_out_chain(prec, L):
    spec = _spec(n_layers=L, channels=8)
    ws, bs = cnn.init_weights(spec, seed=13 + L)
    u = synth.random_ic(12, [2, 3])
    got = cnn.forward(u, ws, bs, spec, prec=prec)
    ref = _written_out(u, ws, bs, L, prec)
    assert np.linalg.norm((got - u) - (ref - u)) <= 1e-13 * np.linalg.norm(ref - u)
    if prec != "exact":
        ex = cnn.forward(u, ws, bs, spec)
        d = np.linalg.norm((got - u) - (ex - u)) / np.linalg.norm(ex - u)
        assert 1e-5 < d < 1e-2      # the roundings are there, and small


@pytest.mark.parametrize("move", ["first_weights", "last_weights", "no_act_round_l0",
                                  "round_last_output", "split_rounds_acts", "no_hidden_weights"])
def test_pins_catch_a_moved_rounding(monkeypatch, move):
    orig = cnn.rounding_plan

    def moved(prec, L):
        rw, ra = orig(prec, L)
        rw, ra = list(rw), list(ra)
        if move == "first_weights":
            rw[0] = prec != "exact"
        elif move == "last_weights":
            rw[L - 1] = prec != "exact"
        elif move == "no_act_round_l0":
            ra[0] = False
        elif move == "round_last_output":
            ra[L - 1] = prec == "bf16"
        elif move == "split_rounds_acts":
            ra = [prec == "bf16x2" and l < L - 1 for l in range(L)] if prec == "bf16x2" else ra
        elif move == "no_hidden_weights":
            rw = [False] * L
        return rw, ra
    monkeypatch.setattr(cnn, "rounding_plan", moved)
    prec = "bf16x2" if move == "split_rounds_acts" else "bf16"
    with pytest.raises(AssertionError):
        test_bf16_network_is_the_written_out_chain(prec, 4)


def test_pins_catch_zero_padding(monkeypatch):
    def zero_pad(x, W, b):
        return torch.nn.functional.conv2d(x, W, b, padding=1)
    monkeypatch.setattr(cnn, "conv3x3_periodic", zero_pad)
    with pytest.raises(AssertionError):
        test_shift_equivariance("gelu")


def test_stored_networks_load_without_pickles():
    """The networks the benchmark loads (paper_2510_07672_amd/weights, made
    by bench.py --save-weights): plain arrays and a JSON record, readable
    with allow_pickle=False, shaped 1 -> C -> ... -> C -> 1 with 3 x 3
    kernels, finite, and carrying the command that trained them."""
    import glob
    import json
    import os
    root = os.path.join(os.path.dirname(__file__), "..", "paper_2510_07672_amd", "weights")
    files = sorted(glob.glob(os.path.join(root, "*.npz")))
    assert files
    for path in files:
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            L, C = meta["cnn"]
            assert meta["command"].startswith("python bench.py ") and "--save-weights" in meta["command"]
            assert meta["training"]["steps"] > 0
            for l in range(L):
                cin = 1 if l == 0 else C
                cout = 1 if l == L - 1 else C
                w, b = z[f"w{l}"], z[f"b{l}"]
                assert w.shape == (cout, cin, 3, 3) and b.shape == (cout,)
                assert w.dtype == np.float32 and np.isfinite(w).all() and np.isfinite(b).all()
