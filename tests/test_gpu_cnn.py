"""GPU parity of the convolutional coarse propagator (Section 3.2) against
the FP64 oracle, through the C ABI.

Tolerances (relative L2 of the network part net = G(u) - u):
  * FP32 path: 1e-5 (FP32 sums of 9 C terms per layer).
  * bf16 path against the oracle's "bf16" network (hidden weights and
    every activation rounded to bfloat16): 2e-3 -- the two differ only in
    FP32 vs FP64 summation and in the rare bfloat16 rounding decisions that
    sit within one FP32 rounding of a tie (each such flip moves one
    activation by one bfloat16 ulp, 2^-8 relative).
  * bf16 path against the exact network: 1e-2 (8-bit activations).
  * hi+lo bf16 path against the oracle's "bf16x2" network (bfloat16 hidden
    weights, activations unrounded): 2e-4.
  * hi+lo bf16 path against the exact network: 5e-3 -- what is left is
    the rounding of the hidden weights (measured on the oracle: <= 2.9e-3
    over the shapes tested here).  With hidden weights that are bfloat16
    numbers, i.e. the network the split kernels compute exactly up to
    their activation pairs: 5e-5 -- a hi + lo pair keeps 16 significant
    bits or more (relative error <= 2^-17 ~ 7.6e-6 per activation), and
    the last layer's weights are hi + lo pairs too; the oracle's split
    emulation of that network measures <= 7e-6.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import allen_cahn as ac  # noqa: E402
from oracle import cnn  # noqa: E402
from paper_2510_07672_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2510_07672_amd import api as A
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def net_rel(out, ref, u):
    a, b = out - u, ref - u
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(api, spec, seed, prec, scale=1.0):
    ws, bs = cnn.init_weights(spec, seed=seed, scale=scale)
    g = api.CnnCoarse(ws, bs, act=spec.act, residual=spec.residual, mass_fix=spec.mass_fix,
                      limiter=spec.limiter, prec=prec)
    return ws, bs, g


def problem(api, n):
    return api.Problem(n=n, length=1.0, eps=0.01, conservative=False, stab=2.0, dt=2e-5, steps=10)


@pytest.mark.parametrize("L,C", [(2, 8), (4, 32), (3, 48), (3, 16), (4, 64)])
def test_cnn_f32_matches_oracle(api, L, C):
    print(f"case cnn f32 L={L} C={C}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C)
    ws, bs, g = make(api, spec, seed=L * 100 + C, prec="f32")
    n = 64
    u0 = synth.random_ic(n, [1, 2, 3])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    ref = cnn.forward(u0, ws, bs, spec)
    assert net_rel(out, ref, u0) <= 1e-5


@pytest.mark.parametrize("L,C,n", [(2, 8, 32), (4, 32, 64), (3, 16, 64), (5, 8, 128)])
def test_cnn_f64_matches_oracle(api, L, C, n):
    print(f"case cnn f64 L={L} C={C} n={n}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C)
    ws, bs, g = make(api, spec, seed=L * 10 + C, prec="f64")
    u0 = synth.random_ic(n, [1, 2])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    ref = cnn.forward(u0, ws, bs, spec)
    assert net_rel(out, ref, u0) <= 1e-12


@pytest.mark.parametrize("L,C,n", [(4, 32, 64), (4, 32, 256), (6, 48, 128), (3, 16, 32), (3, 64, 64)])
def test_cnn_bf16_matches_oracle(api, L, C, n):
    print(f"case cnn bf16 L={L} C={C} n={n}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C)
    ws, bs, g = make(api, spec, seed=7 + C, prec="bf16")
    u0 = synth.random_ic(n, [4, 5])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    emu = cnn.forward(u0, ws, bs, spec, prec="bf16")
    exact = cnn.forward(u0, ws, bs, spec)
    e_emu, e_exact = net_rel(out, emu, u0), net_rel(out, exact, u0)
    print(f"bf16 vs bf16 oracle {e_emu:.2e}, vs exact {e_exact:.2e}", flush=True)
    assert e_emu <= 2e-3
    assert e_exact <= 1e-2


@pytest.mark.parametrize("L,C", [(4, 32), (4, 48), (3, 16), (3, 32), (6, 48)])
def test_cnn_bf16x2_matches_oracle(api, L, C):
    print(f"case cnn bf16x2 L={L} C={C}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C)
    ws, bs, g = make(api, spec, seed=11, prec="bf16x2")
    n = 64
    u0 = synth.random_ic(n, [6, 7])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    ref = cnn.forward(u0, ws, bs, spec, prec="bf16x2")
    e_emu, e_exact = net_rel(out, ref, u0), net_rel(out, cnn.forward(u0, ws, bs, spec), u0)
    print(f"bf16x2 vs split oracle {e_emu:.2e}, vs exact {e_exact:.2e}", flush=True)
    assert e_emu <= 2e-4
    assert e_exact <= 5e-3


def bf16_hidden(ws):
    """The same weights with those of the hidden layers made bfloat16 numbers."""
    return [w if l in (0, len(ws) - 1) else cnn.bf16(w) for l, w in enumerate(ws)]


@pytest.mark.parametrize("L,C,n", [(4, 32, 64), (4, 48, 64), (3, 16, 32), (6, 48, 128),
                                   (3, 32, 256)])
def test_cnn_bf16x2_with_bf16_weights_matches_exact_oracle(api, L, C, n):
    """With bfloat16 hidden weights the split network is the exact network up
    to its activation pairs: compared with the oracle's exact FP64 network."""
    print(f"case cnn bf16x2 bf16-weights L={L} C={C} n={n}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C)
    ws, bs = cnn.init_weights(spec, seed=17 + C)
    ws = bf16_hidden(ws)
    g = api.CnnCoarse(ws, bs, prec="bf16x2")
    u0 = synth.random_ic(n, [8, 9])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    e = net_rel(out, cnn.forward(u0, ws, bs, spec), u0)
    print(f"bf16x2 with bf16 hidden weights vs exact {e:.2e}", flush=True)
    assert e <= 5e-5


@pytest.mark.parametrize("prec", ["bf16", "bf16x2"])
def test_cnn_config3_shape_matches_exact_oracle(api, prec):
    """The 6 x 48 network on its whole 16-field batch of 512^2, in the plan the
    benchmark runs (untuned default: folded for split networks), checked on
    two sampled fields.

    Split form against the exact FP64 network: net-relative <= 5e-3 (the
    rounding of the hidden weights; 2.2e-3 on the oracle's split network)
    and, with bfloat16 hidden weights, <= 5e-5.  Plain bf16: against the
    oracle's bf16 network net-relative <= 5e-3, and against the exact
    network G-relative (|G_bf16(u) - G(u)| / |G(u)|) <= 1e-2.  The
    net-relative distance of the bf16 format itself from the exact network
    is 1.3e-2 for these weights (the oracle's bf16 network measures it):
    the seed-0 network's output is a small difference of O(1) activations
    (RMS 1.2e-4 per point), which 8-bit activations resolve only to ~1%.
    The same cancellation amplifies the bfloat16 rounding decisions that
    FP32 and FP64 sums take differently: the same bf16 network evaluated
    on the CPU with FP32 sums differs from the oracle's by 2.2e-3 on
    field 0, as the GPU does (2.3e-3); hence 5e-3 here, where the 4-layer
    networks above stay under 2e-3."""
    print(f"case cnn config-3 shape 6x48 512^2 x 16 {prec}", flush=True)
    n, B = 512, 16
    spec = cnn.CnnSpec(n_layers=6, channels=48)
    ws, bs = cnn.init_weights(spec, seed=0, scale=0.1)
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=1e-5, steps=100)
    u0 = synth.random_ic(n, range(B))
    samples = [0, 15]
    cases = ((ws, 5e-3), (bf16_hidden(ws), 5e-5)) if prec == "bf16x2" else ((ws, None),)
    for weights, tol in cases:
        g = api.CnnCoarse(weights, bs, prec=prec)
        if prec == "bf16x2":
            assert api.pr_get_coarse_plan(g, n) == "folded"
        out = api.pr_coarse_apply(p, g, dev(u0)).cpu().numpy()
        ref = cnn.forward(u0[samples], weights, bs, spec)
        emu = cnn.forward(u0[samples], weights, bs, spec, prec=prec) if prec == "bf16" else None
        for k, i in enumerate(samples):
            e = net_rel(out[i], ref[k], u0[i])
            if prec == "bf16x2":
                print(f"field {i}: bf16x2 vs exact {e:.2e} (bound {tol:g})", flush=True)
                assert e <= tol
            else:
                e_emu = net_rel(out[i], emu[k], u0[i])
                e_g = float(np.linalg.norm(out[i] - ref[k]) / np.linalg.norm(ref[k]))
                print(f"field {i}: bf16 vs bf16 oracle {e_emu:.2e}, vs exact {e:.2e} net / "
                      f"{e_g:.2e} G", flush=True)
                assert e_emu <= 5e-3
                assert e_g <= 1e-2


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_cnn_shift_equivariant_bitwise(api, prec):
    spec = cnn.CnnSpec(n_layers=4, channels=32)
    ws, bs, g = make(api, spec, seed=3, prec=prec)
    n = 64
    u0 = synth.random_ic(n, [8])
    p = problem(api, n)
    a = api.pr_coarse_apply(p, g, dev(np.roll(u0, (5, -9), axis=(1, 2)))).cpu().numpy()
    b = np.roll(api.pr_coarse_apply(p, g, dev(u0)).cpu().numpy(), (5, -9), axis=(1, 2))
    assert np.array_equal(a, b)


def test_cnn_mass_fix_limiter_tanh(api):
    spec = cnn.CnnSpec(n_layers=4, channels=32, act="tanh", mass_fix=True, limiter=(-0.95, 0.95))
    ws, bs, g = make(api, spec, seed=5, prec="f32")
    n = 64
    u0 = synth.random_ic(n, [9, 10])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    ref = cnn.forward(u0, ws, bs, spec)
    assert np.abs(out - ref).max() <= 1e-5
    assert out.min() >= -0.95 and out.max() <= 0.95
    spec2 = cnn.CnnSpec(n_layers=4, channels=32, mass_fix=True)
    _, _, g2 = make(api, spec2, seed=5, prec="bf16")
    out2 = api.pr_coarse_apply(problem(api, n), g2, dev(u0)).cpu().numpy()
    assert np.abs(out2.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-14


def test_cnn_zero_output_layer_is_identity(api):
    spec = cnn.CnnSpec(n_layers=4, channels=32)
    ws, bs, g = make(api, spec, seed=1, prec="bf16", scale=0.0)
    n = 64
    u0 = synth.random_ic(n, [3])
    out = api.pr_coarse_apply(problem(api, n), g, dev(u0)).cpu().numpy()
    assert np.array_equal(out, u0)


def test_parareal_with_cnn_coarse(api):
    # the exactness of Section 3.3 does not depend on G: k = s is the serial
    # fine solve bit for bit, and the first iterate with an FP32 network
    # follows the oracle run with the FP64 network
    n, s = 64, 5
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=20)
    spec = cnn.CnnSpec(n_layers=4, channels=16)
    ws, bs, g = make(api, spec, seed=2, prec="f32", scale=0.1)
    u0 = synth.random_ic(n, [12, 13])
    U, st = api.pr_solve(p, g, dev(u0), s, tol=0.0)
    assert torch.equal(U, api.pr_serial_fine(p, dev(u0), s))
    U1, _ = api.pr_solve(p, g, dev(u0), s, tol=0.0, max_iter=1, allow_not_converged=True)
    po = ac.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=20)
    ref = ac.parareal(u0, po, s, tol=0.0, max_iter=1, G=lambda v: cnn.forward(v, ws, bs, spec))
    assert float(np.linalg.norm(U1.cpu().numpy() - ref.U) / np.linalg.norm(ref.U)) <= 1e-6
    _, _, gb = make(api, spec, seed=2, prec="bf16", scale=0.1)
    Ub, _ = api.pr_solve(p, gb, dev(u0), s, tol=0.0)
    assert torch.equal(Ub, U)


@pytest.mark.parametrize("L,C,prec,n", [(4, 32, "bf16", 64), (4, 32, "bf16x2", 256),
                                        (3, 16, "bf16", 32), (6, 16, "bf16x2", 64),
                                        (3, 48, "bf16", 128), (3, 32, "bf16x2", 64)])
def test_fused_plan_matches_layered_and_oracle(api, L, C, prec, n):
    print(f"case fused L={L} C={C} {prec} n={n}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C)
    ws, bs, g = make(api, spec, seed=5 * L + C, prec=prec)
    u0 = synth.random_ic(n, [21, 22, 23])
    p = problem(api, n)
    try:
        api.pr_set_coarse_plan("fused")
        assert api.pr_get_coarse_plan(g, n) == "fused"
        fused = api.pr_coarse_apply(p, g, dev(u0)).cpu().numpy()
        api.pr_set_coarse_plan("layered")
        assert api.pr_get_coarse_plan(g, n) == "layered"
        layered = api.pr_coarse_apply(p, g, dev(u0)).cpu().numpy()
    finally:
        api.pr_set_coarse_plan("auto")
    assert net_rel(fused, layered, u0) <= 1e-6
    emu = cnn.forward(u0, ws, bs, spec, prec=prec)
    assert net_rel(fused, emu, u0) <= (2e-3 if prec == "bf16" else 2e-4)
    assert net_rel(fused, cnn.forward(u0, ws, bs, spec), u0) <= (1e-2 if prec == "bf16" else 5e-3)


@pytest.mark.parametrize("L,C,prec,n,nf,act,mass", [(4, 32, "bf16x2", 256, 3, "gelu", False),
                                                    (4, 32, "bf16", 32, 1, "gelu", False),
                                                    (3, 32, "bf16x2", 64, 3, "gelu", True),
                                                    (3, 32, "bf16", 32, 2, "tanh", False),
                                                    (5, 32, "bf16x2", 128, 2, "gelu", True),
                                                    (3, 16, "bf16x2", 64, 5, "tanh", False),
                                                    (6, 48, "bf16x2", 64, 2, "gelu", False),
                                                    (3, 64, "bf16", 128, 2, "gelu", False)])
def test_folded_plan_is_bitwise_layered(api, L, C, prec, n, nf, act, mass):
    """The first convolution computed inside the first hidden layer's launch,
    and at 32 channels the last one's per-tap products in the last hidden
    layer's epilogue, give the layer-by-layer result bit for bit, within the
    bf16 tolerances of the oracle.  L = 3 at 32 channels folds both into
    the one hidden layer; the mass fix reads the gather's tile sums."""
    print(f"case folded L={L} C={C} {prec} n={n} fields={nf} {act} mass_fix={mass}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C, act=act, mass_fix=mass)
    ws, bs, g = make(api, spec, seed=7 * L + C, prec=prec)
    u0 = synth.random_ic(n, range(40, 40 + nf))
    p = problem(api, n)
    try:
        api.pr_set_coarse_plan("folded")
        assert api.pr_get_coarse_plan(g, n) == "folded"
        folded = api.pr_coarse_apply(p, g, dev(u0))
        api.pr_set_coarse_plan("layered")
        layered = api.pr_coarse_apply(p, g, dev(u0))
    finally:
        api.pr_set_coarse_plan("auto")
    assert torch.equal(folded, layered)
    if mass:
        f = folded.cpu().numpy()
        assert np.abs(f.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-14
    emu = cnn.forward(u0, ws, bs, spec, prec=prec)
    assert net_rel(folded.cpu().numpy(), emu, u0) <= (2e-3 if prec == "bf16" else 2e-4)
    assert net_rel(folded.cpu().numpy(), cnn.forward(u0, ws, bs, spec), u0) <= \
        (1e-2 if prec == "bf16" else 5e-3)


@pytest.mark.parametrize("conservative,f32_iters,mass_fix", [(False, 0, False), (True, 1, False),
                                                          (False, 0, True)])
def test_folded_plan_in_parareal_is_bitwise_layered(api, conservative, f32_iters, mass_fix):
    """Through pr_solve the network reads its fields from the window by
    offset tables, and under the folded plan its last kernel also applies the
    Parareal correction (FP32 fine values in the first iteration with
    f32_iters = 1); with a mass fix the correction runs after the fix.  The
    solution and the per-iteration update norms must not change by a bit."""
    print(f"case folded plan in pr_solve, 4 x 32 bf16x2, 64^2, conservative={conservative} "
          f"f32_iters={f32_iters} mass_fix={mass_fix}", flush=True)
    n, s = 64, 6
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=conservative, stab=2.0, dt=1e-4,
                    steps=10, f32_iters=f32_iters)
    spec = cnn.CnnSpec(n_layers=4, channels=32, mass_fix=mass_fix)
    _, _, g = make(api, spec, seed=3, prec="bf16x2", scale=0.1)
    u0 = dev(synth.random_ic(n, [50, 51, 52]))
    try:
        api.pr_set_coarse_plan("folded")
        Uh, sth = api.pr_solve(p, g, u0, s, tol=0.0, max_iter=3, allow_not_converged=True)
        api.pr_set_coarse_plan("layered")
        Ul, stl = api.pr_solve(p, g, u0, s, tol=0.0, max_iter=3, allow_not_converged=True)
    finally:
        api.pr_set_coarse_plan("auto")
    assert torch.equal(Uh, Ul)
    assert sth.iterations == stl.iterations
    assert np.array_equal(sth.history, stl.history)
    # the last iteration's update is that of the solution against the previous one
    Up, _ = api.pr_solve(p, g, u0, s, tol=0.0, max_iter=2, allow_not_converged=True)
    d = (Uh - Up).abs().amax(dim=(1, 2, 3)).cpu().numpy()
    assert np.array_equal(sth.history[-1], d)


def test_fused_plan_mass_fix_limiter_and_autotune(api):
    spec = cnn.CnnSpec(n_layers=4, channels=32, mass_fix=True, limiter=(-0.95, 0.95))
    ws, bs, g = make(api, spec, seed=31, prec="bf16x2")
    n = 64
    u0 = synth.random_ic(n, [24, 25])
    p = problem(api, n)
    out = api.pr_coarse_apply(p, g, dev(u0)).cpu().numpy()
    assert np.abs(out.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-14 or out.min() <= -0.95 \
        or out.max() >= 0.95
    assert out.min() >= -0.95 and out.max() <= 0.95
    spec_nf = cnn.CnnSpec(n_layers=4, channels=32, mass_fix=True)
    _, _, g2 = make(api, spec_nf, seed=31, prec="bf16x2")
    o2 = api.pr_coarse_apply(p, g2, dev(u0)).cpu().numpy()
    assert np.abs(o2.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-14
    choice = api.pr_autotune_coarse(p, g2, dev(u0))
    assert choice in ("fused", "layered", "folded")
    assert api.pr_get_coarse_plan(g2, n) == choice
    # shapes without a fused kernel fall back to layered; untuned, a network
    # with a hidden layer that is split or 32 channels wide takes the folded
    # plan, another unsplit one or one without a hidden layer takes layered
    _, _, g64 = make(api, cnn.CnnSpec(n_layers=4, channels=64), seed=1, prec="bf16")
    _, _, g2l = make(api, cnn.CnnSpec(n_layers=2, channels=32), seed=1, prec="bf16x2")
    _, _, g5 = make(api, cnn.CnnSpec(n_layers=5, channels=16), seed=1, prec="bf16x2")
    try:
        api.pr_set_coarse_plan("fused")
        assert api.pr_get_coarse_plan(g64, n) == "layered"
        api.pr_set_coarse_plan("folded")
        assert api.pr_get_coarse_plan(g64, n) == "folded"
        assert api.pr_get_coarse_plan(g2l, n) == "layered"
    finally:
        api.pr_set_coarse_plan("auto")
    assert api.pr_get_coarse_plan(g64, n) == "layered"
    assert api.pr_get_coarse_plan(g2l, n) == "layered"
    assert api.pr_get_coarse_plan(g5, n) == "folded"
    _, _, g32 = make(api, cnn.CnnSpec(n_layers=5, channels=32), seed=1, prec="bf16")
    assert api.pr_get_coarse_plan(g32, n) == "folded"
