"""GPU checks of the hidden-layer output tiles of the bfloat16 network
(Section 3.2's convolutional coarse propagator): 8 x 32 and 16 x 16 tiles
stage different halos but give each output the same products in the same
order, so every result must agree bit for bit, and stay within the bf16
tolerances of the oracle's emulated networks (2e-3 for bf16, 2e-4 for the
hi + lo split; derived in test_gpu_cnn.py).  Through the C ABI."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cnn  # noqa: E402
from paper_2510_07672_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2510_07672_amd import api as A
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def make(api, spec, seed, prec, scale=1.0):
    ws, bs = cnn.init_weights(spec, seed=seed, scale=scale)
    g = api.CnnCoarse(ws, bs, act=spec.act, residual=spec.residual, mass_fix=spec.mass_fix,
                      limiter=spec.limiter, prec=prec)
    return ws, bs, g


def problem(api, n):
    return api.Problem(n=n, length=1.0, eps=0.01, conservative=False, stab=2.0, dt=2e-5, steps=10)


def net_rel(out, ref, u):
    a, b = out - u, ref - u
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def under_tiles(api, plan, fn):
    """fn() under the 8 x 32 and the 16 x 16 tile (plan fixed), settings
    restored afterwards."""
    out = {}
    try:
        api.pr_set_coarse_plan(plan)
        for tile in ("8x32", "16x16"):
            api.pr_set_coarse_tile(tile)
            out[tile] = fn()
    finally:
        api.pr_set_coarse_tile("auto")
        api.pr_set_coarse_plan("auto")
    return out["8x32"], out["16x16"]


# n = 32 has one 8 x 32 tile per row band and 2 x 2 tiles of 16 x 16; the
# larger grids span many tiles of each shape.  L = 3 folds the first and the
# last convolution into the one hidden layer's launch.
@pytest.mark.parametrize("L,C,prec,n,nf,plan,act", [
    (6, 48, "bf16x2", 64, 3, "folded", "gelu"),
    (6, 48, "bf16", 32, 2, "layered", "gelu"),
    (3, 48, "bf16x2", 128, 1, "folded", "tanh"),
    (4, 32, "bf16x2", 128, 2, "folded", "gelu"),
    (4, 32, "bf16", 64, 1, "layered", "tanh"),
    (3, 32, "bf16", 32, 3, "folded", "gelu"),
    (5, 32, "bf16x2", 256, 1, "layered", "gelu"),
])
def test_tiles_are_bitwise_equal(api, L, C, prec, n, nf, plan, act):
    print(f"case tiles L={L} C={C} {prec} n={n} fields={nf} plan={plan} {act}", flush=True)
    spec = cnn.CnnSpec(n_layers=L, channels=C, act=act)
    ws, bs, g = make(api, spec, seed=11 * L + C, prec=prec)
    u0 = synth.random_ic(n, range(60, 60 + nf))
    p = problem(api, n)
    u = dev(u0)
    a, b = under_tiles(api, plan, lambda: api.pr_coarse_apply(p, g, u))
    assert torch.equal(a, b)
    emu = cnn.forward(u0, ws, bs, spec, prec=prec)
    assert net_rel(b.cpu().numpy(), emu, u0) <= (2e-3 if prec == "bf16" else 2e-4)


def test_tiles_in_training_and_parareal(api):
    """The training forward (every activation kept for the backward pass)
    and the Parareal driver run the same hidden-layer kernels: gradients and
    the solution must not change by a bit with the tile."""
    print("case tiles in pr_cnn_backward and pr_solve, 4 x 32 bf16x2, 64^2", flush=True)
    n = 64
    spec = cnn.CnnSpec(n_layers=4, channels=32)
    _, _, g = make(api, spec, seed=5, prec="bf16x2", scale=0.1)
    u0 = synth.random_ic(n, [70, 71])
    r = synth.random_ic(n, [72, 73])
    p = problem(api, n)
    a, b = under_tiles(api, "layered", lambda: api.pr_cnn_backward(p, g, dev(u0), dev(r)))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    ps = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=10)
    U0 = dev(synth.random_ic(n, [74, 75, 76]))
    run = lambda: api.pr_solve(ps, g, U0, 6, tol=0.0, max_iter=3, allow_not_converged=True)  # noqa: E731
    (Ua, sa), (Ub, sb) = under_tiles(api, "folded", run)
    assert torch.equal(Ua, Ub)
    assert np.array_equal(sa.history, sb.history)


def test_autotune_records_a_tile(api):
    """pr_autotune_coarse times both tiles at 32 and 48 channels and keeps
    the faster as the AUTO choice for (channels, prec, N); the result is the
    same bits whatever it picked.  Other widths take 8 x 32."""
    print("case autotune tiles, 6 x 48 bf16x2, 64^2", flush=True)
    n = 64
    spec = cnn.CnnSpec(n_layers=6, channels=48)
    _, _, g = make(api, spec, seed=9, prec="bf16x2")
    u0 = dev(synth.random_ic(n, [80, 81]))
    p = problem(api, n)
    api.pr_set_coarse_tile("8x32")
    api.pr_set_coarse_plan("layered")
    try:
        ref = api.pr_coarse_apply(p, g, u0)
    finally:
        api.pr_set_coarse_tile("auto")
        api.pr_set_coarse_plan("auto")
    plan = api.pr_autotune_coarse(p, g, u0)
    tile = api.pr_get_coarse_tile(g, n)
    assert plan in ("layered", "folded") and tile in ("8x32", "16x16")
    assert api.pr_get_coarse_plan(g, n) == plan
    assert torch.equal(api.pr_coarse_apply(p, g, u0), ref)
    # the setting overrides the tuned choice; widths built with one tile report it
    try:
        api.pr_set_coarse_tile("16x16" if tile == "8x32" else "8x32")
        assert api.pr_get_coarse_tile(g, n) != tile
    finally:
        api.pr_set_coarse_tile("auto")
    assert api.pr_get_coarse_tile(g, n) == tile
    _, _, g16 = make(api, cnn.CnnSpec(n_layers=4, channels=16), seed=1, prec="bf16x2")
    api.pr_autotune_coarse(p, g16, u0)
    assert api.pr_get_coarse_tile(g16, n) == "8x32"
