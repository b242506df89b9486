"""Pins of the oracle's Crank-Nicolson + Picard fine scheme (Section 3.1,
eq. fully-discrete) and of the Fourier collocation Laplacian.

Each pin is fixed by the mathematics, not by re-running the oracle's own
arithmetic:
  * converged Picard iterates satisfy the scheme pointwise (residual with
    no solve);
  * the Picard map contracts at rate <= dt max|f'| (classic) / 2 dt max|f'|
    (conservative) in L2;
  * a small Fourier mode is amplified by the closed-form CN factor
    (1 + h(1 - eps^2 mu)) / (1 - h(1 - eps^2 mu)), h = dt/2;
  * the conservative scheme keeps the mass for any number of iterations;
  * 0 and +-1 are fixed points of the classic scheme;
  * the time error is second order (first order for the semi-implicit
    step), by Richardson ratios;
  * the collocation Laplacian of a trigonometric mode is exact.
"""

import math

import numpy as np
import pytest

from oracle import allen_cahn as ac
from paper_2510_07672_amd import synth


def prob(n=32, eps=0.05, cons=False, dt=1e-3, lap="fd", picard=3, steps=1, length=1.0):
    return ac.Problem(n=n, length=length, eps=eps, conservative=cons, stab=0.0, dt=dt,
                      steps=steps, scheme="cn", picard=picard, laplacian=lap)


@pytest.mark.parametrize("cons", [False, True])
@pytest.mark.parametrize("lap", ["fd", "spectral"])
def test_converged_picard_solves_the_scheme(cons, lap):
    p = prob(cons=cons, lap=lap)
    u = synth.random_ic(32, [3, 4])
    v = ac.cn_picard_step(u, p, p.dt, iters=12)
    assert np.abs(ac.cn_residual(u, v, p, p.dt)).max() <= 2e-13


@pytest.mark.parametrize("cons", [False, True])
def test_picard_contraction_rate(cons):
    p = prob(cons=cons, dt=2e-2, eps=0.02)
    u = synth.random_ic(32, [5])
    trace = []
    ac.cn_picard_step(u, p, p.dt, iters=6, trace=trace)
    d = [np.linalg.norm(trace[m + 1] - trace[m]) for m in range(len(trace) - 1)]
    bound = (2.0 if cons else 1.0) * p.dt * 2.0   # max |f'| = 2 on [-1, 1]
    for m in range(1, len(d)):
        if d[m - 1] > 1e-13:
            assert d[m] <= 1.05 * bound * d[m - 1]
    assert d[-1] < 1e-6 * d[0]


@pytest.mark.parametrize("cons", [False, True])
@pytest.mark.parametrize("lap", ["fd", "spectral"])
def test_small_mode_cn_factor(cons, lap):
    n, kx, ky, a = 32, 3, 5, 1e-6
    p = prob(n=n, cons=cons, lap=lap, dt=4e-3, eps=0.03)
    u = synth.single_mode(n, kx, ky, a)[None]
    v = ac.cn_picard_step(u, p, p.dt, iters=20)
    h = p.length / n
    if lap == "fd":
        mu = 4 / h ** 2 * (math.sin(math.pi * kx / n) ** 2 + math.sin(math.pi * ky / n) ** 2)
    else:
        mu = (2 * math.pi / p.length) ** 2 * (kx ** 2 + ky ** 2)
    hh = p.dt / 2
    lin = 1 - p.eps ** 2 * mu
    phi = (1 + hh * lin) / (1 - hh * lin)
    assert np.abs(v - phi * u).max() <= 1e-9 * a


@pytest.mark.parametrize("iters", [1, 2, 5])
@pytest.mark.parametrize("lap", ["fd", "spectral"])
def test_conservative_mass_any_iteration_count(iters, lap):
    p = prob(cons=True, lap=lap, dt=5e-3)
    u = synth.random_ic(32, [6, 7])
    v = u
    for _ in range(10):
        v = ac.cn_picard_step(v, p, p.dt, iters=iters)
    assert np.abs(v.mean(axis=(1, 2)) - u.mean(axis=(1, 2))).max() <= 1e-13
    pc = prob(cons=False, lap=lap, dt=5e-3)
    w = ac.cn_picard_step(u, pc, pc.dt, iters=iters)
    assert np.abs(w.mean(axis=(1, 2)) - u.mean(axis=(1, 2))).max() > 1e-8


def test_fixed_points():
    p = prob(dt=1e-2)
    z = np.zeros((1, 32, 32))
    assert np.array_equal(ac.cn_picard_step(z, p, p.dt), z)
    for c in (1.0, -1.0):
        u = np.full((1, 32, 32), c)
        assert np.abs(ac.cn_picard_step(u, p, p.dt, iters=5) - u).max() <= 4e-16


def _richardson(scheme, T=0.08, n=32, eps=0.1):
    x = np.arange(n) / n
    u0 = (0.5 * np.sin(2 * np.pi * x)[:, None] * np.sin(2 * np.pi * x)[None, :])[None]
    out = []
    for m in (10, 20, 40):
        dt = T / m
        p = ac.Problem(n=n, length=1.0, eps=eps, conservative=False, stab=0.0, dt=dt, steps=m,
                       scheme=scheme, picard=30)
        out.append(ac.fine(u0, p))
    e1 = np.abs(out[0] - out[1]).max()
    e2 = np.abs(out[1] - out[2]).max()
    return e1 / e2


def test_cn_is_second_order_ssi_first():
    assert 3.6 <= _richardson("cn") <= 4.4
    assert 1.8 <= _richardson("ssi") <= 2.2


def test_collocation_laplacian_of_a_mode():
    n, L = 32, 1.7
    x = np.arange(n) * L / n
    u = np.sin(2 * np.pi * (3 * x[:, None] + 5 * x[None, :]) / L)
    lap = ac.laplacian_spectral(u, L)
    assert np.abs(lap + (2 * np.pi / L) ** 2 * 34 * u).max() <= 1e-10 * (2 * np.pi / L) ** 2 * 34
    # the solver's symbol is that Laplacian's: irfft2(-mu rfft2 u) = Lap u for any u
    r = synth.random_ic(n, [9])[0]
    mu = ac.symbol_mu(n, L / n, "spectral")
    via_symbol = np.fft.irfft2(-mu * np.fft.rfft2(r), s=(n, n))
    assert np.abs(via_symbol - ac.laplacian_spectral(r, L)).max() <= 1e-9


def test_pins_catch_half_weight_nonlocal_term(monkeypatch):
    orig = ac.cn_nonlocal
    monkeypatch.setattr(ac, "cn_nonlocal", lambda fn, fv, c: 0.5 * orig(fn, fv, c))
    with pytest.raises(AssertionError):
        test_conservative_mass_any_iteration_count(2, "fd")


def test_pins_catch_dropped_explicit_laplacian(monkeypatch):
    real = ac.apply_laplacian
    calls = {"n": 0}

    def lap_first_zero(u, p):
        # the explicit eps^2 Lap U_n term is the first Laplacian evaluated
        calls["n"] += 1
        return 0 * u if calls["n"] == 1 else real(u, p)
    monkeypatch.setattr(ac, "apply_laplacian", lap_first_zero)
    with pytest.raises(AssertionError):
        test_small_mode_cn_factor(False, "fd")


def test_pins_catch_sign_of_f(monkeypatch):
    monkeypatch.setattr(ac, "f_double_well", lambda u: -(u - u ** 3))
    with pytest.raises(AssertionError):
        test_small_mode_cn_factor(False, "fd")


@pytest.mark.parametrize("cons", [False, True])
def test_scheme_loss_gradient_by_finite_differences(cons):
    """The scheme-residual loss of eq. loss_ACN and its gradient in U_{n+1}:
    central differences of the loss in every point of a tiny pair, and the
    loss vanishing on a converged Crank-Nicolson step."""
    n, dt = 8, 4e-3
    po = prob(n=n, cons=cons, dt=dt, eps=0.05)
    u = synth.random_ic(n, [21, 22])
    w = synth.random_ic(n, [23, 24])
    loss, grad = ac.cn_residual_loss(u, w, po, dt)
    assert abs(loss - float((ac.cn_residual(u, w, po, dt) ** 2).mean())) <= 1e-15 * loss
    h = 1e-6
    fd = np.zeros_like(w)
    for idx in np.ndindex(*w.shape):
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        fd[idx] = (ac.cn_residual_loss(u, wp, po, dt)[0] - ac.cn_residual_loss(u, wm, po, dt)[0]) / (2 * h)
    assert np.abs(fd - grad).max() <= 1e-7 * np.abs(grad).max()
    v = ac.cn_picard_step(u, po, dt, iters=30)
    l0, g0 = ac.cn_residual_loss(u, v, po, dt)
    assert l0 <= 1e-26 and np.abs(g0).max() <= 1e-13


def test_scheme_loss_pins_catch_a_dropped_mean_term(monkeypatch):
    orig = ac.cn_residual_loss

    def no_mean(u, v, p, dt):
        import dataclasses
        return orig(u, v, dataclasses.replace(p, conservative=False), dt)
    monkeypatch.setattr(ac, "cn_residual_loss", no_mean)
    with pytest.raises(AssertionError):
        test_scheme_loss_gradient_by_finite_differences(True)


def test_scheme_loss_pins_catch_a_gradient_without_its_mean_term(monkeypatch):
    orig = ac.cn_residual_loss

    def grad_without_mean(u, v, p, dt):
        loss, g = orig(u, v, p, dt)
        r = ac.cn_residual(u, v, p, dt)
        fp = 1.0 - 3.0 * v * v
        return loss, g - (2.0 / r.size) * 0.5 * dt * fp * r.mean(axis=(-2, -1), keepdims=True)
    monkeypatch.setattr(ac, "cn_residual_loss", grad_without_mean)
    with pytest.raises(AssertionError):
        test_scheme_loss_gradient_by_finite_differences(True)
