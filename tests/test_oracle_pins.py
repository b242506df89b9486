"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with an
independent route (a dense linear solve, a shift-only stencil, a closed
form, an invariant the scheme provably keeps, or the exactness statement
of Parareal in Section 3.3).
"""

import math

import numpy as np
import pytest

from oracle import allen_cahn as ac
from paper_2510_07672_amd import synth


def _dense_laplacian(n, h):
    """Periodic 5-point Laplacian as an explicit n^2 x n^2 matrix."""
    I = np.eye(n)
    D = -2.0 * I + np.roll(I, 1, axis=1) + np.roll(I, -1, axis=1)
    return (np.kron(D, I) + np.kron(I, D)) / (h * h)


# ---------------------------------------------------------------------------
# the implicit solve (Section 3.1: one linear system per step)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("conservative", [False, True])
def test_step_solves_the_stencil_system(conservative):
    n, h, eps, S, dt = 64, 1.0 / 64, 0.02, 2.0, 1e-3
    u = synth.random_ic(n, [11])[0]
    a = 1.0 + S * dt
    up = ac.ssi_step(u, n, h, eps, S, dt, conservative)
    fu = u - u ** 3
    m = fu.mean() if conservative else 0.0
    rhs = a * u + dt * (fu - m)
    # residual of ((1+S dt) - dt eps^2 Lap_h) u+ = rhs with the shift stencil
    res = a * up - dt * eps * eps * ac.laplacian_stencil(up, h) - rhs
    assert np.abs(res).max() <= 1e-13 * np.abs(rhs).max()


@pytest.mark.parametrize("conservative", [False, True])
def test_step_matches_dense_solve_tiny(conservative):
    n, L, eps, S, dt = 8, 1.0, 0.1, 2.0, 0.05
    h = L / n
    u = synth.random_ic(n, [3])[0]
    a = 1.0 + S * dt
    A = a * np.eye(n * n) - dt * eps * eps * _dense_laplacian(n, h)
    fu = u - u ** 3
    m = fu.mean() if conservative else 0.0
    rhs = (a * u + dt * (fu - m)).ravel()
    ref = np.linalg.solve(A, rhs).reshape(n, n)
    got = ac.ssi_step(u, n, h, eps, S, dt, conservative)
    assert np.abs(got - ref).max() <= 1e-14


def test_symbol_is_the_stencil_eigenvalue():
    n, h = 16, 1.0 / 16
    mu = ac.symbol_mu(n, h)
    for (ky, kx) in [(0, 0), (1, 0), (3, 5), (8, 8), (15, 2)]:
        i = np.arange(n)[:, None]
        j = np.arange(n)[None, :]
        e = np.cos(2 * np.pi * (ky * i + kx * j) / n)
        lap = ac.laplacian_stencil(e, h)
        kxh = kx if kx <= n // 2 else n - kx
        assert np.allclose(lap, -mu[ky, kxh] * e, atol=1e-9 * max(1.0, mu.max()))


# ---------------------------------------------------------------------------
# special cases with closed forms
# ---------------------------------------------------------------------------

def test_constant_field_classic_scalar_map():
    n, h, eps, S, dt = 32, 1 / 32, 0.02, 2.0, 0.01
    for c in [-0.7, -0.2, 0.3, 0.9]:
        u = np.full((n, n), c)
        up = ac.ssi_step(u, n, h, eps, S, dt, False)
        expect = c + dt * (c - c ** 3) / (1 + S * dt)
        assert np.abs(up - expect).max() <= 4e-16


def test_constant_field_conservative_is_fixed():
    n, h, eps, S, dt = 32, 1 / 32, 0.02, 2.0, 0.01
    for c in [-0.7, 0.3, 0.9]:
        u = np.full((n, n), c)
        up = ac.ssi_step(u, n, h, eps, S, dt, True)
        assert np.abs(up - c).max() <= 4e-16


@pytest.mark.parametrize("conservative", [False, True])
def test_pure_phases_and_zero_are_fixed_points(conservative):
    p = ac.Problem(n=32, length=1.0, eps=0.02, conservative=conservative,
                   stab=2.0, dt=1e-3, steps=50)
    z = ac.fine(np.zeros((1, 32, 32)), p)
    assert np.array_equal(z, np.zeros_like(z))          # bitwise
    for c in (1.0, -1.0):
        v = ac.fine(np.full((1, 32, 32), c), p)
        assert np.abs(v - c).max() <= 2 * np.spacing(1.0)


@pytest.mark.parametrize("conservative", [False, True])
def test_small_fourier_mode_decays_by_linear_factor(conservative):
    # linearised about 0: u+ = (1+(S+1)dt)/(1+S dt+dt eps^2 mu_k) u
    n, L, eps, S, dt = 32, 1.0, 0.05, 2.0, 2e-3
    h = L / n
    for (kx, ky) in [(1, 0), (3, 5), (7, 2), (16, 16)]:
        a0 = 1e-6
        u = synth.single_mode(n, kx, ky, a0)[0]
        mu = (4 / h ** 2) * (math.sin(math.pi * kx / n) ** 2 + math.sin(math.pi * ky / n) ** 2)
        r = (1 + (S + 1) * dt) / (1 + S * dt + dt * eps * eps * mu)
        v = u.copy()
        steps = 20
        for _ in range(steps):
            v = ac.ssi_step(v, n, h, eps, S, dt, conservative)
        expect = (r ** steps) * u
        # O(a0^2) relative error from the cubic term, plus rounding
        assert np.abs(v - expect).max() <= 1e-9 * a0


# ---------------------------------------------------------------------------
# invariants of the discrete scheme (Section 2: MBP, energy, mass)
# ---------------------------------------------------------------------------

def test_discrete_mbp_classic_any_dt():
    n = 48
    u = synth.random_ic(n, [5], amp=1.0)[0]
    u[0, 0], u[1, 1] = 1.0, -1.0
    for dt in [1e-3, 0.1, 1.0, 5.0]:
        v = u.copy()
        for _ in range(30):
            v = ac.ssi_step(v, n, 1.0 / n, 0.02, 2.0, dt, False)
            assert np.abs(v).max() <= 1.0 + 1e-14


def test_discrete_mbp_conservative():
    n = 48
    beta = ac.mbp_bound(True)
    u = synth.random_ic(n, [6], amp=beta)[0]
    u[0, 0] = beta
    for dt in [1e-3, 0.1, 1.0]:       # needs 1 + (S - 3) dt >= 0
        v = u.copy()
        for _ in range(30):
            v = ac.ssi_step(v, n, 1.0 / n, 0.02, 2.0, dt, True)
            assert np.abs(v).max() <= beta + 1e-14


@pytest.mark.parametrize("conservative", [False, True])
def test_discrete_energy_decays(conservative):
    n, eps, S = 64, 0.03, 2.0
    h = 1.0 / n
    u = synth.random_ic(n, [7])[0]
    for dt in [1e-3, 0.05]:
        v = u.copy()
        e_prev = ac.discrete_energy(v, eps, h)
        for _ in range(40):
            v = ac.ssi_step(v, n, h, eps, S, dt, conservative)
            e = ac.discrete_energy(v, eps, h)
            assert e <= e_prev + 1e-13 * abs(e_prev)
            e_prev = e


def test_mass_conserved_to_1e13():
    p = ac.Problem(n=64, length=1.0, eps=0.02, conservative=True,
                   stab=2.0, dt=1e-3, steps=400)
    u0 = synth.random_ic(64, [1, 2])
    u = ac.fine(u0, p)
    assert np.abs(ac.mass(u) - ac.mass(u0)).max() <= 1e-13


def test_classic_does_not_conserve_mass():
    # guards against a conservative term leaking into the classic model
    p = ac.Problem(n=64, length=1.0, eps=0.02, conservative=False,
                   stab=2.0, dt=1e-3, steps=200)
    u0 = synth.random_ic(64, [1]) + 0.2
    u = ac.fine(u0, p)
    assert abs(ac.mass(u) - ac.mass(u0)).max() > 1e-3


# ---------------------------------------------------------------------------
# Parareal (Section 3.3, Algorithm 2)
# ---------------------------------------------------------------------------

def _small_problem(conservative=False):
    return ac.Problem(n=32, length=1.0, eps=0.04, conservative=conservative,
                      stab=2.0, dt=1e-3, steps=10)


@pytest.mark.parametrize("conservative", [False, True])
def test_parareal_k_equals_s_is_the_serial_fine_solve(conservative):
    p, s = _small_problem(conservative), 6
    u0 = synth.random_ic(32, [21, 22])
    ref = ac.serial_fine_trajectory(u0, p, s)
    res = ac.parareal(u0, p, s, tol=0.0)        # never converges early
    assert (res.iterations == s).all()
    assert np.array_equal(res.U, ref)           # bitwise


def test_parareal_first_k_slices_are_fine_after_k_iterations():
    p, s = _small_problem(), 6
    u0 = synth.random_ic(32, [23])
    ref = ac.serial_fine_trajectory(u0, p, s)
    for k in range(1, s + 1):
        res = ac.parareal(u0, p, s, tol=0.0, max_iter=k)
        assert np.array_equal(res.U[:, :k + 1], ref[:, :k + 1])
        if k < s:
            # slices beyond k are generally not yet fine
            assert not np.array_equal(res.U[:, k + 1:], ref[:, k + 1:])


def test_parareal_with_G_equal_F_converges_in_one_iteration():
    p, s = _small_problem(), 5
    u0 = synth.random_ic(32, [24])
    ref = ac.serial_fine_trajectory(u0, p, s)
    res = ac.parareal(u0, p, s, tol=1e-12, G=lambda v: ac.fine(v, p))
    # the initial coarse sweep already is the fine solve, so iteration 1
    # changes nothing beyond rounding and the run stops there
    assert res.iterations[0] == 1
    assert res.history[0][0] <= 1e-13
    assert np.abs(res.U - ref).max() <= 1e-13


def test_parareal_linear_mode_binomial_closed_form():
    # small single mode: U^k_{n+1} = g U^k_n + (phi - g) U^{k-1}_n, whose
    # solution is a0 * sum_{j<=min(k,n)} C(n,j) (phi-g)^j g^(n-j)
    n, L, eps, S = 32, 1.0, 0.05, 2.0
    p = ac.Problem(n=n, length=L, eps=eps, conservative=False, stab=S,
                   dt=1e-3, steps=10)
    s = 6
    a0 = 1e-7
    kx, ky = 3, 1
    h = L / n
    mu = (4 / h ** 2) * (math.sin(math.pi * kx / n) ** 2 + math.sin(math.pi * ky / n) ** 2)
    r = lambda dt: (1 + (S + 1) * dt) / (1 + S * dt + dt * eps * eps * mu)  # noqa: E731
    phi = r(p.dt) ** p.steps
    g = r(p.dt * p.steps)
    u0 = synth.single_mode(n, kx, ky, a0)
    for k in range(0, 4):
        if k == 0:
            U = np.empty((1, s + 1, n, n))
            U[:, 0] = u0
            for j in range(s):
                U[:, j + 1] = ac.coarse_num(U[:, j], p, ac.Coarse(dt=p.dt * p.steps))
        else:
            U = ac.parareal(u0, p, s, tol=0.0, max_iter=k).U
        for m in range(s + 1):
            coef = sum(math.comb(m, j) * (phi - g) ** j * g ** (m - j)
                       for j in range(0, min(k, m) + 1))
            assert np.abs(U[0, m] - coef * u0[0]).max() <= 1e-10 * a0


def test_parareal_batch_freezing_equals_individual_runs():
    p, s = _small_problem(True), 6
    u0 = synth.random_ic(32, [31, 32, 33])
    tol = 1e-6
    batch = ac.parareal(u0, p, s, tol=tol)
    for b in range(3):
        one = ac.parareal(u0[b:b + 1], p, s, tol=tol)
        assert one.iterations[0] == batch.iterations[b]
        assert np.array_equal(one.U[0], batch.U[b])


def test_parareal_converges_toward_fine():
    p, s = _small_problem(), 8
    u0 = synth.random_ic(32, [41])
    ref = ac.serial_fine_trajectory(u0, p, s)
    res = ac.parareal(u0, p, s, tol=1e-10)
    assert res.converged.all()
    assert ac.rel_l2(res.U, ref) <= 1e-9
    hist = [h[0] for h in res.history]
    assert hist[-1] <= 1e-10


# ---------------------------------------------------------------------------
# the pins catch plausible mistakes (mistakes planted in the oracle, on CPU)
# ---------------------------------------------------------------------------

def test_pins_catch_wrong_sign_in_nonlinearity(monkeypatch):
    # a wrong sign on the cubic term is invisible to the small-mode pin
    # (it is O(a0^3)) but not to the constant-field scalar map
    monkeypatch.setattr(ac, "f_double_well", lambda u: u + u * u * u)
    with pytest.raises(AssertionError):
        test_constant_field_classic_scalar_map()
    # a wrong sign on the linear term is caught by the linear factor
    monkeypatch.setattr(ac, "f_double_well", lambda u: -u - u * u * u)
    with pytest.raises(AssertionError):
        test_small_fourier_mode_decays_by_linear_factor(False)


def test_pins_catch_transposed_symbol(monkeypatch):
    real = ac.symbol_mu

    def wrong(n, h, laplacian="fd"):   # drop the y contribution
        m = real(n, h)
        kx = np.arange(n // 2 + 1)
        return np.broadcast_to((4 / h ** 2) * np.sin(np.pi * kx / n) ** 2, m.shape).copy()
    monkeypatch.setattr(ac, "symbol_mu", wrong)
    with pytest.raises(AssertionError):
        test_step_solves_the_stencil_system(False)


def test_pins_catch_missing_mean_in_conservative(monkeypatch):
    monkeypatch.setattr(ac, "_nonlocal_mean",
                        lambda fu, c: np.zeros(fu.shape[:-2] + (1, 1)))
    with pytest.raises(AssertionError):
        test_mass_conserved_to_1e13()


def test_pins_catch_wrong_correction_order(monkeypatch):
    # (G_new + F) - G_old instead of F + (G_new - G_old) breaks bitwise k=s
    src = ac.parareal

    def bad(u0, p, s, tol, max_iter=None, G=None):
        u0 = np.asarray(u0, dtype=np.float64)
        gdt = p.dt * p.steps
        Gf = G or (lambda v: ac.coarse_num(v, p, ac.Coarse(dt=gdt, steps=1)))
        U = np.empty((u0.shape[0], s + 1) + u0.shape[1:])
        U[:, 0] = u0
        gc = np.empty((u0.shape[0], s) + u0.shape[1:])
        for n in range(s):
            gc[:, n] = Gf(U[:, n])
            U[:, n + 1] = gc[:, n]
        for k in range(1, (max_iter or s) + 1):
            fw = np.stack([ac.fine(U[:, n], p) for n in range(k - 1, s)], 1)
            for n in range(k - 1, s):
                gn = Gf(U[:, n])
                U[:, n + 1] = (gn + fw[:, n - k + 1]) - gc[:, n]
                gc[:, n] = gn
        return ac.PararealResult(U=U, iterations=np.full(u0.shape[0], s),
                                 converged=np.ones(u0.shape[0], bool))
    monkeypatch.setattr(ac, "parareal", bad)
    with pytest.raises(AssertionError):
        test_parareal_k_equals_s_is_the_serial_fine_solve(False)
    monkeypatch.setattr(ac, "parareal", src)
