"""FP64 reference for the Allen-Cahn fine propagator and Parareal.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain, slow and
written to be checked against the paper by eye.  Arrays are float64,
C-ordered, shaped [..., N, N] with u[..., i, j] = u(x_i, y_j),
x_i = i*h, h = L/N, i = 0..N-1 (the paper's i = 1..N with the periodic
identification U^0 = U^N, Section 3.1).

Model (Section 2): classic AC  u_t = eps^2 Lap u + f(u), and the
mass-conservative AC (eq. mass_AC_eq) which subtracts the domain mean of
f(u); f(u) = u - u^3 from the double-well potential F(u) = (u^2-1)^2/4.

Fine scheme.  The paper's fine operator (eq. fine_operator) is whichever
fully discrete scheme advances U_n to U_{n+1}; the workloads here fix it
as the stabilised semi-implicit step of the family the introduction
cites (Shen-Yang, Tang-Yang), with the central-difference Laplacian that
Section 3.1 allows:

    (u+ - u)/dt = eps^2 Lap_h u+ + f(u) - m(u) - S (u+ - u)

i.e.  ((1 + S dt) I - dt eps^2 Lap_h) u+ = (1 + S dt) u + dt (f(u) - m(u)),

with m(u) = 0 (classic) or the grid mean of f(u) (conservative; the
discrete nonlocal term g of Section 3.1).  Lap_h is the periodic 5-point
stencil, whose discrete Fourier symbol is -mu_k with
mu_k = (4/h^2)(sin^2(pi kx/N) + sin^2(pi ky/N)); the linear system is
therefore solved exactly by one forward and one inverse 2-D real DFT.

The paper's own fine scheme (Section 3.1, eq. fully-discrete) is also
here: Crank-Nicolson in time, solved by Picard iteration from
U_{n+1,(0)} = U_n,

    (I - dt/2 eps^2 Lap_h) U_{(m+1)} = U_n + dt/2 (eps^2 Lap_h U_n + f(U_n)
                                       + f(U_{(m)})) - dt g(U_n, U_{(m)}),

g = 0 (classic) or the grid mean of (f(U_n) + f(U_{(m)}))/2
(conservative), taken with the full factor dt as in the paper's first
displayed form of the scheme, which is the placement that keeps the mass
(the later displays put g inside the dt/2 bracket).  A fixed number of
Picard iterations stands in for the paper's unstated stopping rule.
Either scheme may use the Fourier collocation Laplacian that Section 3.1
also allows instead of the 5-point stencil.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.fft as sfft

_WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------------------
# problem description
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Problem:
    """The initial-value problem of Section 2 on the grid of Section 3.1.

    n            grid points per side (N); h = length / n
    length       side L of the periodic square [0, L]^2
    eps          interfacial parameter epsilon
    conservative False: classic AC; True: mass-conservative AC
    stab         stabiliser S of the semi-implicit step (>= 0)
    dt           fine step dt*
    steps        fine steps per Parareal slice (c = Delta t / dt*)
    """

    n: int
    length: float
    eps: float
    conservative: bool
    stab: float
    dt: float
    steps: int
    scheme: str = "ssi"      # "ssi" (stabilised semi-implicit) or "cn" (CN + Picard)
    picard: int = 3          # Picard iterations per CN step
    laplacian: str = "fd"    # "fd" (5-point stencil) or "spectral" (Fourier collocation)

    @property
    def h(self) -> float:
        return self.length / self.n


@dataclass(frozen=True)
class Coarse:
    """Numerical coarse propagator: `steps` semi-implicit steps of `dt`."""

    dt: float
    steps: int = 1


# ---------------------------------------------------------------------------
# pointwise pieces (Section 2)
# ---------------------------------------------------------------------------

def f_double_well(u: np.ndarray) -> np.ndarray:
    """f(u) = u - u^3 = -F'(u), F(u) = (u^2 - 1)^2 / 4 (Section 2)."""
    return u - u * u * u


def potential(u: np.ndarray) -> np.ndarray:
    """Double-well potential F(u) = (u^2 - 1)^2 / 4 (Section 2)."""
    return 0.25 * (u * u - 1.0) ** 2


def laplacian_stencil(u: np.ndarray, h: float) -> np.ndarray:
    """Periodic central-difference (5-point) Laplacian, Section 3.1.

    Written with array shifts and no transform; the spectral solver is
    checked against this.
    """
    return (np.roll(u, 1, axis=-2) + np.roll(u, -1, axis=-2)
            + np.roll(u, 1, axis=-1) + np.roll(u, -1, axis=-1)
            - 4.0 * u) / (h * h)


def laplacian_spectral(u: np.ndarray, length: float) -> np.ndarray:
    """Fourier collocation Laplacian (Section 3.1's alternative): multiply
    the DFT coefficient of wavenumber (kx, ky) by -(2 pi / L)^2 (kx^2 + ky^2),
    with k taken in -N/2..N/2-1 (numpy's fftfreq order)."""
    n = u.shape[-1]
    k = np.fft.fftfreq(n, d=1.0 / n)
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    return np.real(np.fft.ifft2(-(2 * np.pi / length) ** 2 * k2 * np.fft.fft2(u)))


def apply_laplacian(u: np.ndarray, p: "Problem") -> np.ndarray:
    """Lap_h u with the problem's choice of discrete Laplacian."""
    return laplacian_stencil(u, p.h) if p.laplacian == "fd" else laplacian_spectral(u, p.length)


def symbol_mu(n: int, h: float, laplacian: str = "fd") -> np.ndarray:
    """mu_k >= 0 with Lap_h e_k = -mu_k e_k, on the rfft2 half grid.

    Shape [n, n//2 + 1]; row index ky = 0..n-1, column kx = 0..n/2.
    5-point stencil: (4/h^2)(sin^2(pi kx/N) + sin^2(pi ky/N)); Fourier
    collocation: (2 pi / L)^2 (kx^2 + ky^2) with wrapped wavenumbers.
    """
    ky = np.arange(n, dtype=np.float64)[:, None]
    kx = np.arange(n // 2 + 1, dtype=np.float64)[None, :]
    if laplacian == "spectral":
        ky = np.minimum(ky, n - ky)
        L = n * h
        return (2 * np.pi / L) ** 2 * (kx * kx + ky * ky)
    sy = np.sin(np.pi * ky / n)
    sx = np.sin(np.pi * kx / n)
    return (4.0 / (h * h)) * (sx * sx + sy * sy)


def _nonlocal_mean(fu: np.ndarray, conservative: bool) -> np.ndarray:
    """Discrete Lagrange multiplier: grid mean of f(u) per field, or 0."""
    if not conservative:
        return np.zeros(fu.shape[:-2] + (1, 1))
    return fu.mean(axis=(-2, -1), keepdims=True)


# ---------------------------------------------------------------------------
# the fine scheme and the propagators (Section 3.1, eq. fine_operator)
# ---------------------------------------------------------------------------

def ssi_step(u: np.ndarray, n: int, h: float, eps: float, stab: float,
             dt: float, conservative: bool, laplacian: str = "fd") -> np.ndarray:
    """One stabilised semi-implicit step; u has shape [..., n, n].

    Right-hand side (1 + S dt) u + dt (f(u) - m), then the exact solve of
    ((1 + S dt) I - dt eps^2 Lap_h) u+ = rhs by division in Fourier space.
    """
    a = 1.0 + stab * dt
    fu = f_double_well(u)
    rhs = a * u + dt * (fu - _nonlocal_mean(fu, conservative))
    denom = a + dt * eps * eps * symbol_mu(n, h, laplacian)
    spec = sfft.rfft2(rhs, axes=(-2, -1), workers=_WORKERS)
    return sfft.irfft2(spec / denom, s=(n, n), axes=(-2, -1), workers=_WORKERS)


def solve_cn_operator(rhs: np.ndarray, p: "Problem", dt: float) -> np.ndarray:
    """v with (I - dt/2 eps^2 Lap_h) v = rhs (exact, by division in Fourier space)."""
    denom = 1.0 + 0.5 * dt * p.eps * p.eps * symbol_mu(p.n, p.h, p.laplacian)
    spec = sfft.rfft2(rhs, axes=(-2, -1), workers=_WORKERS)
    return sfft.irfft2(spec / denom, s=(p.n, p.n), axes=(-2, -1), workers=_WORKERS)


def cn_nonlocal(fn: np.ndarray, fv: np.ndarray, conservative: bool) -> np.ndarray:
    """g(U_n, V): 0, or the grid mean of (f(U_n) + f(V)) / 2 (Section 3.1)."""
    if not conservative:
        return np.zeros(fn.shape[:-2] + (1, 1))
    return 0.5 * (fn.mean(axis=(-2, -1), keepdims=True) + fv.mean(axis=(-2, -1), keepdims=True))


def cn_picard_step(u: np.ndarray, p: "Problem", dt: float, iters: Optional[int] = None,
                   trace: Optional[list] = None) -> np.ndarray:
    """One Crank-Nicolson step (eq. fully-discrete) by `iters` Picard
    iterations from V_(0) = U_n; each solves the linear system of the
    Picard form of Section 3.1.  `trace`, if given, receives every iterate."""
    iters = p.picard if iters is None else iters
    u = np.asarray(u, dtype=np.float64)
    fn = f_double_well(u)
    explicit = u + 0.5 * dt * (p.eps * p.eps * apply_laplacian(u, p) + fn)
    v = u.copy()
    for _ in range(iters):
        fv = f_double_well(v)
        rhs = explicit + 0.5 * dt * fv - dt * cn_nonlocal(fn, fv, p.conservative)
        v = solve_cn_operator(rhs, p, dt)
        if trace is not None:
            trace.append(v)
    return v


def cn_residual(u: np.ndarray, v: np.ndarray, p: "Problem", dt: float) -> np.ndarray:
    """Residual of eq. fully-discrete (mass-keeping placement of g) for the
    pair (U_n, U_{n+1}) = (u, v), computed pointwise with no solve."""
    fu, fv = f_double_well(u), f_double_well(v)
    return (v - u - 0.5 * dt * (p.eps * p.eps * (apply_laplacian(v, p) + apply_laplacian(u, p))
                                + fu + fv) + dt * cn_nonlocal(fu, fv, p.conservative))


def cn_residual_loss(u: np.ndarray, v: np.ndarray, p: "Problem", dt: float):
    """The scheme-based training loss of Algorithm 1 (eq. loss_ACN) for the
    pairs (U_n, U_{n+1}) = (u, v): L = mean of cn_residual^2 over every
    point of every pair, and dL/dv.

    The residual is linear in the stencil and pointwise in f, so with
    J = dr/dv = I - dt/2 (eps^2 Lap_h + diag f'(v)) + dt/2 (1/N^2) 1 f'(v)^T
    (the last term in the conservative model only, f' = 1 - 3 v^2) the
    gradient is (2/M) J^T r; Lap_h is symmetric.  M = number of points."""
    r = cn_residual(u, v, p, dt)
    m = r.size
    fp = 1.0 - 3.0 * v * v
    g = r - 0.5 * dt * (p.eps * p.eps * apply_laplacian(r, p) + fp * r)
    if p.conservative:
        g = g + 0.5 * dt * fp * r.mean(axis=(-2, -1), keepdims=True)
    return float((r * r).mean()), (2.0 / m) * g


def step(u: np.ndarray, p: "Problem", dt: float) -> np.ndarray:
    """One step of the problem's fine scheme with step size dt."""
    if p.scheme == "cn":
        return cn_picard_step(u, p, dt)
    return ssi_step(u, p.n, p.h, p.eps, p.stab, dt, p.conservative, p.laplacian)


def fine(u: np.ndarray, p: Problem) -> np.ndarray:
    """Fine propagator F(t_n, t_{n+1}, U_n): p.steps steps of p.dt."""
    v = np.array(u, dtype=np.float64, copy=True)
    for _ in range(p.steps):
        v = step(v, p, p.dt)
    return v


def coarse_num(u: np.ndarray, p: Problem, g: Coarse) -> np.ndarray:
    """Numerical coarse propagator: g.steps steps of g.dt of the fine scheme."""
    v = np.array(u, dtype=np.float64, copy=True)
    for _ in range(g.steps):
        v = step(v, p, g.dt)
    return v


def serial_fine_trajectory(u0: np.ndarray, p: Problem, s: int) -> np.ndarray:
    """[U_0, F(U_0), F(F(U_0)), ...]: the serial fine solve, [B, s+1, N, N]."""
    u0 = np.asarray(u0, dtype=np.float64)
    out = np.empty((u0.shape[0], s + 1) + u0.shape[1:], dtype=np.float64)
    out[:, 0] = u0
    for n in range(s):
        out[:, n + 1] = fine(out[:, n], p)
    return out


# ---------------------------------------------------------------------------
# Parareal (Section 3.3, Algorithm 2)
# ---------------------------------------------------------------------------

@dataclass
class PararealResult:
    U: np.ndarray                       # [B, s+1, N, N] final iterate
    iterations: np.ndarray              # [B] iteration at which each IC stopped
    converged: np.ndarray               # [B] bool
    history: List[np.ndarray] = field(default_factory=list)  # per k: [B] sup-norm update


def parareal(u0: np.ndarray, p: Problem, s: int, tol: float,
             max_iter: Optional[int] = None, G=None) -> PararealResult:
    """Algorithm 2 for a batch of initial conditions u0 [B, N, N].

    G defaults to the numerical coarse step of one slice length; pass any
    callable [M, N, N] -> [M, N, N] (e.g. a network) instead.

    Readings of points the paper leaves open:
      * the correction is evaluated as F + (G_new - G_old), so a slice
        whose input did not change receives F bit for bit;
      * G(U^{k-1}_n) is kept from the previous sweep rather than
        recomputed (the cost model of Section 3.4 counts it once);
      * the update norm is the sup norm over all slices and points of each
        initial condition, tested with <= tol; an initial condition that
        has converged is frozen, so a batch equals its members run alone;
      * at most s iterations: after k iterations slices 0..k equal the
        serial fine solve (Section 3.3), so k = s is exact.
    """
    u0 = np.asarray(u0, dtype=np.float64)
    B = u0.shape[0]
    if G is None:
        gdt = p.dt * p.steps
        G = lambda v: coarse_num(v, p, Coarse(dt=gdt, steps=1))  # noqa: E731
    if max_iter is None:
        max_iter = s
    max_iter = min(max_iter, s)

    U = np.empty((B, s + 1) + u0.shape[1:], dtype=np.float64)
    gcache = np.empty((B, s) + u0.shape[1:], dtype=np.float64)
    U[:, 0] = u0
    # initial guess: sequential coarse sweep U^0_{n+1} = G(U^0_n)
    for n in range(s):
        gcache[:, n] = G(U[:, n])
        U[:, n + 1] = gcache[:, n]

    active = np.ones(B, dtype=bool)
    iterations = np.zeros(B, dtype=np.int64)
    history: List[np.ndarray] = []
    for k in range(1, max_iter + 1):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        # fine solves on the window n = k-1 .. s-1, all independent
        window = U[idx, k - 1:s]                       # [b, s-k+1, N, N]
        fw = fine(window.reshape((-1,) + u0.shape[1:]), p).reshape(window.shape)
        Unew = U[idx].copy()
        gc = gcache[idx]
        # sequential correction sweep
        for n in range(k - 1, s):
            gnew = G(Unew[:, n])
            Unew[:, n + 1] = fw[:, n - (k - 1)] + (gnew - gc[:, n])
            gc[:, n] = gnew
        upd = np.abs(Unew - U[idx]).max(axis=(1, 2, 3))
        full = np.zeros(B)
        full[idx] = upd
        history.append(full)
        U[idx] = Unew
        gcache[idx] = gc
        iterations[idx] = k
        done = upd <= tol
        active[idx[done]] = False
    converged = ~active
    # reaching k = s makes every slice the fine solution
    converged |= iterations >= s
    return PararealResult(U=U, iterations=iterations, converged=converged,
                          history=history)


# ---------------------------------------------------------------------------
# diagnostics (Section 2: mass, energy, MBP; Section 4: error metric)
# ---------------------------------------------------------------------------

def mass(u: np.ndarray) -> np.ndarray:
    """Grid mean of u per field (the discrete M(t) / |Omega|)."""
    return np.asarray(u, dtype=np.float64).mean(axis=(-2, -1))


def discrete_energy(u: np.ndarray, eps: float, h: float) -> np.ndarray:
    """E_h(u) = h^2 sum( eps^2/2 |grad_h^+ u|^2 + F(u) ) (eq. energy)."""
    dx = (np.roll(u, -1, axis=-2) - u) / h
    dy = (np.roll(u, -1, axis=-1) - u) / h
    dens = 0.5 * eps * eps * (dx * dx + dy * dy) + potential(u)
    return h * h * dens.sum(axis=(-2, -1))


def rel_l2(u: np.ndarray, ref: np.ndarray) -> float:
    """Relative L2 error ||u - ref||_2 / ||ref||_2 (Section 4)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((u - ref).ravel()) / np.linalg.norm(ref.ravel()))


def mbp_bound(conservative: bool) -> float:
    """Maximum-bound value: 1 (classic), 2/sqrt(3) (conservative), Section 2."""
    return 2.0 / math.sqrt(3.0) if conservative else 1.0
