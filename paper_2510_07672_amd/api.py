"""Python binding of libpr: the entry points of include/pr.h under the same
names, taking torch CUDA tensors.  Argument marshalling only -- every step
of the computation runs in the library's HIP kernels.  Workspaces are
torch allocations sized by the library's *_workspace_bytes() calls, and
work is queued on torch's current stream.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float64: L.PR_F64, torch.float32: L.PR_F32}
_PREC = {"f64": L.PR_F64, "f32": L.PR_F32}


@dataclass(frozen=True)
class Problem:
    """Section 2 model on the Section 3.1 grid; see include/pr.h."""
    n: int
    length: float
    eps: float
    conservative: bool
    stab: float
    dt: float
    steps: int
    fine_prec: str = "f64"
    f32_iters: int = 0      # Parareal precision schedule (see pr_solve)
    scheme: str = "ssi"     # "ssi" or "cn" (Crank-Nicolson + Picard)
    picard: int = 3         # Picard iterations per CN step
    laplacian: str = "fd"   # "fd" (5-point) or "spectral" (Fourier collocation)

    def c(self) -> L.Problem:
        return L.Problem(2, self.n, self.length, self.eps, int(self.conservative), self.stab,
                         self.dt, self.steps, _PREC[self.fine_prec], int(self.f32_iters),
                         {"ssi": L.PR_SCHEME_SSI, "cn": L.PR_SCHEME_CN}[self.scheme],
                         int(self.picard), {"fd": L.PR_LAP_FD5, "spectral": L.PR_LAP_SPECTRAL}[self.laplacian])


@dataclass(frozen=True)
class Coarse:
    """Numerical coarse propagator: `steps` semi-implicit steps of `dt`."""
    dt: float
    steps: int = 1
    prec: str = "f64"

    def c(self) -> L.Coarse:
        return L.Coarse(kind=L.PR_G_SCHEME, dt=self.dt, steps=self.steps, prec=_PREC[self.prec])


_CNN_PREC = {"f64": L.PR_F64, "f32": L.PR_F32, "bf16": L.PR_BF16, "bf16x2": L.PR_BF16X2}


class CnnCoarse:
    """Convolutional coarse propagator (Section 3.2) with torch Conv2d
    weights: weights[l] [Cout, Cin, 3, 3], biases[l] [Cout], widths
    1 -> C -> ... -> C -> 1.  The tensors are concatenated into one FP32
    device buffer each, which this object keeps alive."""

    def __init__(self, weights, biases, act="gelu", residual=True, mass_fix=False,
                 limiter=None, prec="bf16", device="cuda"):
        if len(weights) != len(biases) or len(weights) < 2:
            raise ValueError("need >= 2 layers with one bias each")
        C = weights[0].shape[0]
        for l, (w, b) in enumerate(zip(weights, biases)):
            cin = 1 if l == 0 else C
            cout = 1 if l == len(weights) - 1 else C
            if tuple(w.shape) != (cout, cin, 3, 3) or tuple(b.shape) != (cout,):
                raise ValueError(f"layer {l}: expected W {(cout, cin, 3, 3)} and b {(cout,)}")
        self.n_layers, self.channels = len(weights), C
        dt = torch.float64 if prec == "f64" else torch.float32
        # flat parameter buffers, in the layout the library reads (and that
        # pr_cnn_backward's gradients use)
        self.W = torch.cat([w.reshape(-1) for w in weights]).to(device=device, dtype=dt).contiguous()
        self.B = torch.cat([b.reshape(-1) for b in biases]).to(device=device, dtype=dt).contiguous()
        self.act, self.residual, self.mass_fix, self.limiter = act, residual, mass_fix, limiter
        self.prec = prec

    def layers(self):
        """Views of the flat buffers as per-layer (W [Cout,Cin,3,3], b [Cout])."""
        out, wo, bo = [], 0, 0
        C, L = self.channels, self.n_layers
        for l in range(L):
            cin, cout = (1 if l == 0 else C), (1 if l == L - 1 else C)
            out.append((self.W[wo:wo + cout * cin * 9].view(cout, cin, 3, 3),
                        self.B[bo:bo + cout]))
            wo += cout * cin * 9
            bo += cout
        return out

    def c(self) -> L.Coarse:
        lo, hi = self.limiter if self.limiter is not None else (0.0, 0.0)
        return L.Coarse(kind=L.PR_G_CNN, prec=_CNN_PREC[self.prec], n_layers=self.n_layers,
                        channels=self.channels, weights=self.W.data_ptr(),
                        biases=self.B.data_ptr(),
                        act=L.PR_ACT_GELU if self.act == "gelu" else L.PR_ACT_TANH,
                        residual=int(self.residual), mass_fix=int(self.mass_fix),
                        limiter=int(self.limiter is not None), lim_lo=lo, lim_hi=hi)


@dataclass
class SolveStats:
    iterations: int
    n_converged: int
    ic_iterations: np.ndarray
    history: np.ndarray      # [iterations, n_ics] sup-norm updates
    fine_ms: float
    sweep_ms: float
    status: int


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None else 0)


def _fields(u: torch.Tensor, n: int, name: str) -> int:
    if not u.is_cuda or u.dtype != torch.float64 or not u.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA float64 tensor")
    if u.dim() != 3 or u.shape[1] != n or u.shape[2] != n:
        raise ValueError(f"{name} must have shape [B, {n}, {n}], got {tuple(u.shape)}")
    return u.shape[0]


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def pr_fine_propagate(p: Problem, u_in: torch.Tensor, out_dtype=torch.float64,
                      out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """F(U): p.steps fine steps on every field of u_in [B, N, N]."""
    B = _fields(u_in, p.n, "u_in")
    pc = p.c()
    if out is None:
        out = torch.empty((B, p.n, p.n), dtype=out_dtype, device=u_in.device)
    need = L.lib().pr_fine_workspace_bytes(C.byref(pc), B)
    if ws is None or ws.numel() < need:
        ws = workspace(need, u_in.device)
    L.check(L.lib().pr_fine_propagate(C.byref(pc), B, _ptr(u_in), _ptr(out), _DT[out.dtype],
                                      _ptr(ws), ws.numel(), _stream(u_in.device)),
            "pr_fine_propagate")
    return out


def pr_fine_propagate_noalloc(p: Problem, u_in: torch.Tensor, out: torch.Tensor):
    """F(U) into the caller's `out` [B, N, N] (float64 or float32) with the
    library's static scratch: no workspace, no allocation."""
    B = _fields(u_in, p.n, "u_in")
    if out.shape != u_in.shape or out.dtype not in _DT or not out.is_contiguous():
        raise TypeError("out must be a contiguous float64/float32 tensor shaped like u_in")
    pc = p.c()
    L.check(L.lib().pr_fine_propagate_noalloc(C.byref(pc), B, _ptr(u_in), _ptr(out), _DT[out.dtype],
                                              _stream(u_in.device)),
            "pr_fine_propagate_noalloc")
    return out


def pr_coarse_apply(p: Problem, g: Coarse, u_in: torch.Tensor,
                    out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """G(U) with the numerical coarse step."""
    B = _fields(u_in, p.n, "u_in")
    pc, gc = p.c(), g.c()
    if out is None:
        out = torch.empty_like(u_in)
    need = L.lib().pr_coarse_workspace_bytes(C.byref(pc), C.byref(gc), B)
    if ws is None or ws.numel() < need:
        ws = workspace(need, u_in.device)
    L.check(L.lib().pr_coarse_apply(C.byref(pc), C.byref(gc), B, _ptr(u_in), _ptr(out),
                                    _ptr(ws), ws.numel(), _stream(u_in.device)),
            "pr_coarse_apply")
    return out


def pr_cnn_backward(p: Problem, g: "CnnCoarse", u_in: torch.Tensor, grad_out: torch.Tensor,
                    ws: Optional[torch.Tensor] = None):
    """(dL/du, dL/dW, dL/db) of the network at u_in for dL/dG = grad_out; the
    parameter gradients are flat, laid out like g.W and g.B."""
    B = _fields(u_in, p.n, "u_in")
    _fields(grad_out, p.n, "grad_out")
    pc, gc = p.c(), g.c()
    du = torch.empty_like(u_in)
    dW = torch.empty_like(g.W)
    dB = torch.empty_like(g.B)
    need = L.lib().pr_cnn_backward_workspace_bytes(C.byref(pc), C.byref(gc), B)
    if ws is None or ws.numel() < need:
        ws = workspace(need, u_in.device)
    L.check(L.lib().pr_cnn_backward(C.byref(pc), C.byref(gc), B, _ptr(u_in), _ptr(grad_out),
                                    _ptr(du), _ptr(dW), _ptr(dB), _ptr(ws), ws.numel(),
                                    _stream(u_in.device)), "pr_cnn_backward")
    return du, dW, dB


def pr_scheme_loss(p: Problem, dt: float, u_n: torch.Tensor, u_np1: torch.Tensor,
                   grad: bool = True, resid: bool = False, ws: Optional[torch.Tensor] = None):
    """Mean squared Crank-Nicolson residual of the pairs (u_n, u_np1) over one
    step dt (eq. loss_ACN), as a 0-d device tensor, with dloss/du_np1 and
    the residual when asked for: returns (loss, grad or None, resid or None)."""
    B = _fields(u_n, p.n, "u_n")
    if _fields(u_np1, p.n, "u_np1") != B:
        raise ValueError("u_n and u_np1 must hold the same number of fields")
    pc = p.c()
    loss = torch.empty((), dtype=torch.float64, device=u_n.device)
    g = torch.empty_like(u_n) if grad else None
    r = torch.empty_like(u_n) if resid else None
    need = L.lib().pr_scheme_loss_workspace_bytes(C.byref(pc), B)
    if ws is None or ws.numel() < need:
        ws = workspace(need, u_n.device)
    L.check(L.lib().pr_scheme_loss(C.byref(pc), float(dt), B, _ptr(u_n), _ptr(u_np1), _ptr(loss),
                                   _ptr(g), _ptr(r), _ptr(ws), ws.numel(), _stream(u_n.device)),
            "pr_scheme_loss")
    return loss, g, r


def pr_correct(f: torch.Tensor, g_new: torch.Tensor, g_old: torch.Tensor, u: torch.Tensor,
               upd_max: torch.Tensor, update_cache: bool = True):
    """u <- f + (g_new - g_old); upd_max <- max(upd_max, |change|); g_old <- g_new."""
    B, n = u.shape[0], u.shape[-1]
    for t, nm in ((g_new, "g_new"), (g_old, "g_old"), (u, "u")):
        _fields(t, n, nm)
    if f.shape != u.shape or f.dtype not in _DT or not f.is_contiguous():
        raise TypeError("f must be a contiguous float64/float32 tensor shaped like u")
    if upd_max.dtype != torch.float64 or upd_max.numel() != B:
        raise TypeError("upd_max must be float64[B]")
    L.check(L.lib().pr_correct(B, n, _ptr(f), _DT[f.dtype], _ptr(g_new), _ptr(g_old), _ptr(u),
                               _ptr(upd_max), int(update_cache), _stream(u.device)),
            "pr_correct")
    return u


def pr_solve(p: Problem, g: Coarse, u0: torch.Tensor, n_slices: int, tol: float,
             max_iter: Optional[int] = None, U: Optional[torch.Tensor] = None,
             ws: Optional[torch.Tensor] = None, allow_not_converged: bool = False):
    """Algorithm 2 on every IC of u0 [B, N, N]; returns (U [B, s+1, N, N], stats)."""
    B = _fields(u0, p.n, "u0")
    pc, gc = p.c(), g.c()
    max_iter = n_slices + p.f32_iters if max_iter is None else int(max_iter)
    if U is None:
        U = torch.empty((B, n_slices + 1, p.n, p.n), dtype=torch.float64, device=u0.device)
    need = L.lib().pr_solve_workspace_bytes(C.byref(pc), C.byref(gc), B, n_slices)
    if ws is None or ws.numel() < need:
        ws = workspace(need, u0.device)
    ic_it = np.zeros(B, dtype=np.int32)
    hist = np.zeros(max(max_iter, 1) * B, dtype=np.float64)
    st = L.Stats(0, 0, ic_it.ctypes.data_as(C.POINTER(C.c_int32)),
                 hist.ctypes.data_as(C.POINTER(C.c_double)), 0.0, 0.0)
    allow = (L.PR_OK, L.PR_NOT_CONVERGED) if allow_not_converged else (L.PR_OK,)
    status = L.check(L.lib().pr_solve(C.byref(pc), C.byref(gc), B, n_slices, _ptr(u0), _ptr(U),
                                      float(tol), max_iter, C.byref(st), _ptr(ws), ws.numel(),
                                      _stream(u0.device)),
                     "pr_solve", allow)
    k = st.iterations
    stats = SolveStats(k, st.n_converged, ic_it.copy(), hist[:k * B].reshape(k, B).copy(),
                       st.fine_ms, st.sweep_ms, status)
    return U, stats


@dataclass
class Job:
    """One solve of a pr_solve_many batch."""
    problem: Problem
    coarse: object            # Coarse or CnnCoarse
    u0: torch.Tensor          # [B, N, N] float64
    n_slices: int
    tol: float
    max_iter: Optional[int] = None
    U: Optional[torch.Tensor] = None


def _job_c(j: Job):
    B = _fields(j.u0, j.problem.n, "u0")
    mi = j.n_slices + j.problem.f32_iters if j.max_iter is None else int(j.max_iter)
    if j.U is None:
        j.U = torch.empty((B, j.n_slices + 1, j.problem.n, j.problem.n), dtype=torch.float64,
                          device=j.u0.device)
    ic_it = np.zeros(B, dtype=np.int32)
    hist = np.zeros(max(mi, 1) * B, dtype=np.float64)
    st = L.Stats(0, 0, ic_it.ctypes.data_as(C.POINTER(C.c_int32)),
                 hist.ctypes.data_as(C.POINTER(C.c_double)), 0.0, 0.0)
    jc = L.Job(problem=j.problem.c(), coarse=j.coarse.c(), n_ics=B, n_slices=j.n_slices,
               max_iter=mi, tol=float(j.tol), u0=j.u0.data_ptr(), U=j.U.data_ptr(),
               stats=C.pointer(st), status=0)
    return jc, st, ic_it, hist, B


def pr_solve_many(jobs, ws: Optional[torch.Tensor] = None, allow_not_converged: bool = False):
    """Algorithm 2 for a heterogeneous batch of jobs; returns [(U, stats)] in job order."""
    if not jobs:
        return []
    keep = [_job_c(j) for j in jobs]
    arr = (L.Job * len(jobs))(*[k[0] for k in keep])
    need = L.lib().pr_solve_many_workspace_bytes(len(jobs), arr)
    if need == 0:
        raise ValueError("pr_solve_many_workspace_bytes rejected the batch")
    dev = jobs[0].u0.device
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    allow = (L.PR_OK, L.PR_NOT_CONVERGED) if allow_not_converged else (L.PR_OK,)
    L.check(L.lib().pr_solve_many(len(jobs), arr, _ptr(ws), ws.numel(), _stream(dev)),
            "pr_solve_many", allow)
    out = []
    for j, (jc, st, ic_it, hist, B), a in zip(jobs, keep, arr):
        k = st.iterations
        out.append((j.U, SolveStats(k, st.n_converged, ic_it.copy(),
                                    hist[:k * B].reshape(k, B).copy(), st.fine_ms, st.sweep_ms,
                                    a.status)))
    return out


def pr_serial_fine(p: Problem, u0: torch.Tensor, n_slices: int,
                   U: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """Serial fine solve [U_0, F(U_0), ...] -> U [B, s+1, N, N] (blocking)."""
    B = _fields(u0, p.n, "u0")
    pc = p.c()
    if U is None:
        U = torch.empty((B, n_slices + 1, p.n, p.n), dtype=torch.float64, device=u0.device)
    need = L.lib().pr_serial_workspace_bytes(C.byref(pc), B)
    if ws is None or ws.numel() < need:
        ws = workspace(need, u0.device)
    L.check(L.lib().pr_serial_fine(C.byref(pc), B, n_slices, _ptr(u0), _ptr(U), _ptr(ws),
                                   ws.numel(), _stream(u0.device)), "pr_serial_fine")
    return U


_PLAN = {"auto": L.PR_PLAN_AUTO, "stream": L.PR_PLAN_STREAM, "resident": L.PR_PLAN_RESIDENT}
_PLAN_NAME = {v: k for k, v in _PLAN.items()}


def pr_set_fine_plan(n: int, prec: str, plan: str) -> None:
    """Launch plan for (n, prec): 'auto', 'stream' or 'resident' (n <= 128)."""
    L.check(L.lib().pr_set_fine_plan(n, _PREC[prec], _PLAN[plan]), "pr_set_fine_plan")


def pr_get_fine_plan(n: int, prec: str) -> str:
    return _PLAN_NAME[L.lib().pr_get_fine_plan(n, _PREC[prec])]


_SPLIT = {"auto": L.PR_FFT_SPLIT_AUTO, "r8": L.PR_FFT_SPLIT_R8, "r4_tail": L.PR_FFT_SPLIT_R4_TAIL}
_SPLIT_NAME = {v: k for k, v in _SPLIT.items()}


def pr_set_fft_split(n: int, prec: str, split: str) -> None:
    """FFT radix split of the streaming semi-implicit passes for (n, prec):
    'auto', 'r8' (radix 8 first, the leftover last) or 'r4_tail' (a trailing
    8 x 2 as 4 x 4; differs for n = 16, 128, 1024)."""
    L.check(L.lib().pr_set_fft_split(n, _PREC[prec], _SPLIT[split]), "pr_set_fft_split")


def pr_get_fft_split(n: int, prec: str) -> str:
    v = L.lib().pr_get_fft_split(n, _PREC[prec])
    if v < 0:
        raise ValueError("unsupported (n, prec) = (%d, %s)" % (n, prec))
    return _SPLIT_NAME[v]


def pr_autotune_fine(p: Problem, u_in: torch.Tensor) -> str:
    """Time both plans on u_in and keep the faster as the 'auto' choice (and,
    for the streaming plan, the working-set budget, the FFT radix split and
    queue vs per-pass)."""
    B = _fields(u_in, p.n, "u_in")
    pc = p.c()
    out = torch.empty_like(u_in)
    ws = workspace(L.lib().pr_fine_workspace_bytes(C.byref(pc), B), u_in.device)
    ch = C.c_int32(0)
    L.check(L.lib().pr_autotune_fine(C.byref(pc), B, _ptr(u_in), _ptr(out), _ptr(ws), ws.numel(),
                                     _stream(u_in.device), C.byref(ch)), "pr_autotune_fine")
    return _PLAN_NAME[ch.value]


_CPLAN = {"auto": L.PR_CNN_PLAN_AUTO, "layered": L.PR_CNN_PLAN_LAYERED, "fused": L.PR_CNN_PLAN_FUSED,
          "folded": L.PR_CNN_PLAN_FOLDED}
_CPLAN_NAME = {v: k for k, v in _CPLAN.items()}


def pr_set_coarse_plan(plan: str) -> None:
    """Network inference plan, process-wide: 'auto', 'layered', 'fused' or
    'folded' (one launch per hidden layer, with the first convolution and,
    at 32 channels, the last one's per-tap products folded into them)."""
    L.check(L.lib().pr_set_coarse_plan(_CPLAN[plan]), "pr_set_coarse_plan")


def pr_get_coarse_plan(g: "CnnCoarse", n: int) -> str:
    return _CPLAN_NAME[L.lib().pr_get_coarse_plan(C.byref(g.c()), n)]


_CTILE = {"auto": L.PR_CNN_TILE_AUTO, "8x32": L.PR_CNN_TILE_8X32, "16x16": L.PR_CNN_TILE_16X16}
_CTILE_NAME = {v: k for k, v in _CTILE.items()}


def pr_set_coarse_tile(tile: str) -> None:
    """Output tile of the bf16 hidden-layer launches, process-wide: 'auto',
    '8x32' or '16x16' (32 and 48 channels).  Same bits under either."""
    L.check(L.lib().pr_set_coarse_tile(_CTILE[tile]), "pr_set_coarse_tile")


def pr_get_coarse_tile(g: "CnnCoarse", n: int) -> str:
    """The tile pr_coarse_apply uses for g on n x n fields; 'none' for a
    network without bf16 hidden layers."""
    v = L.lib().pr_get_coarse_tile(C.byref(g.c()), n)
    if v < 0:
        raise ValueError("not a valid network for n = %d" % n)
    return _CTILE_NAME.get(v, "none") if v else "none"


def pr_autotune_coarse(p: Problem, g: "CnnCoarse", u_in: torch.Tensor) -> str:
    """Time the network plans available for g on u_in, each bf16 layered or
    folded plan under both hidden-layer tiles, and keep the fastest pair as
    the 'auto' choices (pr_get_coarse_tile reports the tile)."""
    B = _fields(u_in, p.n, "u_in")
    pc, gc = p.c(), g.c()
    out = torch.empty_like(u_in)
    ws = workspace(L.lib().pr_coarse_workspace_bytes(C.byref(pc), C.byref(gc), B), u_in.device)
    ch = C.c_int32(0)
    L.check(L.lib().pr_autotune_coarse(C.byref(pc), C.byref(gc), B, _ptr(u_in), _ptr(out),
                                       _ptr(ws), ws.numel(), _stream(u_in.device), C.byref(ch)),
            "pr_autotune_coarse")
    return _CPLAN_NAME[ch.value]


def pr_set_fine_working_set(nbytes: int) -> None:
    """Budget (bytes of spectra in flight) of chunked streaming F calls; 0 = off."""
    L.check(L.lib().pr_set_fine_working_set(int(nbytes)), "pr_set_fine_working_set")


def pr_get_fine_working_set(n: int, prec: str) -> int:
    return int(L.lib().pr_get_fine_working_set(n, _PREC[prec]))


def pr_set_fine_queue(on) -> None:
    """Run the semi-implicit fine solves as one persistent work-queue launch
    per (N, precision) class (True / 1) or pass by pass (False / 0, default);
    2: the queue with every XCD queue adopted (device-wide hand-over only)."""
    L.check(L.lib().pr_set_fine_queue(int(on)), "pr_set_fine_queue")


def pr_get_fine_queue() -> int:
    return int(L.lib().pr_get_fine_queue())


def pr_get_fine_queue_choice(n: int, prec: str = "f64") -> int:
    """1 if the fine solves of (n, prec) take the work queue now, 0 if not,
    -1 for an unsupported pair."""
    return int(L.lib().pr_get_fine_queue_choice(int(n), _PREC[prec]))


def pr_set_overlap(chunks: int) -> None:
    """Fine-batch chunks overlapped with the sequential sweep (1 = no overlap)."""
    L.check(L.lib().pr_set_overlap(int(chunks)), "pr_set_overlap")


def pr_get_overlap() -> int:
    return int(L.lib().pr_get_overlap())


def pr_set_graphs(enabled: bool) -> None:
    """Replay captured launch sequences (True, default) or launch eagerly."""
    L.lib().pr_set_graphs(int(bool(enabled)))


def pr_get_graphs() -> bool:
    return bool(L.lib().pr_get_graphs())


def pr_abi_version() -> int:
    return L.lib().pr_abi_version()
