"""Training of the convolutional coarse propagator (Section 3.2).

Two losses:
  * `train`: the mean squared distance to fine-propagator trajectories
    (the loss the workloads fix), over unrolled checkpointed rollouts;
  * `train_scheme`: Algorithm 1 with the scheme-based loss eq. loss_ACN,
    the residual of the Crank-Nicolson scheme (eq. fully-discrete) over one
    coarse step, which needs no fine-solver data; the residual, the loss
    and its gradient run in libpr (pr_scheme_loss).

Data: R initial conditions, each advanced slice by slice with the FP64
fine propagator (pr_serial_fine), so targets are U_{t+1} = F(U_t).
Training step: a batch of trajectories, an unrolled rollout of `rollout`
network applications from U_t (checkpointed every `ckpt` steps), the mean
squared distance to U_{t+1..t+rollout}, and an Adam update of the flat
parameter buffers.  The optimiser is torch's; forward and backward of the
network run in libpr.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List

import torch

from . import api, autograd, synth


def init_network(n_layers: int, channels: int, seed: int, prec: str = "bf16",
                 act: str = "gelu", out_scale: float = 0.1, **kw) -> api.CnnCoarse:
    """torch.nn.Conv2d default initialisation under a fixed seed; the last
    layer is scaled by out_scale so the untrained G starts near u -> u."""
    g = torch.Generator().manual_seed(seed)
    widths = [1] + [channels] * (n_layers - 1) + [1]
    ws, bs = [], []
    for l in range(n_layers):
        bound = 1.0 / math.sqrt(widths[l] * 9)
        w = (torch.rand((widths[l + 1], widths[l], 3, 3), generator=g) * 2 - 1) * bound
        b = (torch.rand((widths[l + 1],), generator=g) * 2 - 1) * bound
        if l == n_layers - 1:
            w, b = w * out_scale, b * out_scale
        ws.append(w)
        bs.append(b)
    return api.CnnCoarse(ws, bs, act=act, prec=prec, **kw)


def make_dataset(p: api.Problem, seeds, n_slices: int, device="cuda") -> torch.Tensor:
    """[R, n_slices + 1, N, N] fine trajectories (FP64 fine propagator)."""
    import dataclasses
    p64 = dataclasses.replace(p, fine_prec="f64")
    u0 = torch.from_numpy(synth.random_ic(p.n, seeds)).to(device)
    return api.pr_serial_fine(p64, u0, n_slices)


@dataclass
class TrainLog:
    loss: List[float] = field(default_factory=list)
    step_ms: List[float] = field(default_factory=list)


def train(net: api.CnnCoarse, p: api.Problem, data: torch.Tensor, steps: int, batch: int = 32,
          rollout: int = 8, ckpt: int = 2, lr: float = 1e-3, seed: int = 0,
          progress=None, lr_final: float = None, lr_drop: float = None) -> TrainLog:
    """`steps` Adam updates on random (trajectory, start) pairs; `progress`,
    if given, is called as progress(step, loss, ms) after every update.
    With `lr_final` the learning rate follows a cosine from `lr` down to it
    over the run; with `lr_drop` = q it drops to lr / 10 for the last
    fraction q of the steps; otherwise it stays at `lr`."""
    R, T1 = data.shape[0], data.shape[1]
    if T1 - 1 < rollout:
        raise ValueError("trajectories shorter than the rollout")
    net.W.requires_grad_(True)
    net.B.requires_grad_(True)
    opt = torch.optim.Adam([net.W, net.B], lr=lr)
    sched = (torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=max(1, steps), eta_min=lr_final)
             if lr_final is not None else None)
    gen = torch.Generator().manual_seed(seed)
    log = TrainLog()
    drop_at = steps - int(round(steps * lr_drop)) if lr_drop else None
    for it in range(steps):
        if drop_at is not None and it == drop_at:
            for grp in opt.param_groups:
                grp["lr"] = lr * 0.1
        idx = torch.randint(0, R, (batch,), generator=gen)
        t0 = torch.randint(0, T1 - rollout, (batch,), generator=gen)
        u0 = data[idx, t0].contiguous()
        tgt = torch.stack([data[idx, t0 + k + 1] for k in range(rollout)])
        torch.cuda.synchronize()
        tic = time.perf_counter()
        out = autograd.cnn_rollout(net, p, u0, rollout, ckpt)
        loss = ((out - tgt) ** 2).mean()
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if sched is not None:
            sched.step()
        torch.cuda.synchronize()
        log.step_ms.append((time.perf_counter() - tic) * 1e3)
        log.loss.append(float(loss.item()))
        if progress is not None:
            progress(len(log.loss), log.loss[-1], log.step_ms[-1])
    net.W.requires_grad_(False)
    net.B.requires_grad_(False)
    return log


def train_scheme(net: api.CnnCoarse, p: api.Problem, u0: torch.Tensor, dt: float, n_steps: int,
                 inner: int = 4, subset: int = 16, lr: float = 1e-3, seed: int = 0,
                 progress=None) -> TrainLog:
    """Algorithm 1: the initial conditions u0 [R, N, N] are split at random
    into subsets of `subset`; for each subset, for n = 0..n_steps-1, take
    `inner` Adam updates on the mean squared scheme residual of
    (U_n, G(U_n)) (eq. loss_ACN, step dt), then fix U_{n+1} = G(U_n) and go
    on.  `progress(update, loss, ms)` is called after every update."""
    net.W.requires_grad_(True)
    net.B.requires_grad_(True)
    opt = torch.optim.Adam([net.W, net.B], lr=lr)
    gen = torch.Generator().manual_seed(seed)
    order = torch.randperm(u0.shape[0], generator=gen)
    log = TrainLog()
    for s0 in range(0, u0.shape[0], subset):
        U = u0[order[s0:s0 + subset].to(u0.device)].contiguous()
        for _ in range(n_steps):
            for _ in range(inner):
                torch.cuda.synchronize()
                tic = time.perf_counter()
                out = autograd.cnn_apply(net, p, U)
                loss = autograd.scheme_loss(p, U, out, dt)
                opt.zero_grad(set_to_none=True)
                loss.backward()
                opt.step()
                torch.cuda.synchronize()
                log.step_ms.append((time.perf_counter() - tic) * 1e3)
                log.loss.append(float(loss.item()))
                if progress is not None:
                    progress(len(log.loss), log.loss[-1], log.step_ms[-1])
            with torch.no_grad():
                U = api.pr_coarse_apply(p, net, U)
    net.W.requires_grad_(False)
    net.B.requires_grad_(False)
    return log
