"""Benchmark of the Parareal hot path on one MI355X.

One timed step = one pass of the whole hot path over one batch: the
initial coarse sweep, then one Parareal iteration with the fine solves of
every slice of every initial condition in one batch (stage-in, 2-D FFT
steps with the pointwise right-hand side, the spectral divide and, for the
conservative model, the FP64 mass multiplier) and the sequential
coarse/correction sweep with its FP64 norm -- i.e. pr_solve with
max_iter = 1.  Default workload: the largest, the mass-conservative
512^2 batch of 16 ICs x 128 slices with the 6 x 48 network; the 256^2
workload follows as a second section.

value = fine-step grid-point updates per second (B * s * c * N^2 / time)
roofline_fine = the fine sweep (row + column pass of every step), timed
with HIP events inside pr_solve on the launch stream, against HBM;
roofline_coarse = one network call, timed with events on the same stream,
against the bf16 matrix-core peak; roofline = whichever of the two takes
the larger share of the step.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

CONFIGS = {
    "c1": dict(workload="classic AC 64x64 eps=0.02 FP64, 1 IC x 8 slices x 100 steps dt=1e-4, "
                        "numerical G (1 step of 0.01)",
               n=64, eps=0.02, dt=1e-4, steps=100, slices=8, ics=1, conservative=False,
               seed0=0, g_steps=1, cnn=(4, 32)),
    "c2": dict(workload="classic AC 256x256 eps=0.01, 8 ICs x 64 slices x 200 steps dt=2e-5 "
                        "(512 fine solves per launch), G = u + CNN(u) 4 conv x 32 ch",
               n=256, eps=0.01, dt=2e-5, steps=200, slices=64, ics=8, conservative=False,
               seed0=0, g_steps=1, cnn=(4, 32), train_steps=2000, train_traj=512),
    "c3": dict(workload="mass-conservative AC 512x512 eps=0.01, 16 ICs x 128 slices x 100 steps "
                        "dt=1e-5 (2048 fine solves per launch), G = u + CNN(u) 6 conv x 48 ch",
               n=512, eps=0.01, dt=1e-5, steps=100, slices=128, ics=16, conservative=True,
               seed0=0, g_steps=1, cnn=(6, 48), train_steps=60, train_traj=128),
}


def note(msg: str) -> None:
    """Progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_point_step(prec: str, scheme: str = "ssi", picard: int = 1) -> int:
    """Algorithmic HBM bytes per grid point and fine step.

    Semi-implicit step: one column pass and one row pass, each reading and
    writing the field's N*N real numbers once (as N/2 x N complex values):
    4 words.  Crank-Nicolson with M Picard iterations: per iteration a
    column pass (read and write the row spectra, read the second spectral
    buffer, and write it at the first and the last iteration) and a row
    pass (read and write): 5 M + 2 words (6 for M = 1)."""
    w = 8 if prec == "f64" else 4
    if scheme == "cn":
        return w * (5 * picard + (1 if picard == 1 else 2))
    return 4 * w


def kernel_src_hash(files=("fine_kernels.hip", "fft_lds.h", "internal.h")) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2510_07672_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def network_traffic(cfg_name):
    """HBM bytes of one network call (every kernel of the call: weight
    packing, hidden layers, gather) from the committed FETCH_SIZE /
    WRITE_SIZE summary of the workload's network, scaled by a plain copy;
    None if the network kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"coarse_cnn_{cfg_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("src_hash") != kernel_src_hash(("cnn_kernels.hip", "gelu_coef.h", "internal.h")):
        return None
    return d["bytes_per_call"]


def measured_traffic(cfg_name, prec, n, nfields):
    """HBM bytes of one fine step over `nfields` fields (middle row pass +
    column pass of the fine sweep) from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, already scaled by the plain-copy
    calibration; None if the kernels changed since the counters were
    taken.  A streaming call may run its fields in working-set chunks: the
    largest dispatch covers grid / (N^2 / 16) fields (256-thread column
    blocks of 2048 / N columns), and the step is scaled from it."""
    path = os.path.join(ROOT, "profiles", f"fine_step_{cfg_name}_{prec}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("src_hash") != kernel_src_hash():
        return None
    per = d["per_dispatch"]
    t = "double" if prec == "f64" else "float"

    def biggest(names):
        cands = [(int(k.split("@")[1]), v) for k, v in per.items() if k.split("@")[0] in names]
        return max(cands, key=lambda c: c[0]) if cands else None
    # the middle row pass and the column pass, named with or without their
    # right-hand-side and radix-split template arguments
    row = biggest({f"pr::k_row<{n}, {t}, 1>", f"pr::k_row<{n}, {t}, 1, 0>",
                   f"pr::k_row<{n}, {t}, 1, 0, 0>", f"pr::k_row<{n}, {t}, 1, 0, 1>"})
    col = biggest({f"pr::k_col<{n}, {t}>", f"pr::k_col<{n}, {t}, 0>", f"pr::k_col<{n}, {t}, 1>"})
    if row is None or col is None:
        return None
    fields_per_dispatch = col[0] * 16 // (n * n)
    row, col = row[1], col[1]
    per_step = (row["fetch_MB"] + row["write_MB"] + col["fetch_MB"] + col["write_MB"]) * 1e6
    return per_step * nfields / max(1, fields_per_dispatch)


def cpu_baseline(cfg, prec, budget_s=12.0):
    """The FP64 oracle on host cores: fine steps of the same fields."""
    from oracle import allen_cahn as ac
    from paper_2510_07672_amd import synth
    n = cfg["n"]
    p = ac.Problem(n=n, length=1.0, eps=cfg["eps"], conservative=cfg["conservative"], stab=2.0,
                   dt=cfg["dt"], steps=1)
    u = synth.random_ic(n, range(cfg["seed0"], cfg["seed0"] + cfg["ics"]))
    ac.fine(u, p)  # warm-up (plans, pages)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        u = ac.fine(u, p)
        steps += 1
    dt = time.perf_counter() - t0
    pts = steps * u.shape[0] * n * n
    return {"value": pts / dt / 1e9, "unit": "Gpts/s", "cores": os.cpu_count(),
            "kind": "oracle",
            "sample": f"{steps} FP64 fine steps of {u.shape[0]} {n}x{n} fields "
                      f"(scipy.fft, workers={os.cpu_count()}) in {dt:.1f} s"}


def parareal_vs_serial(api, p, g, u0, s, kmax, target=1e-6):
    """Wall-clock of Parareal stopped after k iterations against the FP64
    serial fine solve on the same GPU.

    Accuracy criterion: the worst relative L2 error of any slice of any
    initial condition, max_{b, n} |U_bn - ref_bn| / |ref_bn|, is <= target
    (slices 0..k are exact after k iterations, so an error over the stacked
    trajectory would dilute the later slices').  The smallest k meeting it
    gives the speedup; the smallest k whose stacked trajectory error is
    <= target is reported beside it as a second key.  With p.f32_iters = K
    the first K iterations run FP32 fine solves (precision schedule), and k
    counts them too."""
    import dataclasses
    import torch
    p64 = dataclasses.replace(p, fine_prec="f64", f32_iters=0)

    def timed(fn, reps=3):
        best = None
        out = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            best = dt if best is None else min(best, dt)
        return out, best

    ref, t_ser64 = timed(lambda: api.pr_serial_fine(p64, u0, s))
    note(f"serial FP64 fine solve: {t_ser64:.1f} ms")
    ser_same, t_ser = timed(lambda: api.pr_serial_fine(p, u0, s))
    nref = torch.linalg.vector_norm(ref).item()
    rel_same = torch.linalg.vector_norm(ser_same - ref).item() / nref
    ref_slice = torch.linalg.vector_norm(ref, dim=(-2, -1))          # [B, s+1]
    hist = []
    found = stacked = None
    per_slice = None

    def solve(k):
        return api.pr_solve(p, g, u0, s, tol=0.0, max_iter=k, allow_not_converged=True)
    for k in range(1, min(kmax, s) + p.f32_iters + 1):
        (U, st), t = timed(lambda: solve(k), reps=1)
        err = torch.linalg.vector_norm(U - ref).item() / nref
        ps = (torch.linalg.vector_norm(U - ref, dim=(-2, -1)) / ref_slice).max(dim=0).values
        worst, final = ps.max().item(), ps[-1].item()
        del U
        hist.append({"k": k, "rel_l2": float(f"{err:.3e}"), "worst_slice_rel_l2": float(f"{worst:.3e}"),
                     "final_slice_rel_l2": float(f"{final:.3e}"), "ms": round(t, 2)})
        note(f"parareal f32_iters={p.f32_iters} k={k}: rel-L2 {err:.3e} stacked, {worst:.3e} "
             f"worst slice, {final:.3e} final slice, in {t:.1f} ms")
        if stacked is None and err <= target:
            _, tk = timed(lambda: solve(k), reps=3)
            stacked = {"k": k, "ms": round(tk, 2), "rel_l2": float(f"{err:.3e}")}
        if worst <= target:
            _, tk = (None, stacked["ms"]) if stacked and stacked["k"] == k else \
                timed(lambda: solve(k), reps=3)
            found = {"k": k, "ms": round(tk, 2), "worst": worst, "final": final, "rel_l2": err}
            per_slice = [float(f"{x:.2e}") for x in ps[1:].tolist()]
            break
    res = {"target_rel_l2": target,
           "criterion": "max over ICs and slices of the per-slice rel-L2 against the FP64 serial "
                        "fine solve <= target",
           "serial_fp64_ms": round(t_ser64, 2),
           "serial_same_prec_ms": round(t_ser, 2), "serial_same_prec_rel_l2": float(f"{rel_same:.3e}"),
           "history": hist}
    if found:
        res.update({"k": found["k"], "parareal_ms": found["ms"],
                    "worst_slice_rel_l2": float(f"{found['worst']:.3e}"),
                    "final_slice_rel_l2": float(f"{found['final']:.3e}"),
                    "stacked_rel_l2": float(f"{found['rel_l2']:.3e}"),
                    "per_slice_rel_l2_max_over_ics": per_slice,
                    "speedup_vs_serial_fp64": round(t_ser64 / found["ms"], 3),
                    "speedup_vs_serial_same_prec": round(t_ser / found["ms"], 3)})
    else:
        res.update({"k": None, "speedup_vs_serial_fp64": None,
                    "note": f"per-slice rel-L2 {target} not reached within {min(kmax, s)} iterations"})
    if stacked:
        res["stacked_criterion"] = {"k": stacked["k"], "parareal_ms": stacked["ms"],
                                    "rel_l2": stacked["rel_l2"],
                                    "speedup_vs_serial_fp64": round(t_ser64 / stacked["ms"], 3)}
    if p.f32_iters:
        res["f32_iters"] = p.f32_iters
    return res


def schedule_compare(api, p, g, u0, s, kmax, schedules=(1, 2)):
    """Parareal with FP64 fine solves from the start against the FP32-then-
    FP64 schedule, each at its smallest k whose worst slice reaches rel-L2
    1e-6."""
    import dataclasses
    out = {}
    for K in schedules:
        r = parareal_vs_serial(api, dataclasses.replace(p, f32_iters=K), g, u0, s, kmax)
        out[f"f32_iters_{K}"] = r
    return out


# The uneven batch (--config c5): 48 concurrent solves, the recipe fixed here (seeded, synthetic)
def c5_jobs(api, torch, synth, f32_iters, fine_prec="f64", g_prec="f64"):
    """Job i: N = (128, 256, 1024)[i % 3], slices = (16, 32, 64, 128, 256)[i % 5],
    eps = 0.01 + 0.02 i / 47, classic for even i and mass-conservative for
    odd i, S = 2, dt = 2e-5, 20 fine steps per slice, one IC (seed 5000 + i);
    G = one semi-implicit step of the slice length."""
    jobs = []
    for i in range(48):
        n = (128, 256, 1024)[i % 3]
        s = (16, 32, 64, 128, 256)[i % 5]
        eps = 0.01 + 0.02 * i / 47
        p = api.Problem(n=n, length=1.0, eps=eps, conservative=bool(i % 2), stab=2.0, dt=2e-5,
                        steps=20, fine_prec=fine_prec, f32_iters=f32_iters)
        u0 = torch.from_numpy(synth.random_ic(n, [5000 + i])).to("cuda")
        jobs.append(api.Job(p, api.Coarse(dt=20 * 2e-5, steps=1, prec=g_prec), u0, s, 5e-7))
    return jobs


def uneven_bench(args, reps=None, queue_compare=True):
    """The 48-solve uneven batch (c5) through pr_solve_many, FP64 plain
    form against the mixed form (FP32-then-FP64 fine schedule), each run
    until every job's sup-norm update is <= 5e-7, then checked against each
    job's FP64 serial fine solve (rel-L2 <= 1e-6 per job)."""
    import dataclasses
    import torch
    from paper_2510_07672_amd import api, synth
    ref_jobs = c5_jobs(api, torch, synth, 0)
    refs, t_ser = [], 0.0
    for j in ref_jobs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        refs.append(api.pr_serial_fine(j.problem, j.u0, j.n_slices))
        torch.cuda.synchronize()
        t_ser += time.perf_counter() - t0
    pts = sum(j.n_slices * j.problem.steps * j.problem.n ** 2 for j in ref_jobs)

    outs = {}

    def run(f32_iters, g_prec, reps, key=None):
        best, res = None, None
        for _ in range(reps):
            jobs = c5_jobs(api, torch, synth, f32_iters, g_prec=g_prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = api.pr_solve_many(jobs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best:
                best, res = dt, out
        if key is not None:
            outs[key] = [U for U, _ in res]
        errs = [float(torch.linalg.vector_norm(U - r) / torch.linalg.vector_norm(r))
                for (U, _), r in zip(res, refs)]
        iters = [int(st.iterations) for _, st in res]
        # the longest-running job took part in every iteration: its times
        # are the batch's fine and sweep times
        longest = max(res, key=lambda r: r[1].iterations)[1]
        fine_pts = sum(sum(max(0, j.n_slices - (k - 1)) for k in range(1, it + 1))
                       * j.problem.steps * j.problem.n ** 2
                       for j, it in zip(ref_jobs, iters))
        return {"ms": round(best * 1e3, 1), "max_rel_l2": float(f"{max(errs):.3e}"),
                "jobs_within_1e-6": sum(e <= 1e-6 for e in errs),
                "iterations_max": max(iters), "iterations_mean": round(float(np.mean(iters)), 2),
                "fine_gpts_per_s": round(fine_pts / best / 1e9, 1),
                "fine_ms": round(longest.fine_ms, 1), "sweep_ms": round(longest.sweep_ms, 1)}
    note(f"serial FP64 of 48 jobs: {t_ser * 1e3:.0f} ms")
    reps = args.steps if reps is None else reps
    plain = run(0, "f64", reps, key="pp")
    note(f"plain FP64 form: {plain['ms']} ms")
    queue = None
    if queue_compare:
        # the same solves with the fine sweep of each iteration as one
        # persistent work-queue launch per (N, precision) class
        was = api.pr_get_fine_queue()
        api.pr_set_fine_queue(1)
        try:
            queue = run(0, "f64", reps, key="q")
        finally:
            api.pr_set_fine_queue(was)
        queue["bitwise_equal_to_per_pass"] = all(
            bool(torch.equal(a, b)) for a, b in zip(outs["pp"], outs["q"]))
        note(f"plain FP64 form, work queue: {queue['ms']} ms")
    # G stays FP64: an FP32 coarse step puts ~1e-7 of rounding noise into
    # G(U^k) - G(U^{k-1}), which keeps the sup-norm update from settling
    mixed = {f"f32_iters_{K}": run(K, "f64", reps) for K in (1, 2)}
    best_k = min(mixed, key=lambda k: mixed[k]["ms"] if mixed[k]["jobs_within_1e-6"] == 48 else 1e12)
    best = mixed[best_k]
    return {"metric": "uneven batched Parareal: speedup of the mixed-precision form over the "
                      "FP64 plain form at rel-L2<=1e-6 (48 solves, one GPU)",
            "value": round(plain["ms"] / best["ms"], 3), "unit": "x", "n_gpus": 1,
            "steps": args.steps, "warmup": 0, "ms_per_step": best["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32 then f64", "data": "synthetic",
            "config": {"workload": "48 solves: N in {128, 256, 1024}, slices in {16..256}, "
                                   "eps 0.01..0.03, classic and conservative, dt 2e-5, 20 fine "
                                   "steps per slice, numerical G; all in one pr_solve_many"},
            "fine_point_steps_serial": pts, "serial_fp64_ms": round(t_ser * 1e3, 1),
            "plain_fp64": plain, "mixed": mixed, "best_mixed": best_k,
            "plain_fp64_work_queue": queue,
            "speedup_vs_serial_fp64": round(t_ser * 1e3 / best["ms"], 3)}


def copy_rates(sizes=(1 << 28, 1 << 30, 1 << 32), reps=5):
    """What a plain read-once write-once stream reaches on this GPU: torch's
    device copy at several sizes (events on the current stream, best of
    `reps`), in GB/s of bytes read plus bytes written."""
    import torch
    out = {}
    for nb in sizes:
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            y.copy_(x)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[f"{nb >> 20} MiB"] = round(2 * nb / (best * 1e-3) / 1e9, 1)
        del x, y
        torch.cuda.empty_cache()
    return {"copy_GB_per_s": out, "note": "torch copy_, bytes read + bytes written per second"}


def calib_copy(nbytes=1 << 30, reps=3):
    """A plain copy of `nbytes` bytes: reads nbytes and writes nbytes per
    launch, so HBM counters per dispatch can be scaled against it."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": nbytes, "reps": reps}), flush=True)


def trained_cnn(api, p, cfg, prec, steps, n_traj=512, n_slices=16, batch=32, loss="mse",
                lr_final=None, lr_drop=None, train_prec="bf16", lr=1e-3, init=None):
    """The workload's network, trained with Adam on fine-solver trajectories
    from seeds 1000.. (bf16 forward, FP32 gradients, 8-step rollouts
    checkpointed every 2), then evaluated in `prec`.  init: a stored network
    (save_weights) to continue from instead of the seed-0 initialisation."""
    from paper_2510_07672_amd import train
    L, C = cfg["cnn"]
    prior = None
    if init:
        g0, prior = load_weights(api, init, train_prec)
        if (g0.n_layers, g0.channels) != (L, C):
            raise SystemExit(f"{init} holds a {g0.n_layers} x {g0.channels} network, not {L} x {C}")
        net = g0
    else:
        net = train.init_network(L, C, seed=0, prec=train_prec)
    info = None
    if steps > 0 and loss == "scheme":
        # Algorithm 1: subsets of `batch` random ICs evolved by G itself, 4
        # updates per state on the residual of one coarse step
        import torch
        from paper_2510_07672_amd import synth
        dt_g = p.dt * p.steps
        n_states = max(1, steps // (4 * max(1, n_traj // batch)))
        u0 = torch.from_numpy(synth.random_ic(p.n, range(1000, 1000 + n_traj))).to("cuda")

        def progress(step, lv, ms):
            if step % 20 == 0:
                note(f"scheme-loss update {step} loss {lv:.3e} ({ms:.0f} ms)")
        log = train.train_scheme(net, p, u0, dt_g, n_steps=n_states, inner=4, subset=batch,
                                 lr=1e-3, progress=progress)
        info = {"loss": "scheme residual (eq. loss_ACN), one coarse step", "updates": len(log.loss),
                "trajectories": n_traj, "states_per_subset": n_states, "batch": batch,
                "loss_first": log.loss[0], "loss_last": log.loss[-1],
                "step_ms_median": round(sorted(log.step_ms)[len(log.step_ms) // 2], 2)}
    elif steps > 0:
        t0 = time.perf_counter()
        data = train.make_dataset(p, range(1000, 1000 + n_traj), n_slices)
        t_data = time.perf_counter() - t0
        note(f"training data: {n_traj} trajectories x {n_slices} slices in {t_data:.1f} s")

        def progress(step, loss, ms):
            if step % 10 == 0 or step == steps:
                note(f"train step {step}/{steps} loss {loss:.3e} ({ms:.0f} ms)")
        log = train.train(net, p, data, steps=steps, batch=batch, rollout=8, ckpt=2, lr=lr,
                          progress=progress, lr_final=lr_final, lr_drop=lr_drop)
        lr_txt = f"{lr:g}"
        if lr_final is not None:
            lr_txt = f"cosine {lr:g} -> {lr_final:g}"
        elif lr_drop:
            lr_txt = f"{lr:g}, then {lr / 10:g} for the last {lr_drop:g} of the steps"
        info = {"steps": steps, "lr": lr_txt, "forward_prec": train_prec,
                "trajectories": n_traj, "slices_per_trajectory": n_slices,
                "batch": batch,
                "data_s": round(t_data, 2), "loss_first": log.loss[0], "loss_last": log.loss[-1],
                "step_ms_median": round(sorted(log.step_ms)[len(log.step_ms) // 2], 2)}
        if prior is not None:
            # continued from a stored network: its record, and the total
            info["continued_from"] = {k: prior.get(k) for k in ("stored", "command", "steps", "lr",
                                                                "loss_last")}
            info["steps"] = steps + int(prior.get("steps", 0))
            info["steps_this_run"] = steps
        del data
    lay = net.layers()
    ws = [w.detach().float().cpu() for w, _ in lay]
    bs = [b.detach().float().cpu() for _, b in lay]
    return api.CnnCoarse(ws, bs, act="gelu", residual=True, prec=prec), info


WEIGHTS_DIR = os.path.join(ROOT, "paper_2510_07672_amd", "weights")


def save_weights(path, g, info, cname, cfg):
    """The workload's trained network as a plain .npz (FP32 arrays and a
    JSON string: no pickles), with the recipe and the command that made it."""
    import numpy as np
    arrays = {}
    for l, (w, b) in enumerate(g.layers()):
        arrays[f"w{l}"] = w.detach().float().cpu().numpy()
        arrays[f"b{l}"] = b.detach().float().cpu().numpy()
    meta = {"workload": cname, "cnn": list(cfg["cnn"]), "training": info,
            "command": "python bench.py " + " ".join(sys.argv[1:])}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, meta=np.array(json.dumps(meta)), **arrays)
    note(f"weights saved to {path}")


def load_weights(api, path, prec):
    """A network stored by save_weights, evaluated in `prec`, and its
    training record (recipe, command, file)."""
    import numpy as np
    import torch
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        L = meta["cnn"][0]
        ws = [torch.from_numpy(z[f"w{l}"].copy()) for l in range(L)]
        bs = [torch.from_numpy(z[f"b{l}"].copy()) for l in range(L)]
    info = dict(meta.get("training") or {})
    info["stored"] = os.path.relpath(path, ROOT)
    info["command"] = meta.get("command")
    return api.CnnCoarse(ws, bs, act="gelu", residual=True, prec=prec), info


def training_bench(args):
    """Training (c4): one step = an 8-step rollout of the network on a
    batch of 32 trajectories at 256^2 (bf16 forward, FP32 gradients,
    checkpoints every 2 steps), the MSE against fine-solver states, the
    backward through the hand-written kernels and an Adam update."""
    import torch
    from paper_2510_07672_amd import api, train
    n = 256
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=False, stab=2.0, dt=2e-5, steps=200)
    data = train.make_dataset(p, range(2000, 2032), 16)
    net = train.init_network(4, 32, seed=0, prec="bf16")
    train.train(net, p, data, steps=args.warmup, batch=32)
    log = train.train(net, p, data, steps=args.steps, batch=32, seed=1)
    ms = float(np.median(log.step_ms))
    # network applications per step: 8 forward + 8 recomputed in backward
    # (inside pr_cnn_backward) + 4 segment recomputations
    apps = 32 * (8 + 8 + 4)
    return {"metric": "CNN coarse-propagator training steps/s (8-step rollout, batch 32, 256^2)",
            "value": round(1e3 / ms, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16 forward, f32 grads",
            "data": "synthetic",
            "config": {"workload": "training: 8-step unrolled rollout, batch 32 trajectories, "
                                   "256x256 classic AC, 4 conv x 32 ch GELU, MSE vs fine states, "
                                   "checkpoint every 2 steps"},
            "network_applications_per_s": round(apps / ms * 1e3, 1),
            "loss_first": log.loss[0], "loss_last": log.loss[-1]}


def tune_network(api, p, g, u0, args):
    """Untimed set-up: pr_autotune_coarse times the network's plans and
    hidden-layer tiles on the batch and keeps the fastest as the AUTO
    choice, which every later call (the timed ones included) then takes.
    --cnn-plan / --cnn-tile pin them instead."""
    if args.cnn_plan or args.cnn_tile:
        if args.cnn_plan:
            api.pr_set_coarse_plan(args.cnn_plan)
        if args.cnn_tile:
            api.pr_set_coarse_tile(args.cnn_tile)
        how = "pinned"
    else:
        api.pr_autotune_coarse(p, g, u0)
        how = "pr_autotune_coarse"
    return {"plan": api.pr_get_coarse_plan(g, p.n), "tile": api.pr_get_coarse_tile(g, p.n),
            "chosen_by": how}


def cnn_kernel_rate(api, p, g, u0, reps=20):
    """Average duration of one network application on the batch (torch
    events on the stream the library launches on) and its rate against the
    bf16 matrix-core peak.  The network's own work is 2 * 9 * sum_l
    C_in C_out flops per pixel (first, hidden and last layers); the split
    form issues the hidden layers' products twice (hi and lo), which is
    reported separately as the issued matrix-core rate, not as work."""
    import torch
    out = torch.empty_like(u0)
    api.pr_coarse_apply(p, g, u0, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        api.pr_coarse_apply(p, g, u0, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    B, n = u0.shape[0], u0.shape[-1]
    L, C = g.n_layers, g.channels
    px = B * n * n
    model_flops = 2 * 9 * (C + C * C * (L - 2) + C) * px
    issued = 2 * 9 * C * C * (L - 2) * px * (2 if g.prec == "bf16x2" else 1)
    peak = {"bf16": 2500.0, "bf16x2": 2500.0, "f32": 157.3, "f64": 78.6}[g.prec]
    return {"ms_per_call": round(ms, 4), "fields": B, "layers": L, "channels": C, "prec": g.prec,
            "flops_per_px": 2 * 9 * (C + C * C * (L - 2) + C),
            "model_tflops": round(model_flops / ms / 1e9, 1), "peak_tflops": peak,
            "mfma_frac": round(model_flops / ms / 1e9 / peak, 4),
            "issued_mfma_tflops": round(issued / ms / 1e9, 1),
            "algorithmic_bytes_per_call": network_bytes(B, n, L, C, g.prec),
            "algorithmic_GB_per_s": round(network_bytes(B, n, L, C, g.prec) / ms / 1e6, 1),
            "hbm_frac": round(network_bytes(B, n, L, C, g.prec) / ms / 1e6 / HBM_PEAK_GBS, 4)}


def dram_traffic(cfg_name, prec, n, nfields):
    """DRAM-addressed bytes of one fine step over `nfields` fields, from the
    committed TCC_EA0_RDREQ_DRAM / TCC_EA0_WRREQ_DRAM counter summary
    (requests scaled to bytes by a plain copy of known size).  These
    requests leave the L2 for the memory side; the last-level (MALL) cache
    there serves part of them, so they bound the HBM bytes from above.
    None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"fine_step_{cfg_name}_{prec}_dram.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("src_hash") != kernel_src_hash():
        return None
    return d["bytes_per_field_step"] * nfields


def fine_rate(api, p, u0, steps, working_set=None):
    """Streaming fine steps on the fields of u0 (one pr_fine_propagate call of
    `steps` steps, HIP events on its stream): algorithmic GB/s."""
    import dataclasses
    import torch
    q = dataclasses.replace(p, steps=steps)
    old = None
    if working_set is not None:
        old = api.pr_get_fine_working_set(p.n, p.fine_prec)
        api.pr_set_fine_working_set(working_set)
    try:
        import ctypes
        from paper_2510_07672_amd import _lib as L
        out = torch.empty_like(u0)
        ws = api.workspace(L.lib().pr_fine_workspace_bytes(ctypes.byref(q.c()), u0.shape[0]),
                           u0.device)
        api.pr_fine_propagate(q, u0, out=out, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.pr_fine_propagate(q, u0, out=out, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
    finally:
        if old is not None:
            api.pr_set_fine_working_set(old)
    del out, ws
    bpp = bytes_per_point_step(p.fine_prec, p.scheme, p.picard)
    gbs = u0.shape[0] * p.n * p.n * steps * bpp / (ms * 1e-3) / 1e9
    return {"fields": u0.shape[0], "steps": steps, "ms": round(ms, 3), "GB/s": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def fp32_fine_section(api, torch, p, g, u0, s, k=6, steps=3):
    """The workload with the FP32 fine step the workload text names: the
    timed Parareal iteration with FP32 fine solves (16 B per point and
    step), and what an FP32 fine state does to the accuracy: the serial
    FP32 fine solve and Parareal with FP32 F after k iterations, each
    against the FP64 serial fine solve, worst slice over the ICs."""
    import dataclasses
    p32 = dataclasses.replace(p, fine_prec="f32", f32_iters=0)
    p64 = dataclasses.replace(p, fine_prec="f64", f32_iters=0)
    B, n, c = u0.shape[0], p.n, p.steps
    U = torch.empty((B, s + 1, n, n), dtype=torch.float64, device="cuda")

    def one(max_iter):
        return api.pr_solve(p32, g, u0, s, tol=0.0, max_iter=max_iter, U=U, allow_not_converged=True)
    one(1)
    torch.cuda.synchronize()
    fine = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = one(1)
        fine.append(st.fine_ms)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    pts = B * s * c * n * n
    fine_ms = float(np.mean(fine))
    ref = api.pr_serial_fine(p64, u0, s)
    ref_slice = torch.linalg.vector_norm(ref, dim=(-2, -1))

    def worst(V):
        return float((torch.linalg.vector_norm(V - ref, dim=(-2, -1)) / ref_slice).max())
    ser32 = worst(api.pr_serial_fine(p32, u0, s))
    one(k)
    par32 = worst(U)
    del U, ref
    gbs = pts * 16 / (fine_ms * 1e-3) / 1e9
    note(f"FP32 fine step: {ms:.1f} ms per iteration, fine sweep {gbs:.1f} GB/s; serial FP32 "
         f"{ser32:.2e}, Parareal k={k} {par32:.2e} from the FP64 serial solve (worst slice)")
    return {"value": round(pts / (ms * 1e-3) / 1e9, 2), "unit": "Gpts/s", "ms_per_step": round(ms, 3),
            "fine_prec": "f32", "fine_sweep_ms": round(fine_ms, 3),
            "fine_GB_per_s": round(gbs, 1), "fine_frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_point_step": 16,
            "serial_fp32_worst_slice_rel_l2": float(f"{ser32:.3e}"),
            f"parareal_k{k}_worst_slice_rel_l2": float(f"{par32:.3e}"),
            "note": "an FP32 fine state drifts from the FP64 serial fine solve by the FP32 "
                    "transforms' rounding, step after step: neither the serial FP32 solve nor "
                    "Parareal with FP32 F meets rel-L2 1e-6; the precision schedule (FP32 first "
                    "iterations, then FP64) does, see parareal_schedule"}


def network_bytes(B, n, L, C, prec):
    """HBM bytes one call of the folded network plan moves at least: the
    first hidden layer reads the FP64 state and writes its activations,
    each further hidden layer reads and writes activations (hi + lo
    bfloat16 in the split form), the last hidden layer writes nine FP32
    per-tap products instead, and the gather reads those and the state and
    writes G(u) in FP64 (halo re-reads not counted)."""
    px = B * n * n
    act = C * (4 if prec == "bf16x2" else 2)
    return px * (8 + act + 2 * act * (L - 4) + act + 36 + 36 + 8 + 8)


def network_only(args, api, torch, synth):
    """The workload's network G alone: per-call time, model flop rate and
    the folded plan's algorithmic HBM rate."""
    cfg = CONFIGS[args.config]
    n, B = cfg["n"], cfg["ics"]
    p = api.Problem(n=n, length=1.0, eps=cfg["eps"], conservative=cfg["conservative"], stab=2.0,
                    dt=cfg["dt"], steps=cfg["steps"])
    g, _ = trained_cnn(api, p, cfg, args.cnn_prec, 0)
    u0 = torch.from_numpy(synth.random_ic(n, range(cfg["seed0"], cfg["seed0"] + B))).to("cuda")
    tuned = tune_network(api, p, g, u0, args)
    ck = cnn_kernel_rate(api, p, g, u0, reps=10 * args.steps)
    ck.update(tuned)
    ck["workload"] = cfg["workload"]
    return ck


def _event_ms(torch, fn, reps, trials=3):
    """Best of `trials` mean durations of fn() over `reps` calls (events on
    torch's current stream, which the library launches on)."""
    fn()
    torch.cuda.synchronize()
    best = None
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        best = ms if best is None else min(best, ms)
    return best


def tile_sweep(args, api, torch, synth):
    """The network's inference plans under each hidden-layer tile, per call,
    on the workloads' shapes and a few others (seed-0 weights), and what
    pr_autotune_coarse picks; the settings are restored to 'auto'."""
    import ctypes
    from paper_2510_07672_amd import _lib as Lb
    from paper_2510_07672_amd import train
    shapes = [(512, 6, 48, "bf16x2", 16), (512, 6, 48, "bf16", 16), (1024, 6, 48, "bf16x2", 4),
              (64, 6, 48, "bf16x2", 16), (256, 4, 32, "bf16x2", 8), (256, 4, 32, "bf16x2", 64),
              (128, 4, 32, "bf16x2", 32)]
    rows = []
    for n, L, C, prec, nf in shapes:
        g = train.init_network(L, C, seed=1, prec=prec)
        p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=1e-5, steps=10)
        u = torch.from_numpy(synth.random_ic(n, range(nf))).to("cuda")
        out = torch.empty_like(u)
        wsb = api.workspace(Lb.lib().pr_coarse_workspace_bytes(ctypes.byref(p.c()),
                                                                ctypes.byref(g.c()), nf), "cuda")
        ms = {}
        try:
            for plan in ("layered", "folded"):
                for tile in ("8x32", "16x16"):
                    api.pr_set_coarse_plan(plan)
                    api.pr_set_coarse_tile(tile)
                    ms[f"{plan}/{tile}"] = round(_event_ms(
                        torch, lambda: api.pr_coarse_apply(p, g, u, out=out, ws=wsb), 40), 4)
        finally:
            api.pr_set_coarse_plan("auto")
            api.pr_set_coarse_tile("auto")
        chosen = api.pr_autotune_coarse(p, g, u)
        rows.append({"n": n, "layers": L, "channels": C, "prec": prec, "fields": nf,
                     "ms_per_call": ms, "autotune": f"{chosen}/{api.pr_get_coarse_tile(g, n)}"})
        note(f"tile sweep {n}^2 {L}x{C} {prec} x{nf}: {ms} -> {rows[-1]['autotune']}")
    return {"sweep": "network plan x hidden-layer tile", "rows": rows}


def split_sweep(args, api, torch, synth):
    """The streaming semi-implicit fine step under both FFT radix splits
    where they differ (N = 128, 1024), per step, with its algorithmic HBM
    rate; the settings are restored to 'auto'."""
    import ctypes
    from paper_2510_07672_amd import _lib as Lb
    cases = [(1024, "f64", 32, 20), (1024, "f64", 256, 10), (1024, "f32", 32, 20),
             (1024, "f32", 256, 10), (128, "f64", 512, 50), (128, "f64", 4096, 20),
             (128, "f32", 1024, 50)]
    rows = []
    for n, prec, nf, steps in cases:
        p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5,
                        steps=steps, fine_prec=prec)
        u = torch.from_numpy(synth.random_ic(n, range(nf))).to("cuda")
        wsb = api.workspace(Lb.lib().pr_fine_workspace_bytes(ctypes.byref(p.c()), nf), "cuda")
        out = torch.empty_like(u)
        bpp = 32 if prec == "f64" else 16
        us, gbs = {}, {}
        try:
            api.pr_set_fine_plan(n, prec, "stream")
            for split in ("r8", "r4_tail"):
                api.pr_set_fft_split(n, prec, split)
                t = _event_ms(torch, lambda: api.pr_fine_propagate(p, u, out=out, ws=wsb), 3)
                us[split] = round(t * 1e3 / steps, 2)
                gbs[split] = round(bpp * nf * n * n / (t * 1e-3 / steps) / 1e9, 1)
        finally:
            api.pr_set_fft_split(n, prec, "auto")
            api.pr_set_fine_plan(n, prec, "auto")
        rows.append({"n": n, "prec": prec, "fields": nf, "us_per_step": us, "GB_per_s": gbs})
        note(f"split sweep {n}^2 {prec} x{nf}: {us}")
    return {"sweep": "FFT radix split of the streaming semi-implicit step", "rows": rows}


def size_sweep(args, api, torch, synth):
    """The fine step (semi-implicit, streaming plan, default working-set
    chunking and radix split) per step at the workloads' grid sizes and
    batches, FP64 and FP32, with its algorithmic HBM rate."""
    import ctypes
    from paper_2510_07672_amd import _lib as Lb
    cases = [(256, 512, 200), (512, 2048, 100), (1024, 256, 20)]
    rows = []
    for n, nf, steps in cases:
        for prec in ("f64", "f32"):
            p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5,
                            steps=steps, fine_prec=prec)
            u = torch.from_numpy(synth.random_ic(n, range(nf))).to("cuda")
            wsb = api.workspace(Lb.lib().pr_fine_workspace_bytes(ctypes.byref(p.c()), nf), "cuda")
            out = torch.empty_like(u)
            t = _event_ms(torch, lambda: api.pr_fine_propagate(p, u, out=out, ws=wsb), 3)
            bpp = 32 if prec == "f64" else 16
            gbs = bpp * nf * n * n / (t * 1e-3 / steps) / 1e9
            rows.append({"n": n, "fields": nf, "prec": prec, "us_per_step": round(t * 1e3 / steps, 1),
                         "GB_per_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
            note(f"size sweep {n}^2 x{nf} {prec}: {rows[-1]['us_per_step']} us/step, {gbs:.0f} GB/s")
            del u, out, wsb
    return {"sweep": "fine step by grid size", "rows": rows}


def run_config(args, cname, api, torch, synth, full=True):
    """The timed step and its sections for workload `cname` (c1, c2, c3)."""
    cfg = CONFIGS[cname]
    n, s, B, c = cfg["n"], cfg["slices"], cfg["ics"], cfg["steps"]
    p = api.Problem(n=n, length=1.0, eps=cfg["eps"], conservative=cfg["conservative"], stab=2.0,
                    dt=cfg["dt"], steps=c, fine_prec=args.prec, scheme=args.scheme,
                    picard=args.picard)
    coarse = args.coarse or ("num" if cname == "c1" else "cnn")
    g_num = api.Coarse(dt=cfg["dt"] * c / cfg["g_steps"], steps=cfg["g_steps"], prec="f64")
    train_info = None
    if coarse == "cnn":
        # the network stored for the workload (paper_2510_07672_amd/weights,
        # made by this script with --save-weights), unless training is asked for
        stored = os.path.join(WEIGHTS_DIR, f"{cname}.npz")
        asked = full and (args.train_steps is not None or args.train_loss != "mse")
        if os.path.exists(stored) and not asked and not args.no_stored_weights:
            g, train_info = load_weights(api, stored, args.cnn_prec)
            note(f"{cname}: network loaded from {train_info['stored']}")
        else:
            steps = cfg.get("train_steps", 0) if (args.train_steps is None or not full) else args.train_steps
            n_traj = cfg.get("train_traj", 128) if (args.train_traj is None or not full) else args.train_traj
            g, train_info = trained_cnn(api, p, cfg, args.cnn_prec, steps,
                                        n_traj=n_traj, batch=args.train_batch,
                                        loss=args.train_loss, lr_final=args.train_lr_final,
                                        lr_drop=cfg.get("train_lr_drop") if args.train_lr_drop is None
                                        else args.train_lr_drop, train_prec=args.train_prec,
                                        lr=args.train_lr, init=args.init_weights if full else None)
            if full and args.save_weights:
                save_weights(args.save_weights, g, train_info, cname, cfg)
    else:
        g = g_num
    u0 = torch.from_numpy(synth.random_ic(n, range(cfg["seed0"], cfg["seed0"] + B))).to("cuda")
    tuned = tune_network(api, p, g, u0, args) if coarse == "cnn" else None
    U = torch.empty((B, s + 1, n, n), dtype=torch.float64, device="cuda")
    ws = None

    def one():
        return api.pr_solve(p, g, u0, s, tol=0.0, max_iter=1, U=U, ws=ws, allow_not_converged=True)

    _, st = one()
    note(f"{cname}: first step done")
    import ctypes
    from paper_2510_07672_amd import _lib as L
    need = L.lib().pr_solve_workspace_bytes(ctypes.byref(p.c()), ctypes.byref(g.c()), B, s)
    ws = api.workspace(need, "cuda")
    steps_t = args.steps if full else max(1, min(args.steps, 3))
    for _ in range(args.warmup if full else 1):
        one()
    torch.cuda.synchronize()
    fine_ms, sweep_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps_t):
        _, st = one()
        fine_ms.append(st.fine_ms)
        sweep_ms.append(st.sweep_ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps_t
    pts = B * s * c * n * n
    value = pts / (ms_per_step * 1e-3) / 1e9
    del U, ws

    fine_ms_avg = float(np.mean(fine_ms))
    bpp = bytes_per_point_step(args.prec, args.scheme, args.picard)
    achieved = pts * bpp / (fine_ms_avg * 1e-3) / 1e9
    traffic = measured_traffic(cname, args.prec, n, B * s) if args.scheme == "ssi" else None
    dram = dram_traffic(cname, args.prec, n, B * s) if args.scheme == "ssi" else None
    step_alg_bytes = B * s * n * n * bpp
    fine_time_s = fine_ms_avg * 1e-3 / c   # per fine step over the batch
    roof_fine = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None if traffic is None else round(traffic),
        "traffic_unit": "bytes per fine step over the batch (row + column pass), FETCH_SIZE + "
                        "WRITE_SIZE scaled by a plain copy",
        "traffic_dram": None if dram is None else round(dram),
        "traffic_dram_note": "requests leaving L2 for DRAM addresses (TCC_EA0_RDREQ_DRAM + "
                             "WRREQ_DRAM, scaled by a plain copy); the MALL serves part of them",
        "dram_frac": None if dram is None else round(dram / fine_time_s / 1e9 / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": step_alg_bytes,
        "kernel": ("fine step = k_col + k_row<MID> per step, over the whole F sweep"
                   if args.scheme == "ssi" else
                   f"fine step = {args.picard} x (k_col_cn + k_row<MID, f(v)>), over the F sweep"),
        "bytes_per_point_step": bpp,
        "fine_sweep_ms": round(fine_ms_avg, 3), "sweep_ms": round(float(np.mean(sweep_ms)), 3)}
    if full and args.scheme == "ssi" and not args.no_mall:
        # the same fine sweep with no working-set chunking: every pass streams
        # all B s fields, far beyond the 256 MB MALL, so (nearly) every byte
        # comes from HBM
        uu = u0.repeat(s, 1, 1).contiguous()
        chunked = fine_rate(api, p, uu, 10)
        beyond = fine_rate(api, p, uu, 10, working_set=0)
        roof_fine["chunked_10_steps"] = chunked
        roof_fine["beyond_mall"] = dict(beyond, working_set="off (one chunk of all fields)")
        note(f"{cname}: fine step chunked {chunked['GB/s']} GB/s, unchunked {beyond['GB/s']} GB/s")
        if args.prec == "f64":
            # the FP32 fine step (16 B per point and step) on the same fields,
            # the precision of the schedule's first iterations
            import dataclasses
            p32 = dataclasses.replace(p, fine_prec="f32")
            roof_fine["f32_step"] = {"chunked_10_steps": fine_rate(api, p32, uu, 10),
                                     "beyond_mall": fine_rate(api, p32, uu, 10, working_set=0)}
        del uu
    out = {
        "value": round(value, 2), "unit": "Gpts/s", "ms_per_step": round(ms_per_step, 3),
        "steps": steps_t,
        "config": {"workload": cfg["workload"] + ("" if args.scheme == "ssi" else
                                                  f"; fine scheme CN + {args.picard} Picard iterations"),
                   "n": n, "ics": B, "slices": s, "fine_steps": c,
                   "fine_solves_per_launch": B * s, "fine_prec": args.prec, "scheme": args.scheme,
                   "overlap_chunks": args.overlap},
        "roofline_fine": roof_fine,
    }
    roof = roof_fine
    if coarse == "cnn":
        ck = cnn_kernel_rate(api, p, g, u0)
        ck.update(tuned)
        out["coarse_kernel"] = ck
        # one network call per slice in the initial sweep and one in the
        # correction sweep of the iteration
        coarse_ms = 2 * s * ck["ms_per_call"]
        # the network's arithmetic intensity (model flops over the folded
        # plan's HBM bytes, ~130 flop/B at 6 x 48 split) is below the bf16
        # ridge point (2500 TFLOP/s / 8 TB/s = 312 flop/B): its roofline is
        # HBM; the matrix-core rate is reported beside it
        nt = network_traffic(cname)
        roof_coarse = {"bound": "hbm", "achieved": ck["algorithmic_GB_per_s"], "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": ck["hbm_frac"],
                       "traffic": None if nt is None else round(nt),
                       "traffic_unit": "bytes per call, FETCH_SIZE + WRITE_SIZE scaled by a plain copy",
                       "algorithmic_bytes_per_call": ck["algorithmic_bytes_per_call"],
                       "kernel": f"network G call ({g.n_layers} conv x {g.channels} ch, {g.prec}; "
                                 f"{ck['plan']} plan, {ck['tile']} tiles) on {B} fields, per call",
                       "mfma": {"achieved": ck["model_tflops"], "peak": ck["peak_tflops"],
                                "unit": "TFLOP/s", "frac": ck["mfma_frac"],
                                "flops_per_call": ck["flops_per_px"] * B * n * n,
                                "issued_tflops": ck["issued_mfma_tflops"]},
                       "ms_per_call": ck["ms_per_call"], "calls_per_step": 2 * s,
                       "ms_per_step": round(coarse_ms, 2)}
        out["roofline_coarse"] = roof_coarse
        if coarse_ms > fine_ms_avg:
            roof = roof_coarse
        out["config"]["coarse"] = (f"u + CNN(u), {g.n_layers} conv layers x {g.channels} ch, GELU, "
                                   f"{g.prec}; " + (("trained on the scheme residual"
                                   if train_info.get("loss") else
                                   f"trained {train_info['steps']} Adam steps on "
                                   f"{train_info['trajectories']} fine trajectories")
                                   if train_info else "seed-0 weights, untrained"))
        if train_info:
            out["training"] = train_info
    else:
        out["config"]["coarse"] = "numerical: one semi-implicit step per slice"
    out["roofline"] = dict(roof, dominant="network G" if roof is not roof_fine else "fine step F",
                           note="the component with the larger share of the timed step: fine "
                                "sweep %.1f ms vs network calls %.1f ms" % (
                                    fine_ms_avg, out.get("roofline_coarse", {}).get("ms_per_step", 0.0)))
    if not args.no_parareal:
        out["parareal"] = parareal_vs_serial(api, p, g, u0, s, args.kmax)
        if args.prec == "f64" and full:
            out["parareal_schedule"] = schedule_compare(api, p, g, u0, s, args.kmax,
                                                        schedules=(1,) if cname == "c3" else (1, 2))
        if coarse == "cnn":
            out["parareal_numerical_coarse"] = parareal_vs_serial(api, p, g_num, u0, s, args.kmax)
    if not args.no_cpu and full:
        out["cpu_baseline"] = cpu_baseline(cfg, args.prec)
    if full and args.prec == "f64" and not args.no_extra:
        out["fp32_fine"] = fp32_fine_section(api, torch, p, g, u0, s)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS) + ["c4", "c5"],
                    help="workload of the headline line (default c3, the largest; the c2 "
                         "figures follow under the key config2 unless --no-extra)")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--scheme", default="ssi", choices=["ssi", "cn"],
                    help="fine scheme: the semi-implicit step the workloads fix, or the paper's "
                         "Crank-Nicolson + Picard")
    ap.add_argument("--picard", type=int, default=2, help="Picard iterations per CN step")
    ap.add_argument("--overlap", type=int, default=1,
                    help="fine-batch chunks overlapped with the sequential sweep (1 = none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-parareal", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 256^2 section (key config2) and the uneven batch (key uneven_batch)")
    ap.add_argument("--no-mall", action="store_true",
                    help="skip the fine-step rates with and without working-set chunking")
    ap.add_argument("--kmax", type=int, default=16)
    ap.add_argument("--coarse", default=None, choices=["num", "cnn"],
                    help="numerical coarse step, or the workload's convolutional network "
                         "(default: the network for c2 and c3, the scheme for c1)")
    ap.add_argument("--cnn-prec", default="bf16x2", choices=["bf16", "bf16x2", "f32"])
    ap.add_argument("--cnn-plan", default=None, choices=["layered", "fused", "folded"],
                    help="pin the network plan and hidden-layer tile (with --cnn-tile) "
                         "instead of running pr_autotune_coarse before the timed region; "
                         "a counter run pins the autotuner's choice so that it sees only "
                         "those kernels")
    ap.add_argument("--cnn-tile", default=None, choices=["8x32", "16x16"])
    ap.add_argument("--train-steps", type=int, default=None,
                    help="Adam steps on fine trajectories before timing (network only); "
                         "default 2000 for c2 and 60 for c3")
    ap.add_argument("--save-weights", default=None,
                    help="store the network trained in this run (.npz) for later runs")
    ap.add_argument("--init-weights", default=None,
                    help="continue training from this stored network (.npz) instead of the "
                         "seed-0 initialisation")
    ap.add_argument("--train-lr", type=float, default=1e-3, help="Adam learning rate (start)")
    ap.add_argument("--no-stored-weights", action="store_true",
                    help="train at run time even where paper_2510_07672_amd/weights holds "
                         "the workload's network")
    ap.add_argument("--train-traj", type=int, default=None,
                    help="fine trajectories (16 slices each) the network is trained on "
                         "(default 512 for c2, 128 for c3)")
    ap.add_argument("--train-batch", type=int, default=32)
    ap.add_argument("--train-lr-final", type=float, default=None,
                    help="cosine learning-rate decay from 1e-3 to this value over the run")
    ap.add_argument("--train-lr-drop", type=float, default=None,
                    help="fraction of the training steps, at the end, run at a tenth of the "
                         "learning rate")
    ap.add_argument("--train-prec", default="bf16", choices=["bf16", "bf16x2"],
                    help="network precision of the training forward passes")
    ap.add_argument("--train-loss", default="mse", choices=["mse", "scheme"],
                    help="mse against fine trajectories, or the scheme-residual loss of "
                         "Algorithm 1 over one coarse step")
    ap.add_argument("--fine-queue", action="store_true",
                    help="run the fine solves as one persistent work-queue launch per size and "
                         "precision class (pr_set_fine_queue)")
    ap.add_argument("--working-set", type=int, default=None,
                    help="working-set budget in bytes of chunked streaming fine calls "
                         "(0 = one chunk, every field through each step in turn)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--tile-sweep", action="store_true",
                    help="time the network's plans under each hidden-layer tile on several "
                         "shapes, and the autotuner's choice (one JSON line)")
    ap.add_argument("--split-sweep", action="store_true",
                    help="time the fine step under both FFT radix splits where they differ "
                         "(one JSON line)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="time the fine step at 256^2, 512^2 and 1024^2, FP64 and FP32 (one JSON line)")
    ap.add_argument("--network-only", action="store_true",
                    help="time only the network G of the workload (seed-0 weights, --steps x 10 "
                         "calls) and print its per-call figures")
    ap.add_argument("--copy-rate", action="store_true",
                    help="only time plain device copies of 256 MiB, 1 GiB and 4 GiB")
    args = ap.parse_args()
    if args.calib_copy:
        calib_copy()
        return
    if args.copy_rate:
        print(json.dumps(copy_rates()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (its fine "
              "solves would shard by slice with no communication, the correction sweep passing "
              "one state per GPU boundary)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_07672_amd import api, synth
    api.pr_set_overlap(args.overlap)
    if args.working_set is not None:
        api.pr_set_fine_working_set(args.working_set)
    if args.fine_queue:
        api.pr_set_fine_queue(True)

    if args.config == "c4":
        print(json.dumps(training_bench(args)), flush=True)
        return
    if args.network_only:
        print(json.dumps(network_only(args, api, torch, synth)), flush=True)
        return
    if args.tile_sweep:
        print(json.dumps(tile_sweep(args, api, torch, synth)), flush=True)
        return
    if args.split_sweep:
        print(json.dumps(split_sweep(args, api, torch, synth)), flush=True)
        return
    if args.size_sweep:
        print(json.dumps(size_sweep(args, api, torch, synth)), flush=True)
        return
    if args.config == "c5":
        print(json.dumps(uneven_bench(args)), flush=True)
        return
    res = run_config(args, args.config, api, torch, synth, full=True)
    out = {
        "metric": "Parareal speedup vs serial fine at rel-L2<=1e-6; fine-step Gpts/s; %HBM roofline",
        "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
        "steps": res.pop("steps"), "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic", "config": res.pop("config"), "roofline": res.pop("roofline"),
    }
    cpu = res.pop("cpu_baseline", None)
    out.update(res)
    if args.config == "c3" and not args.no_extra:
        torch.cuda.empty_cache()
        note("256^2 section")
        c2 = run_config(args, "c2", api, torch, synth, full=False)
        out["config2"] = c2
        torch.cuda.empty_cache()
        note("uneven batch section")
        ub = uneven_bench(args, reps=2)
        out["uneven_batch"] = {k: ub[k] for k in (
            "metric", "value", "unit", "config", "serial_fp64_ms", "plain_fp64", "mixed",
            "best_mixed", "plain_fp64_work_queue", "speedup_vs_serial_fp64")}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
