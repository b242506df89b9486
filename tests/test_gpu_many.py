"""GPU checks of the uneven batched driver (pr_solve_many) and of the
FP32-then-FP64 precision schedule of Algorithm 2 (Section 3.3).

  * A heterogeneous batch gives every job the bits it gets alone through
    pr_solve: fields of jobs with different eps, dt, S, model and slice
    counts share launches only through per-field parameters, which must
    not change any value.
  * Each FP64 job matches the oracle's Algorithm 2 (same iteration counts,
    rel-L2 <= 1e-12).
  * Schedule: the FP32 iterations never freeze an IC; after f32_iters + s
    iterations the result is the FP64 serial fine solve bit for bit, and
    after f32_iters + k the first k slices are; converged results sit as
    close to the FP64 serial solve as plain Parareal's.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import allen_cahn as ac  # noqa: E402
from paper_2510_07672_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2510_07672_amd import api as A
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_problem(p):
    return ac.Problem(n=p.n, length=p.length, eps=p.eps, conservative=p.conservative,
                      stab=p.stab, dt=p.dt, steps=p.steps)


def mixed_jobs(api, tol=1e-9):
    """Five jobs: two N, both models, different eps / dt / steps / slices /
    IC counts; jobs 0 and 1 share (N, precision, steps) and so one launch."""
    spec = [  # n, eps, cons, dt, steps, slices, seeds, g_dt
        (32, 0.04, False, 1e-3, 10, 6, [1, 2], 1e-2),
        (32, 0.03, True, 5e-4, 10, 9, [3], 5e-3),
        (64, 0.02, False, 1e-4, 20, 4, [4, 5, 6], 2e-3),
        (32, 0.05, True, 1e-3, 7, 3, [7], 7e-3),
        (64, 0.025, True, 2e-4, 20, 7, [8, 9], 4e-3),
    ]
    jobs = []
    for n, eps, cons, dt, steps, s, seeds, gdt in spec:
        p = api.Problem(n=n, length=1.0, eps=eps, conservative=cons, stab=2.0, dt=dt, steps=steps)
        jobs.append(api.Job(p, api.Coarse(dt=gdt, steps=1), dev(synth.random_ic(n, seeds)), s, tol))
    return jobs


def test_many_equals_each_alone_and_oracle(api):
    jobs = mixed_jobs(api)
    out = api.pr_solve_many(jobs)
    for j, (U, st) in zip(jobs, out):
        print(f"case job n={j.problem.n} eps={j.problem.eps} s={j.n_slices}", flush=True)
        U1, st1 = api.pr_solve(j.problem, j.coarse, j.u0, j.n_slices, tol=j.tol)
        assert torch.equal(U, U1)
        assert list(st.ic_iterations) == list(st1.ic_iterations)
        assert st.status == 0
        u0 = j.u0.cpu().numpy()
        op = oracle_problem(j.problem)
        res = ac.parareal(u0, op, j.n_slices, tol=j.tol,
                          G=lambda u, p=op, g=j.coarse: ac.coarse_num(u, p, ac.Coarse(g.dt, g.steps)))
        assert list(st.ic_iterations) == list(res.iterations)
        assert rel(U.cpu().numpy(), res.U) <= 1e-12


def test_many_order_and_empty_jobs(api):
    jobs = mixed_jobs(api)
    out = api.pr_solve_many(jobs)
    rev = [api.Job(j.problem, j.coarse, j.u0, j.n_slices, j.tol) for j in jobs[::-1]]
    out_r = api.pr_solve_many(rev)
    for (U, _), (Ur, _) in zip(out, out_r[::-1]):
        assert torch.equal(U, Ur)
    # a job without ICs takes part in nothing
    empty = api.Job(jobs[0].problem, jobs[0].coarse,
                    torch.empty((0, 32, 32), dtype=torch.float64, device="cuda"), 5, 1e-9)
    out_e = api.pr_solve_many([empty] + [api.Job(j.problem, j.coarse, j.u0, j.n_slices, j.tol)
                                         for j in jobs[:2]])
    assert out_e[0][1].iterations == 0 and out_e[0][0].shape[0] == 0
    assert torch.equal(out_e[1][0], out[0][0]) and torch.equal(out_e[2][0], out[1][0])


def test_many_mixed_precisions_and_cnn(api):
    from oracle import cnn
    n = 64
    spec = cnn.CnnSpec(n_layers=3, channels=16)
    ws, bs = cnn.init_weights(spec, seed=2, scale=0.1)
    net = api.CnnCoarse(ws, bs, prec="bf16")
    p64 = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=20)
    p32 = api.Problem(n=n, length=1.0, eps=0.03, conservative=True, stab=2.0, dt=1e-4, steps=20,
                      fine_prec="f32")
    psc = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=20,
                      f32_iters=2)
    jobs = [api.Job(p64, net, dev(synth.random_ic(n, [11])), 6, 1e-8),
            api.Job(p32, api.Coarse(dt=2e-3), dev(synth.random_ic(n, [12, 13])), 5, 1e-6),
            api.Job(psc, net, dev(synth.random_ic(n, [14])), 6, 1e-8),
            api.Job(p64, api.Coarse(dt=2e-3), dev(synth.random_ic(n, [15])), 6, 1e-8)]
    out = api.pr_solve_many(jobs)
    for j, (U, st) in zip(jobs, out):
        U1, st1 = api.pr_solve(j.problem, j.coarse, j.u0, j.n_slices, tol=j.tol)
        assert torch.equal(U, U1), j.problem
        assert list(st.ic_iterations) == list(st1.ic_iterations)


@pytest.mark.parametrize("conservative", [False, True])
@pytest.mark.parametrize("k32", [1, 3])
def test_schedule_reaches_fp64_serial_bitwise(api, conservative, k32):
    s = 6
    p = api.Problem(n=64, length=1.0, eps=0.02, conservative=conservative, stab=2.0, dt=1e-4,
                    steps=25, f32_iters=k32)
    g = api.Coarse(dt=25e-4)
    u0 = dev(synth.random_ic(64, [40, 41]))
    ser = api.pr_serial_fine(p, u0, s)
    U, st = api.pr_solve(p, g, u0, s, tol=0.0)
    assert st.iterations == k32 + s
    assert torch.equal(U, ser)
    for k in (1, 2):
        Uk, stk = api.pr_solve(p, g, u0, s, tol=0.0, max_iter=k32 + k, allow_not_converged=True)
        assert stk.status == 6
        assert torch.equal(Uk[:, :k + 1], ser[:, :k + 1])
        # slices past the exact prefix are FP32-seeded iterates, not yet exact
        assert not torch.equal(Uk[:, k + 1:], ser[:, k + 1:])


def test_schedule_never_freezes_in_fp32_iterations(api):
    p = api.Problem(n=32, length=1.0, eps=0.04, conservative=False, stab=2.0, dt=1e-3, steps=10)
    g = api.Coarse(dt=1e-2)
    u0 = dev(synth.random_ic(32, [42]))
    _, st0 = api.pr_solve(p, g, u0, 6, tol=10.0)
    assert st0.iterations == 1
    import dataclasses
    _, st2 = api.pr_solve(dataclasses.replace(p, f32_iters=2), g, u0, 6, tol=10.0)
    assert st2.iterations == 3 and st2.history.shape == (3, 1)


def test_schedule_converges_to_the_fp64_solution(api):
    # 64^2, eps 0.02, dt 1e-4, 100 steps/slice, 8 slices
    import dataclasses
    p = api.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=100)
    g = api.Coarse(dt=1e-2)
    u0 = synth.random_ic(64, [0, 1])
    ser = ac.serial_fine_trajectory(u0, oracle_problem(p), 8)
    U0, st0 = api.pr_solve(p, g, dev(u0), 8, tol=1e-10)
    e0 = rel(U0.cpu().numpy(), ser)
    for k32 in (1, 2):
        U, st = api.pr_solve(dataclasses.replace(p, f32_iters=k32), g, dev(u0), 8, tol=1e-10)
        assert (st.ic_iterations > k32).all()
        assert rel(U.cpu().numpy(), ser) <= max(10 * e0, 1e-10)


@pytest.mark.parametrize("chunks", [2, 3, 16])
def test_overlapped_sweep_gives_the_same_bits(api, chunks):
    """Fine chunks on a second stream overlapped with the sweep: the result
    of pr_solve and pr_solve_many is the same bits as without overlap."""
    from oracle import cnn
    spec = cnn.CnnSpec(n_layers=3, channels=16)
    ws, bs = cnn.init_weights(spec, seed=4, scale=0.1)
    net = api.CnnCoarse(ws, bs, prec="bf16x2")
    # 32 channels: the folded plan applies the correction in the network's
    # last kernel, after the sweep has waited for the fine chunk
    w32, b32 = cnn.init_weights(cnn.CnnSpec(n_layers=3, channels=32), seed=6, scale=0.1)
    net32 = api.CnnCoarse(w32, b32, prec="bf16x2")
    p = api.Problem(n=64, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=20)
    u0 = dev(synth.random_ic(64, [50, 51, 52]))
    jobs = mixed_jobs(api)
    try:
        api.pr_set_overlap(1)
        Uc, stc = api.pr_solve(p, net32, u0, 11, tol=0.0, max_iter=4, allow_not_converged=True)
        Ua, sta = api.pr_solve(p, net, u0, 11, tol=1e-9)
        Ub, stb = api.pr_solve(p, api.Coarse(dt=2e-3), u0, 11, tol=0.0, max_iter=3,
                               allow_not_converged=True)
        ref_many = [U.clone() for U, _ in api.pr_solve_many(jobs)]
        api.pr_set_overlap(chunks)
        assert api.pr_get_overlap() == chunks
        Uc2, stc2 = api.pr_solve(p, net32, u0, 11, tol=0.0, max_iter=4, allow_not_converged=True)
        Ua2, sta2 = api.pr_solve(p, net, u0, 11, tol=1e-9)
        Ub2, _ = api.pr_solve(p, api.Coarse(dt=2e-3), u0, 11, tol=0.0, max_iter=3,
                              allow_not_converged=True)
        jobs2 = mixed_jobs(api)
        out2 = api.pr_solve_many(jobs2)
    finally:
        api.pr_set_overlap(1)
    assert torch.equal(Ua, Ua2) and list(sta.ic_iterations) == list(sta2.ic_iterations)
    assert torch.equal(Ub, Ub2)
    assert torch.equal(Uc, Uc2) and np.array_equal(stc.history, stc2.history)
    for r, (U, _) in zip(ref_many, out2):
        assert torch.equal(r, U)


def test_many_combined_features_bitwise(api):
    """A batch mixing both schemes, both Laplacians, numerical and network
    coarse propagators, a precision schedule and a small working-set budget
    (so fine calls run in several chunks) gives each job its own bits."""
    from oracle import cnn
    spec = cnn.CnnSpec(n_layers=3, channels=16)
    ws, bs = cnn.init_weights(spec, seed=6, scale=0.1)
    net = api.CnnCoarse(ws, bs, prec="bf16x2")
    n = 64
    ps = [api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=10,
                      f32_iters=1),
          api.Problem(n=n, length=1.0, eps=0.03, conservative=False, stab=0.0, dt=1e-4, steps=10,
                      scheme="cn", picard=2, laplacian="spectral"),
          api.Problem(n=128, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=10)]
    gs = [net, api.Coarse(dt=1e-3), net]
    seeds = [[60, 61], [62], [63, 64]]
    try:
        api.pr_set_fine_working_set(3 * n * n * 8)
        jobs = [api.Job(p, g, dev(synth.random_ic(p.n, sd)), 6, 1e-9)
                for p, g, sd in zip(ps, gs, seeds)]
        out = api.pr_solve_many(jobs)
        for j, (U, st) in zip(jobs, out):
            U1, st1 = api.pr_solve(j.problem, j.coarse, j.u0, j.n_slices, tol=j.tol)
            assert torch.equal(U, U1)
            assert list(st.ic_iterations) == list(st1.ic_iterations)
    finally:
        api.pr_set_fine_working_set(256 << 20)


def test_many_folded_network_plan_gives_the_same_bits(api):
    """Jobs sharing one 32-channel split network form one coarse group: under
    the folded plan the network's last kernel applies their corrections
    through the shared offset tables (a job in FP32 iterations splits the
    corrections into two groups, and those steps run them separately).  The
    solutions, iteration counts and update norms match the layered plan's
    bit for bit."""
    from oracle import cnn
    print("case pr_solve_many, folded vs layered network plan", flush=True)
    n = 64
    spec = cnn.CnnSpec(n_layers=4, channels=32)
    ws, bs = cnn.init_weights(spec, seed=4, scale=0.1)
    net = api.CnnCoarse(ws, bs, prec="bf16x2")
    pa = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=10)
    pb = api.Problem(n=n, length=1.0, eps=0.03, conservative=True, stab=2.0, dt=1e-4, steps=10)
    pc = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=10,
                     f32_iters=1)

    def jobs():
        return [api.Job(pa, net, dev(synth.random_ic(n, [61, 62])), 6, 1e-9),
                api.Job(pb, net, dev(synth.random_ic(n, [63])), 4, 1e-9),
                api.Job(pc, net, dev(synth.random_ic(n, [64, 65])), 5, 1e-9)]

    try:
        api.pr_set_coarse_plan("folded")
        out_f = api.pr_solve_many(jobs(), allow_not_converged=True)
        api.pr_set_coarse_plan("layered")
        out_l = api.pr_solve_many(jobs(), allow_not_converged=True)
    finally:
        api.pr_set_coarse_plan("auto")
    for (Uf, sf), (Ul, sl) in zip(out_f, out_l):
        assert torch.equal(Uf, Ul)
        assert list(sf.ic_iterations) == list(sl.ic_iterations)
        assert np.array_equal(sf.history, sl.history)
