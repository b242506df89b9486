"""The work-queue fine sweep (one persistent launch per (N, precision)
class for the fine solves of a call or of a Parareal iteration, Section 3.3)
against the pass-by-pass launches: bit for bit, for single F calls (every
supported size, both precisions, both models, with and without working-set
chunks) and for heterogeneous pr_solve_many batches (solutions, iteration
counts and update norms), and against the oracle."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import allen_cahn as ac  # noqa: E402
from paper_2510_07672_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2510_07672_amd import api as A
    yield A
    A.pr_set_fine_queue(False)
    A.pr_set_fine_working_set(256 << 20)


def both(api, fn, mode=1):
    api.pr_set_fine_queue(0)
    a = fn()
    api.pr_set_fine_queue(mode)
    try:
        b = fn()
    finally:
        api.pr_set_fine_queue(False)
    return a, b


@pytest.mark.parametrize("n,prec,nf", [(64, "f64", 5), (128, "f64", 3), (256, "f64", 7),
                                       (512, "f64", 3), (1024, "f64", 2), (64, "f32", 4),
                                       (128, "f32", 3), (256, "f32", 5)])
@pytest.mark.parametrize("cons", [False, True])
def test_queue_fine_matches_per_pass(api, n, prec, nf, cons):
    print(f"case queue F n={n} {prec} fields={nf} conservative={cons}", flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=cons, stab=2.0, dt=2e-5, steps=6,
                    fine_prec=prec)
    u0 = torch.from_numpy(synth.random_ic(n, range(10, 10 + nf))).cuda()
    api.pr_set_fine_plan(n, prec, "stream")
    try:
        a, b = both(api, lambda: api.pr_fine_propagate(p, u0))
    finally:
        api.pr_set_fine_plan(n, prec, "auto")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("n,prec,nf,cons", [(64, "f32", 5, True), (256, "f64", 9, True),
                                            (512, "f64", 3, False)])
def test_queue_adopted_matches_per_pass(api, n, prec, nf, cons):
    """Every XCD queue adopted (mode 2): the items of a queue run on blocks
    of any XCD, which hand results over with device-wide releases; the
    fallback for a placement of blocks that leaves an XCD without any."""
    print(f"case queue F adopted n={n} {prec} fields={nf} conservative={cons}", flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=cons, stab=2.0, dt=2e-5, steps=6,
                    fine_prec=prec)
    u0 = torch.from_numpy(synth.random_ic(n, range(20, 20 + nf))).cuda()
    a, b = both(api, lambda: api.pr_fine_propagate(p, u0), mode=2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_queue_fine_with_chunks_matches_oracle(api):
    """Working-set chunks of 3 fields (a 12 MiB budget at 512^2 FP64): the
    queue orders its items chunk by chunk; F on 8 fields against the oracle."""
    print("case queue F 512^2 x 8 in chunks of 3", flush=True)
    n, nf = 512, 8
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=1e-5, steps=10)
    u0 = synth.random_ic(n, range(20, 20 + nf))
    d = torch.from_numpy(u0).cuda()
    api.pr_set_fine_working_set(3 * n * n * 8)
    try:
        a, b = both(api, lambda: api.pr_fine_propagate(p, d))
    finally:
        api.pr_set_fine_working_set(256 << 20)
    assert torch.equal(a, b)
    po = ac.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=1e-5, steps=10)
    ref = ac.fine(u0[[0, 7]], po)
    got = b.cpu().numpy()[[0, 7]]
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def uneven_jobs(api, f32_iters):
    """Jobs of three sizes, both models, different eps and slice counts, with
    an FP32-then-FP64 schedule (FP32 fine solves of 64^2..256^2 take the
    queue; the numerical G)."""
    jobs = []
    spec = [(64, 6, 0.03, False), (128, 5, 0.02, True), (256, 4, 0.015, False),
            (64, 7, 0.025, True), (256, 3, 0.01, True), (512, 3, 0.012, False)]
    for i, (n, s, eps, cons) in enumerate(spec):
        p = api.Problem(n=n, length=1.0, eps=eps, conservative=cons, stab=2.0, dt=2e-5, steps=10,
                        f32_iters=f32_iters)
        u0 = torch.from_numpy(synth.random_ic(n, [700 + i, 800 + i])).cuda()
        jobs.append(api.Job(p, api.Coarse(dt=10 * 2e-5, steps=1), u0, s, 1e-9))
    return jobs


@pytest.mark.parametrize("f32_iters,mode", [(0, 1), (1, 1), (1, 2)])
def test_queue_solve_many_matches_per_pass(api, f32_iters, mode):
    print(f"case queue pr_solve_many 6 jobs f32_iters={f32_iters} mode={mode}", flush=True)
    a, b = both(api, lambda: api.pr_solve_many(uneven_jobs(api, f32_iters)), mode=mode)
    for (Ua, sa), (Ub, sb) in zip(a, b):
        assert torch.equal(Ua, Ub)
        assert sa.iterations == sb.iterations
        assert np.array_equal(sa.history, sb.history)


def test_queue_parareal_matches_oracle(api):
    """Parareal on 64^2 with 8 slices and the numerical G through the queue
    against the oracle's Algorithm 2: same iterations, rel-L2 <= 1e-12."""
    print("case queue Parareal 64^2 x 8 slices", flush=True)
    n, s = 64, 8
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=100)
    po = ac.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=100)
    u0 = synth.random_ic(n, [0])
    api.pr_set_fine_queue(True)
    try:
        U, st = api.pr_solve(p, api.Coarse(dt=0.01, steps=1), torch.from_numpy(u0).cuda(), s,
                             tol=1e-10)
    finally:
        api.pr_set_fine_queue(False)
    res = ac.parareal(u0, po, s, tol=1e-10)
    assert st.iterations == int(res.iterations.max())
    assert list(st.ic_iterations) == list(res.iterations)
    assert np.linalg.norm(U.cpu().numpy() - res.U) <= 1e-12 * np.linalg.norm(res.U)


def test_autotune_records_a_queue_choice(api):
    """pr_autotune_fine times the queue against the per-pass launches for a
    class the queue covers and records the faster one; F gives the same
    bits either way, before and after."""
    print("case queue autotune 256^2 x 16", flush=True)
    n, nf = 256, 16
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5, steps=8)
    u0 = torch.from_numpy(synth.random_ic(n, range(40, 40 + nf))).cuda()
    api.pr_set_fine_queue(0)
    api.pr_set_fine_queue(1)
    ref_q = api.pr_fine_propagate(p, u0)
    api.pr_set_fine_queue(0)
    assert api.pr_autotune_fine(p, u0) == "stream"
    assert api.pr_get_fine_queue_choice(n, "f64") in (0, 1)
    out = api.pr_fine_propagate(p, u0)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_q)
    assert api.pr_get_fine_queue_choice(500, "f64") == -1

