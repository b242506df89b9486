"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances:
  * FP64 fine path: rel-L2 <= 1e-12 per field (FFT round-off only).
  * FP32 fine path, one step from the float-rounded state: rel-L2 <= 1e-5.
  * FP32 over c steps: the float state carries ~1e-7 relative error per
    step (rounding of the state and of the transform), so the bound is
    c * 2.5e-7 (5e-5 at c = 200).
  * The correction is a fixed three-term expression evaluated in IEEE
    double in a stated order, so it is compared bit for bit.
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
    assert A.pr_abi_version() == 13
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_problem(p):
    return ac.Problem(n=p.n, length=p.length, eps=p.eps, conservative=p.conservative,
                      stab=p.stab, dt=p.dt, steps=p.steps)


def field_rel(a, b):
    return [rel(a[i], b[i]) for i in range(a.shape[0])]


# ------------------------------------------------------------------ F, FP64

@pytest.mark.parametrize("n,steps", [(16, 7), (32, 9), (64, 100), (128, 20), (256, 6), (512, 3),
                                     (1024, 2)])
@pytest.mark.parametrize("conservative", [False, True])
def test_fine_f64_matches_oracle(api, n, steps, conservative):
    print(f"case fine f64 n={n} steps={steps} cons={conservative}", flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=conservative, stab=2.0, dt=1e-4,
                    steps=steps)
    u0 = synth.random_ic(n, [1, 2, 3])
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    ref = ac.fine(u0, oracle_problem(p))
    assert max(field_rel(out, ref)) <= 1e-12


def test_fine_f64_config1_shape(api):
    # 64^2, eps 0.02, S 2, dt 1e-4, 100 steps: one slice of the 8-slice run
    p = api.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=100)
    u0 = synth.random_ic(64, range(8))
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    ref = ac.fine(u0, oracle_problem(p))
    assert max(field_rel(out, ref)) <= 1e-12


# ------------------------------------------------------------------ F, FP32

@pytest.mark.parametrize("n", [64, 256, 512])
@pytest.mark.parametrize("conservative", [False, True])
def test_fine_f32_one_step(api, n, conservative):
    print(f"case fine f32 one step n={n} cons={conservative}", flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=conservative, stab=2.0, dt=2e-5,
                    steps=1, fine_prec="f32")
    u0 = synth.random_ic(n, [5, 6])
    out = api.pr_fine_propagate(p, dev(u0), out_dtype=torch.float32).cpu().numpy()
    u32 = u0.astype(np.float32).astype(np.float64)
    ref = ac.fine(u32, oracle_problem(p))
    assert max(field_rel(out.astype(np.float64), ref)) <= 1e-5


def test_fine_f32_many_steps_bound(api):
    n, steps = 256, 200
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=False, stab=2.0, dt=2e-5,
                    steps=steps, fine_prec="f32")
    u0 = synth.random_ic(n, [7])
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    ref = ac.fine(u0, oracle_problem(p))
    assert max(field_rel(out, ref)) <= steps * 2.5e-7


# ------------------------------------------------------------- invariants

def test_fixed_points_and_mass_on_gpu(api):
    n = 64
    for cons in (False, True):
        p = api.Problem(n=n, length=1.0, eps=0.02, conservative=cons, stab=2.0, dt=1e-3, steps=50)
        u = np.stack([np.zeros((n, n)), np.ones((n, n)), -np.ones((n, n))])
        out = api.pr_fine_propagate(p, dev(u)).cpu().numpy()
        assert np.array_equal(out[0], u[0])
        assert np.abs(out[1:] - u[1:]).max() <= 4 * np.spacing(1.0)
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-3, steps=400)
    u0 = synth.random_ic(n, [1, 2])
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    assert np.abs(out.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-13


def test_discrete_mbp_on_gpu(api):
    n = 128
    u0 = synth.random_ic(n, [9], amp=1.0)
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=0.5, steps=40)
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    assert np.abs(out).max() <= 1.0 + 1e-13


# ------------------------------------------------------------------ G

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_coarse_apply_matches_oracle(api, prec):
    n = 64
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=100)
    g = api.Coarse(dt=1e-2, steps=2, prec=prec)
    u0 = synth.random_ic(n, [4, 5])
    out = api.pr_coarse_apply(p, g, dev(u0)).cpu().numpy()
    ref = ac.coarse_num(u0, oracle_problem(p), ac.Coarse(dt=1e-2, steps=2))
    tol = 1e-12 if prec == "f64" else 2e-6
    assert max(field_rel(out, ref)) <= tol


# ------------------------------------------------------------- correction

@pytest.mark.parametrize("fdt", [torch.float64, torch.float32])
def test_correct_bitwise(api, fdt):
    rng = np.random.default_rng(0)
    B, n = 3, 64
    f = rng.standard_normal((B, n, n))
    if fdt == torch.float32:
        f = f.astype(np.float32)
    gn, go, u = (rng.standard_normal((B, n, n)) for _ in range(3))
    upd0 = np.array([0.0, 10.0, 0.5])
    tf, tgn, tgo, tu = dev(f), dev(gn), dev(go), dev(u)
    tupd = dev(upd0)
    api.pr_correct(tf, tgn, tgo, tu, tupd)
    expect = f.astype(np.float64) + (gn - go)
    assert np.array_equal(tu.cpu().numpy(), expect)
    assert np.array_equal(tgo.cpu().numpy(), gn)
    m = np.abs(expect - u).max(axis=(1, 2))
    assert np.array_equal(tupd.cpu().numpy(), np.maximum(upd0, m))


def test_correct_propagates_nan(api):
    B, n = 2, 16
    f = np.zeros((B, n, n))
    f[1, 3, 4] = np.nan
    z = np.zeros((B, n, n))
    upd = dev(np.zeros(B))
    api.pr_correct(dev(f), dev(z), dev(z.copy()), dev(z.copy()), upd)
    r = upd.cpu().numpy()
    assert r[0] == 0.0 and np.isnan(r[1])


# ------------------------------------------------------------- Parareal

def config1():
    import paper_2510_07672_amd.api as A
    p = A.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=100)
    g = A.Coarse(dt=1e-2, steps=1)
    return p, g, 8


def test_solve_config1_matches_oracle(api):
    p, g, s = config1()
    u0 = synth.random_ic(64, [0])
    U, st = api.pr_solve(p, g, dev(u0), s, tol=1e-10)
    res = ac.parareal(u0, oracle_problem(p), s, tol=1e-10)
    assert st.iterations == int(res.iterations.max())
    assert list(st.ic_iterations) == list(res.iterations)
    assert rel(U.cpu().numpy(), res.U) <= 1e-12
    ser = ac.serial_fine_trajectory(u0, oracle_problem(p), s)
    assert rel(U.cpu().numpy(), ser) <= 1e-9


@pytest.mark.parametrize("conservative", [False, True])
def test_solve_k_equals_s_is_gpu_serial_fine_bitwise(api, conservative):
    p = api.Problem(n=32, length=1.0, eps=0.04, conservative=conservative, stab=2.0, dt=1e-3,
                    steps=10)
    g = api.Coarse(dt=1e-2, steps=1)
    s = 6
    u0 = dev(synth.random_ic(32, [21, 22, 23]))
    U, st = api.pr_solve(p, g, u0, s, tol=0.0)
    assert st.iterations == s and (st.ic_iterations == s).all()
    ser = api.pr_serial_fine(p, u0, s)
    assert torch.equal(U, ser)
    ref = ac.serial_fine_trajectory(u0.cpu().numpy(), oracle_problem(p), s)
    assert rel(U.cpu().numpy(), ref) <= 1e-12


def test_solve_prefix_exact_after_k(api):
    p = api.Problem(n=32, length=1.0, eps=0.04, conservative=False, stab=2.0, dt=1e-3, steps=10)
    g = api.Coarse(dt=1e-2, steps=1)
    s = 6
    u0 = dev(synth.random_ic(32, [24]))
    ser = api.pr_serial_fine(p, u0, s)
    for k in (1, 3):
        U, st = api.pr_solve(p, g, u0, s, tol=0.0, max_iter=k, allow_not_converged=True)
        assert st.status == 6  # PR_NOT_CONVERGED
        assert torch.equal(U[:, :k + 1], ser[:, :k + 1])


def test_solve_batch_equals_members_and_is_deterministic(api):
    p = api.Problem(n=32, length=1.0, eps=0.04, conservative=True, stab=2.0, dt=1e-3, steps=10)
    g = api.Coarse(dt=1e-2, steps=1)
    s = 6
    u0 = synth.random_ic(32, [31, 32, 33])
    Ub, stb = api.pr_solve(p, g, dev(u0), s, tol=1e-7)
    Ub2, _ = api.pr_solve(p, g, dev(u0), s, tol=1e-7)
    assert torch.equal(Ub, Ub2)
    perm = [2, 0, 1]
    Up, stp = api.pr_solve(p, g, dev(u0[perm]), s, tol=1e-7)
    assert torch.equal(Up, Ub[perm])
    for b in range(3):
        U1, st1 = api.pr_solve(p, g, dev(u0[b:b + 1]), s, tol=1e-7)
        assert st1.ic_iterations[0] == stb.ic_iterations[b]
        assert torch.equal(U1[0], Ub[b])
    res = ac.parareal(u0, oracle_problem(p), s, tol=1e-7)
    assert list(stb.ic_iterations) == list(res.iterations)
    assert rel(Ub.cpu().numpy(), res.U) <= 1e-12


def test_fine_batch_invariance_bitwise(api):
    p = api.Problem(n=128, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5, steps=5,
                    fine_prec="f32")
    u0 = synth.random_ic(128, range(5))
    a = api.pr_fine_propagate(p, dev(u0))
    b = api.pr_fine_propagate(p, dev(u0[::-1].copy()))
    c = api.pr_fine_propagate(p, dev(u0[2:3]))
    assert torch.equal(a, b.flip(0))
    assert torch.equal(a[2:3], c)


def test_solve_numeric_error(api):
    from paper_2510_07672_amd import _lib as L
    p = api.Problem(n=32, length=1.0, eps=0.04, conservative=False, stab=2.0, dt=1e-3, steps=5)
    g = api.Coarse(dt=5e-3, steps=1)
    u0 = synth.random_ic(32, [1, 2])
    u0[1, 5, 5] = np.nan
    with pytest.raises(L.PrError) as ei:
        api.pr_solve(p, g, dev(u0), 4, tol=1e-8)
    assert ei.value.status == L.PR_ERR_NUMERIC
    assert "IC 1" in str(ei.value)


def test_empty_batch_and_workspace_errors(api):
    import ctypes as C
    from paper_2510_07672_amd import _lib as L
    p = api.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=3)
    e = torch.empty((0, 64, 64), dtype=torch.float64, device="cuda")
    assert api.pr_fine_propagate(p, e).shape == (0, 64, 64)
    u = dev(synth.random_ic(64, [1]))
    out = torch.zeros_like(u)
    pc = p.c()
    need = L.lib().pr_fine_workspace_bytes(C.byref(pc), 1)
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    st = L.lib().pr_fine_propagate(C.byref(pc), 1, C.c_void_p(u.data_ptr()),
                                   C.c_void_p(out.data_ptr()), 0, C.c_void_p(small.data_ptr()),
                                   need - 1, None)
    assert st == L.PR_ERR_WORKSPACE
    assert torch.count_nonzero(out) == 0


# ------------------------------------------------------- launch plans

@pytest.fixture
def plan(api):
    set_ = []

    def use(n, prec, name):
        api.pr_set_fine_plan(n, prec, name)
        set_.append((n, prec))
    yield use
    for n, prec in set_:
        api.pr_set_fine_plan(n, prec, "auto")


@pytest.mark.parametrize("n,steps", [(16, 9), (32, 7), (64, 100), (128, 30)])
@pytest.mark.parametrize("conservative", [False, True])
@pytest.mark.parametrize("which", ["resident", "stream"])
def test_small_n_plans_match_oracle_f64(api, plan, n, steps, conservative, which):
    print(f"case plan={which} n={n} cons={conservative}", flush=True)
    plan(n, "f64", which)
    assert api.pr_get_fine_plan(n, "f64") == which
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=conservative, stab=2.0, dt=1e-4,
                    steps=steps)
    u0 = synth.random_ic(n, [11, 12, 13, 14, 15])
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    ref = ac.fine(u0, oracle_problem(p))
    assert max(field_rel(out, ref)) <= 1e-12
    if conservative:
        assert np.abs(out.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-13


@pytest.mark.parametrize("n", [16, 64, 128])
@pytest.mark.parametrize("conservative", [False, True])
def test_resident_f32_one_step(api, plan, n, conservative):
    plan(n, "f32", "resident")
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=conservative, stab=2.0, dt=2e-5,
                    steps=1, fine_prec="f32")
    u0 = synth.random_ic(n, [5, 6])
    out = api.pr_fine_propagate(p, dev(u0), out_dtype=torch.float32).cpu().numpy()
    ref = ac.fine(u0.astype(np.float32).astype(np.float64), oracle_problem(p))
    assert max(field_rel(out.astype(np.float64), ref)) <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [32, 128])
def test_resident_equals_stream_bitwise_classic(api, plan, n, prec):
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=13,
                    fine_prec=prec)
    u0 = dev(synth.random_ic(n, range(6)))
    plan(n, prec, "resident")
    a = api.pr_fine_propagate(p, u0)
    plan(n, prec, "stream")
    b = api.pr_fine_propagate(p, u0)
    assert torch.equal(a, b)


def test_autotune_picks_a_plan(api, plan):
    p = api.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=20)
    u0 = dev(synth.random_ic(64, range(4)))
    choice = api.pr_autotune_fine(p, u0)
    assert choice in ("resident", "stream")
    assert api.pr_get_fine_plan(64, "f64") == choice
    p2 = api.Problem(n=256, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=2)
    assert api.pr_autotune_fine(p2, dev(synth.random_ic(256, [1]))) == "stream"
    plan(64, "f64", "auto")


# ------------------------------------------------------- graph replay

@pytest.fixture
def graphs(api):
    yield api
    api.pr_set_graphs(True)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replays_match_eager(graphs, prec):
    api = graphs
    p = api.Problem(n=256, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5, steps=5,
                    fine_prec=prec)
    u0 = dev(synth.random_ic(256, range(6)))
    api.pr_set_graphs(False)
    ref = api.pr_fine_propagate(p, u0)
    api.pr_set_graphs(True)
    ws = None
    import ctypes as C
    from paper_2510_07672_amd import _lib as L
    need = L.lib().pr_fine_workspace_bytes(C.byref(p.c()), 6)
    ws = api.workspace(need, "cuda")
    for rep in range(4):
        out = api.pr_fine_propagate(p, u0, ws=ws)
        # the program's own eager work between replays
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        _ = (x * x).sum().item()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"


def test_graph_cache_eviction(graphs):
    """More distinct launch sequences than the graph cache holds (32): each
    new one evicts the least recently used graph after that graph's last
    launch has finished (an event per entry, no device-wide wait); every
    result equals the eager launch bit for bit, also for sequences whose
    graphs were evicted and are captured again."""
    print("case graph cache eviction: 40 step counts at 64^2", flush=True)
    api = graphs
    u0 = dev(synth.random_ic(64, range(3)))
    api.pr_set_fine_plan(64, "f64", "stream")
    try:
        refs = {}
        api.pr_set_graphs(False)
        for c in range(1, 41):
            p = api.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4,
                            steps=c)
            refs[c] = api.pr_fine_propagate(p, u0)
        api.pr_set_graphs(True)
        ws = api.workspace(1 << 24, "cuda")
        for c in list(range(1, 41)) + [1, 2, 3]:
            p = api.Problem(n=64, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4,
                            steps=c)
            out = api.pr_fine_propagate(p, u0, ws=ws)
            assert torch.equal(out, refs[c]), f"steps {c}"
    finally:
        api.pr_set_fine_plan(64, "f64", "auto")
        api.pr_set_graphs(True)


def test_graph_solve_matches_eager_solve(graphs):
    api = graphs
    p = api.Problem(n=256, length=1.0, eps=0.01, conservative=False, stab=2.0, dt=2e-5, steps=4)
    g = api.Coarse(dt=8e-5, steps=1)
    u0 = dev(synth.random_ic(256, [1, 2, 3]))
    api.pr_set_graphs(False)
    Ue, ste = api.pr_solve(p, g, u0, 5, tol=1e-9)
    api.pr_set_graphs(True)
    for rep in range(2):
        Ug, stg = api.pr_solve(p, g, u0, 5, tol=1e-9)
        assert torch.equal(Ug, Ue)
        assert list(stg.ic_iterations) == list(ste.ic_iterations)
    Se = None
    api.pr_set_graphs(False)
    Se = api.pr_serial_fine(p, u0, 5)
    api.pr_set_graphs(True)
    assert torch.equal(api.pr_serial_fine(p, u0, 5), Se)


@pytest.mark.parametrize("budget_fields", [0, 1, 3, 7])
def test_working_set_chunking_gives_the_same_bits(api, budget_fields):
    """Streaming F in chunks sized by the working-set budget (here a few
    fields of 256^2 per chunk, or off) gives the same bits as one call."""
    n = 256
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5, steps=4)
    pc = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=0.0, dt=2e-5, steps=3,
                     scheme="cn", picard=2)
    u0 = dev(synth.random_ic(n, range(10)))
    try:
        api.pr_set_fine_working_set(0)
        ref = api.pr_fine_propagate(p, u0)
        refc = api.pr_fine_propagate(pc, u0)
        refs, _ = api.pr_solve(p, api.Coarse(dt=8e-5), u0[:4].contiguous(), 5, tol=0.0, max_iter=2,
                               allow_not_converged=True)
        api.pr_set_fine_working_set(budget_fields * n * n * 8)
        assert torch.equal(api.pr_fine_propagate(p, u0), ref)
        assert torch.equal(api.pr_fine_propagate(pc, u0), refc)
        U, _ = api.pr_solve(p, api.Coarse(dt=8e-5), u0[:4].contiguous(), 5, tol=0.0, max_iter=2,
                            allow_not_converged=True)
        assert torch.equal(U, refs)
    finally:
        api.pr_set_fine_working_set(256 << 20)
