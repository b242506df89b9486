"""GPU parity of the second FFT radix split of the streaming semi-implicit
passes (Section 3.1's FFT-diagonalised step): a trailing 8 x 2 of stages
taken as 4 x 4 at N = 16, 128 and 1024.  The split changes only the order
of the transforms' operations, so the fine solve must stay within the FP64
path's rel-L2 1e-12 of the oracle (FP32: the 1e-5 per step of the FP32
path) and within rounding of the other split; replayed graphs must take
the split in force.  Through the C ABI."""

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


@pytest.fixture
def split(api):
    """Set splits (and the streaming plan for N <= 128) for the test, and
    afterwards put the plan back to 'auto' and the split to 'r8', the
    untuned default: an autotuner record left by a test would otherwise
    change the split that later tests in the process run under."""
    touched = []

    def use(n, prec, name):
        api.pr_set_fine_plan(n, prec, "stream")
        api.pr_set_fft_split(n, prec, name)
        touched.append((n, prec))
    yield use
    for n, prec in touched:
        api.pr_set_fft_split(n, prec, "r8")
        api.pr_set_fine_plan(n, prec, "auto")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_problem(p):
    return ac.Problem(n=p.n, length=p.length, eps=p.eps, conservative=p.conservative,
                      stab=p.stab, dt=p.dt, steps=p.steps)


@pytest.mark.parametrize("n,steps,nf", [(16, 9, 5), (128, 20, 3), (1024, 2, 2)])
@pytest.mark.parametrize("conservative", [False, True])
def test_r4_tail_matches_oracle_f64(api, split, n, steps, nf, conservative):
    print(f"case split r4_tail f64 n={n} steps={steps} cons={conservative}", flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=conservative, stab=2.0, dt=1e-4,
                    steps=steps)
    u0 = synth.random_ic(n, range(20, 20 + nf))
    split(n, "f64", "r4_tail")
    assert api.pr_get_fft_split(n, "f64") == "r4_tail"
    out = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    ref = ac.fine(u0, oracle_problem(p))
    assert max(rel(out[i], ref[i]) for i in range(nf)) <= 1e-12
    if conservative:
        assert np.abs(out.mean(axis=(1, 2)) - u0.mean(axis=(1, 2))).max() <= 1e-13
    split(n, "f64", "r8")
    out8 = api.pr_fine_propagate(p, dev(u0)).cpu().numpy()
    assert max(rel(out[i], out8[i]) for i in range(nf)) <= 1e-13


@pytest.mark.parametrize("n", [128, 1024])
def test_r4_tail_f32_one_step(api, split, n):
    print(f"case split r4_tail f32 n={n}", flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=True, stab=2.0, dt=2e-5, steps=1,
                    fine_prec="f32")
    u0 = synth.random_ic(n, [30, 31])
    split(n, "f32", "r4_tail")
    out = api.pr_fine_propagate(p, dev(u0), out_dtype=torch.float32).cpu().numpy()
    u32 = u0.astype(np.float32).astype(np.float64)
    ref = ac.fine(u32, oracle_problem(p))
    assert max(rel(out[i].astype(np.float64), ref[i]) for i in range(2)) <= 1e-5


def test_split_only_where_it_differs(api, split):
    """N without a second split report r8 whatever the setting; bad values
    are rejected."""
    for n in (32, 64, 256, 512):
        split(n, "f64", "r4_tail")
        assert api.pr_get_fft_split(n, "f64") == "r8"
    from paper_2510_07672_amd import _lib as L
    with pytest.raises(L.PrError):
        api.pr_set_fft_split(1000, "f64", "r8")


def test_graphs_follow_the_split(api, split):
    """With graph replay on, switching the split between calls replays the
    sequence captured for that split: each split's replays equal its eager
    result bit for bit, and the two splits differ only by rounding."""
    print("case split graphs 1024^2 f64", flush=True)
    n = 1024
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=3)
    u0 = dev(synth.random_ic(n, [40, 41]))
    eager = {}
    try:
        api.pr_set_graphs(False)
        for name in ("r8", "r4_tail"):
            split(n, "f64", name)
            eager[name] = api.pr_fine_propagate(p, u0)
    finally:
        api.pr_set_graphs(True)
    for rep in range(2):
        for name in ("r8", "r4_tail"):
            split(n, "f64", name)
            out = api.pr_fine_propagate(p, u0)
            torch.cuda.synchronize()
            assert torch.equal(out, eager[name]), f"{name} replay {rep}"
    a, b = eager["r8"].cpu().numpy(), eager["r4_tail"].cpu().numpy()
    assert rel(b, a) <= 1e-13


def test_parareal_with_r4_tail_matches_oracle(api, split):
    """Algorithm 2 with the numerical G at 128^2 under the second split: the
    solve after k = s iterations is the serial fine solve (oracle)."""
    print("case split parareal 128^2", flush=True)
    n, s = 128, 4
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=True, stab=2.0, dt=1e-4, steps=10)
    g = api.Coarse(dt=1e-3, steps=1, prec="f64")
    u0 = synth.random_ic(n, [50, 51])
    split(n, "f64", "r4_tail")
    U, st = api.pr_solve(p, g, dev(u0), s, tol=0.0, max_iter=s, allow_not_converged=True)
    ref = ac.serial_fine_trajectory(u0, oracle_problem(p), s)
    Uc = U.cpu().numpy()
    assert rel(Uc, ref) <= 1e-12


def test_autotune_records_a_split(api, split):
    print("case split autotune 1024^2 f64", flush=True)
    n = 1024
    p = api.Problem(n=n, length=1.0, eps=0.02, conservative=False, stab=2.0, dt=1e-4, steps=3)
    u0 = dev(synth.random_ic(n, [60, 61, 62, 63]))
    split(n, "f64", "auto")
    assert api.pr_autotune_fine(p, u0) == "stream"
    assert api.pr_get_fft_split(n, "f64") in ("r8", "r4_tail")
    api.pr_set_fft_split(n, "f64", "r8")
    assert api.pr_get_fft_split(n, "f64") == "r8"
