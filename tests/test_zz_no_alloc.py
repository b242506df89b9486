"""pr_fine_propagate_noalloc: F with the library's static scratch instead of
a caller workspace, against pr_fine_propagate bit for bit, on two calls in a
row (the second with fewer fields, on the scratch the first one left), and
its rejection of batches that exceed the scratch."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2510_07672_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2510_07672_amd import api as A
    return A


@pytest.mark.parametrize("n,nf1,nf2,cons,out_dtype", [(256, 48, 17, True, torch.float64),
                                                      (128, 40, 9, False, torch.float64),
                                                      (512, 12, 5, True, torch.float32)])
def test_noalloc_matches_workspace_call(api, n, nf1, nf2, cons, out_dtype):
    print(f"case noalloc n={n} fields {nf1} then {nf2} conservative={cons} out={out_dtype}",
          flush=True)
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=cons, stab=2.0, dt=2e-5, steps=7)
    for nf, seed0 in ((nf1, 100), (nf2, 300)):
        u0 = torch.from_numpy(synth.random_ic(n, range(seed0, seed0 + nf))).cuda()
        ref = api.pr_fine_propagate(p, u0, out_dtype=out_dtype)
        out = torch.full_like(ref, float("nan"))
        api.pr_fine_propagate_noalloc(p, u0, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"{nf} fields"


def test_noalloc_rejects_batches_beyond_the_scratch(api):
    from paper_2510_07672_amd import _lib as L
    n = 256
    p = api.Problem(n=n, length=1.0, eps=0.01, conservative=False, stab=2.0, dt=2e-5, steps=3)
    u0 = torch.from_numpy(synth.random_ic(n, range(200))).cuda()
    out = torch.zeros_like(u0)
    with pytest.raises(L.PrError) as ei:
        api.pr_fine_propagate_noalloc(p, u0, out)
    assert ei.value.status == L.PR_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out)) == 0
    # a batch that fits still runs after the rejection
    ref = api.pr_fine_propagate(p, u0[:8].contiguous())
    got = torch.empty_like(ref)
    api.pr_fine_propagate_noalloc(p, u0[:8].contiguous(), got)
    assert torch.equal(got, ref)
