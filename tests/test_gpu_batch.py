"""GPU: batching of pairs and the launch-shape autotuner.

A batch shares every launch; with the same launch shape each pair's result
equals its single-pair result bit for bit.  A different shape (workgroups
per chain) only reorders the partial sums inside a row, so after autotuning
results agree to rounding.
"""
import numpy as np
import pytest

from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def solve(ctx, I0, I1, Al, passes=1):
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    A = Al.clone()
    res = api.run_pipeline(ctx, I0, I1, A, U, rtol=1e-8, max_sweeps=2000, passes=passes)
    return U, A, res


def test_two_full_size_pairs_equal_their_single_runs(gpu):
    # 640x480 pairs of seeds 2 and 3 as one batch (the batched form that is timed)
    W, H = 640, 480
    pairs = [synth.make_pair("plain640", s) for s in (2, 3)]
    I0 = dev(np.stack([q.I0 for q in pairs]))
    I1 = dev(np.stack([q.I1 for q in pairs]))
    Al = dev(np.stack([synth.constant_alpha(W, H)] * 2))
    ctx = api.sf_create(W, H, 2, 4, 4, 8)
    P = api.sf_subdomain_geometry(ctx, 0)["P"]
    U, A, res = solve(ctx, I0, I1, Al, passes=1)
    ctx.close()
    for b in range(2):
        c1 = api.sf_create(W, H, 1, 4, 4, 8, band_tile=P)       # the batch's shape, one pair
        U1, A1, r1 = solve(c1, I0[b:b + 1].contiguous(), I1[b:b + 1].contiguous(), Al[b:b + 1].contiguous(), 1)
        assert [s[0] for s in r1.sweeps] == [s[b] for s in res.sweeps]
        assert torch.equal(U1[0], U[b]) and torch.equal(A1[0], A[b])
        c1.close()


@pytest.mark.parametrize("W,H,px,py,d", [(72, 56, 3, 3, 8), (640, 480, 4, 4, 8)])
def test_autotune_picks_a_shape_and_keeps_results(gpu, W, H, px, py, d):
    p = synth.make_pair("plain640", 3, W=W, H=H)
    al = synth.random_alpha(W, H, 5)
    I0, I1, Al = dev(p.I0[None]), dev(p.I1[None]), dev(al[None])
    ctx = api.sf_create(W, H, 1, px, py, d)
    U0, _, r0 = solve(ctx, I0, I1, Al)
    nt_blocks = min((3 * min(x1 - x0, y1 - y0) + 31) // 32
                    for x0, x1, y0, y1 in (api.sf_subdomain_geometry(ctx, i)["box"]
                                           for i in range(api.sf_num_subdomains(ctx))))
    scratch = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    bt = api.sf_autotune(ctx, scratch, 2)
    assert 1 <= bt <= nt_blocks
    assert api.sf_subdomain_geometry(ctx, 0)["P"] == bt
    U1, _, r1 = solve(ctx, I0, I1, Al)
    assert [s[0] for s in r1.sweeps] == [s[0] for s in r0.sweeps]
    assert float(torch.linalg.norm(U1 - U0) / torch.linalg.norm(U0)) <= 1e-12
    ctx.close()


def test_autotune_needs_factors(gpu):
    ctx = api.sf_create(32, 24, 1, 2, 1, 2)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SfError) as e:
        api.sf_autotune(ctx, U, 2)
    assert e.value.code == api.SF_ERR_STATE
    ctx.close()
