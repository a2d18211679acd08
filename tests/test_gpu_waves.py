"""GPU: device-memory estimate and pairs processed in waves that fit a budget.

sf_memory_bytes must cover what sf_create allocates (read as the drop in free
device memory), and run_pipeline_waves, which runs a batch of pairs as waves
of as many pairs as fit the budget, must give every pair the result of its
own single-pair pipeline bit for bit (same launch shape).
"""
import numpy as np
import pytest

from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision", [api.SF_FP64, api.SF_FP32])
def test_memory_estimate_covers_the_allocation(gpu, precision):
    W, H, px, py, d = 640, 480, 4, 4, 8
    est = api.sf_memory_bytes(W, H, 1, px, py, d, factor_precision=precision)
    # a first context takes the runtime's one-time costs (code objects, queues)
    first = api.sf_create(W, H, 1, px, py, d, factor_precision=precision)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = api.sf_create(W, H, 1, px, py, d, factor_precision=precision)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    ctx.close()
    first.close()
    print("estimate", est, "allocated", used)
    # allocations are rounded up to pages; nothing else is allocated in between
    assert est <= used <= est + 64 * 2**20, (est, used)


def test_pairs_in_waves_equal_their_single_runs(gpu):
    W, H, px, py, d, N = 48, 40, 2, 2, 4, 5
    pairs = [synth.make_pair("plain64", 20 + i, W=W, H=H) for i in range(N)]
    I0 = dev(np.stack([p.I0 for p in pairs]))
    I1 = dev(np.stack([p.I1 for p in pairs]))
    A0 = np.stack([synth.random_alpha(W, H, 40 + i) for i in range(N)])
    c1 = api.sf_create(W, H, 1, px, py, d)
    P = api.sf_subdomain_geometry(c1, 0)["P"]
    c1.close()
    kw = dict(rtol=1e-9, max_sweeps=800, passes=1)
    # a budget of exactly two pairs: waves of 2, 2 and 1 (two contexts)
    budget = api.sf_memory_bytes(W, H, 2, px, py, d)
    Al = dev(A0)
    U = torch.empty((N, 3, H, W), dtype=torch.float64, device="cuda")
    wave, res = api.run_pipeline_waves(I0, I1, Al, U, px, py, d, budget_bytes=budget, band_tile=P, **kw)
    assert wave == 2 and len(res) == 3
    for i in range(N):
        ctx = api.sf_create(W, H, 1, px, py, d, band_tile=P)
        a1 = dev(A0[i:i + 1])
        u1 = torch.zeros((1, 3, H, W), dtype=torch.float64, device="cuda")
        r1 = api.run_pipeline(ctx, I0[i:i + 1].contiguous(), I1[i:i + 1].contiguous(), a1, u1, **kw)
        ctx.close()
        w, j = divmod(i, 2)
        assert [s[0] for s in r1.sweeps] == [s[j] for s in res[w].sweeps]
        assert torch.equal(u1[0], U[i]) and torch.equal(a1[0], Al[i])


def test_waves_refuse_a_budget_below_one_pair(gpu):
    W, H = 32, 24
    I0 = torch.zeros((2, H, W), dtype=torch.float64, device="cuda")
    Al = torch.full((2, H - 1, W - 1, 2), 0.1, dtype=torch.float64, device="cuda")
    U = torch.empty((2, 3, H, W), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SfError) as e:
        api.run_pipeline_waves(I0, I0, Al, U, 2, 1, 2, budget_bytes=1024)
    assert e.value.code == api.SF_ERR_OOM
