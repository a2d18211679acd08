"""GPU: a context made on a non-blocking stream (torch's side streams are).

Every upload, clear and launch of the library is queued on the context's
stream, so the whole pipeline run there, also with graph-replayed solves and
the sweep-shape tuner, must give the results of the same pipeline on the
default stream bit for bit.
"""
import numpy as np
import pytest

from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def pipeline(I0, I1, A0, W, H, graph, tune):
    ctx = api.sf_create(W, H, 1, 3, 2, 6)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    alpha = A0.clone()
    if tune:
        api.sf_assemble(ctx, I0, I1, alpha)
        api.sf_factor_subdomains(ctx)
        api.sf_autotune(ctx, U, trials=2)
        U.zero_()
    res = api.run_pipeline(ctx, I0, I1, alpha, U, rtol=1e-9, max_sweeps=800, passes=2, graph=graph)
    return ctx, U, alpha, res


@pytest.mark.parametrize("graph,tune", [(False, False), (True, False), (False, True)])
def test_pipeline_on_a_side_stream_equals_default_stream(gpu, graph, tune):
    W, H = 70, 52
    p = synth.make_pair("plain640", 11, W=W, H=H)
    I0, I1 = dev(p.I0[None]), dev(p.I1[None])
    A0 = dev(synth.random_alpha(W, H, 11)[None])
    ctx_d, U_d, a_d, r_d = pipeline(I0, I1, A0, W, H, graph, False)
    torch.cuda.synchronize()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx_s, U_s, a_s, r_s = pipeline(I0, I1, A0, W, H, graph, tune)
    side.synchronize()
    assert r_s.status == r_d.status == api.SF_OK
    if tune:
        # the tuner may pick another sweep shape, which changes rounding only
        for a, b in zip(r_s.sweeps, r_d.sweeps):
            assert abs(a[0] - b[0]) <= 1
        assert float((U_s - U_d).abs().max() / U_d.abs().max()) <= 1e-8
        assert float((a_s - a_d).abs().max() / a_d.abs().max()) <= 1e-8
    else:
        assert r_s.sweeps == r_d.sweeps
        assert torch.equal(U_s, U_d) and torch.equal(a_s, a_d)
    ctx_s.close()
    ctx_d.close()
