"""Deferred status (sf_config.deferred_status = 1): sf_assemble and
sf_factor_subdomains only enqueue, and their status comes back from the next
call that collects it.  The results must be those of the waiting form, bit
for bit, and every status the waiting form returns must still be returned,
by that later call."""
import numpy as np
import pytest

from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def solve(deferred, prec=api.SF_FP64, pivot_tol=0.0):
    W, H = 72, 56
    p = synth.make_pair("plain640", 3, W=W, H=H)
    al = synth.random_alpha(W, H, 4)
    ctx = api.sf_create(W, H, 1, 3, 3, 8, factor_precision=prec, pivot_tol=pivot_tol, deferred_status=deferred)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-10, 500)
    out = (code, sw, rr, U.cpu().numpy(), api.sf_factor_fallbacks(ctx))
    ctx.close()
    return out


@pytest.mark.parametrize("prec,pivot_tol", [(api.SF_FP64, 0.0), (api.SF_FP32_FACTOR, 0.0),
                                            (api.SF_FP32_FACTOR, 0.999)])
def test_deferred_equals_waiting(gpu, prec, pivot_tol):
    # pivot_tol 0.999 rejects FP32 pivots, so the FP64 refactorisation runs
    # inside the solve's status collection
    a = solve(0, prec, pivot_tol)
    b = solve(1, prec, pivot_tol)
    assert a[0] == b[0] == api.SF_OK and a[1] == b[1] and a[2] == b[2]
    assert np.array_equal(a[3], b[3])
    assert a[4] == b[4]
    if pivot_tol > 0.5:
        assert b[4] == 9


def test_deferred_statuses(gpu):
    W, H = 20, 16
    p = synth.make_pair("plain64", 2, W=W, H=H)
    al = synth.constant_alpha(W, H)
    ctx = api.sf_create(W, H, 1, 2, 2, 4, deferred_status=1)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    # a non-finite frame: assemble and factor enqueue, the solve reports it
    bad = p.I0.copy()
    bad[3, 4] = np.nan
    api.sf_assemble(ctx, dev(bad[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    with pytest.raises(api.SfError) as e:
        api.sf_schwarz_solve(ctx, U, 1e-8, 10)
    assert e.value.code == api.SF_NONFINITE
    # the context is back to "created": a solve is out of order
    with pytest.raises(api.SfError) as e:
        api.sf_schwarz_solve(ctx, U, 1e-8, 10)
    assert e.value.code == api.SF_ERR_STATE
    # an alpha <= 0, collected by sf_sync
    al0 = al.copy()
    al0[2, 3, 1] = 0.0
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al0[None]))
    with pytest.raises(api.SfError) as e:
        api.sf_sync(ctx)
    assert e.value.code == api.SF_ERR_INVALID
    api.sf_sync(ctx)                      # nothing pending any more
    # a singular subdomain matrix: the residual call collects SF_NOT_SPD
    flat = np.full((1, H, W), 0.5)
    c1 = api.sf_create(W, H, 1, 1, 1, 0, deferred_status=1)
    api.sf_assemble(c1, dev(flat), dev(flat), dev(al[None]))
    api.sf_factor_subdomains(c1)
    r = torch.empty(c1.field_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SfError) as e:
        api.sf_residual(c1, U, r)
    assert e.value.code == api.SF_NOT_SPD
    assert e.value.detail["pair"] == 0 and e.value.detail["subdomain"] == 0
    with pytest.raises(api.SfError) as e:
        api.sf_schwarz_solve(c1, U, 1e-8, 10)
    assert e.value.code == api.SF_ERR_STATE
    c1.close()
    # good data: the same calls succeed
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 200)
    assert code == api.SF_OK and rr[0] <= 1e-8
    ctx.close()
