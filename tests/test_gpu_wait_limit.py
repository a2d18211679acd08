"""Bounded device-side waits (sf_set_wait_limit).  With the bound at zero
polls, every wait of one workgroup on another that is not satisfied at once
gives up: the factorisation and the solves return SF_ERR_DEVICE and every
kernel still ends normally.  With the default bound restored, the same
context computes what a fresh one does, bit for bit (the exchange tags of the
abandoned launches are never taken for new ones)."""
import numpy as np
import pytest

from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

W, H = 72, 56
DEFAULT_POLLS = 1 << 20


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def assembled(prec):
    p = synth.make_pair("plain640", 3, W=W, H=H)
    al = synth.random_alpha(W, H, 4)
    ctx = api.sf_create(W, H, 1, 3, 3, 8, factor_precision=prec)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    return ctx


def solved(ctx):
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-10, 500)
    return code, sw, rr, U.cpu().numpy()


def local_rhs(ctx, sub, seed):
    x0, x1, y0, y1 = api.sf_subdomain_geometry(ctx, sub)["box"]
    n = 3 * (x1 - x0) * (y1 - y0)
    return dev(np.random.default_rng(seed).standard_normal(n)), n


@pytest.mark.parametrize("prec", [api.SF_FP64, api.SF_FP32_FACTOR])
def test_abandoned_waits_then_recovery(gpu, prec):
    ref_ctx = assembled(prec)
    api.sf_factor_subdomains(ref_ctx)
    ref = solved(ref_ctx)
    assert ref[0] == api.SF_OK
    b, n = local_rhs(ref_ctx, 4, 11)
    x_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    api.sf_subdomain_solve(ref_ctx, 4, b, x_ref)
    ref_ctx.close()

    ctx = assembled(prec)
    with pytest.raises(api.SfError) as e:
        api.sf_set_wait_limit(ctx, -1)
    assert e.value.code == api.SF_ERR_INVALID
    # the factorisation's ranks and pivot server wait on each other at every
    # pivot step: with no polls allowed the launch is abandoned
    api.sf_set_wait_limit(ctx, 0)
    with pytest.raises(api.SfError) as e:
        api.sf_factor_subdomains(ctx)
    assert e.value.code == api.SF_ERR_DEVICE
    assert 0 <= e.value.detail["subdomain"] < 9
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SfError) as e:           # back to assembled
        api.sf_schwarz_solve(ctx, U, 1e-10, 500)
    assert e.value.code == api.SF_ERR_STATE

    api.sf_set_wait_limit(ctx, DEFAULT_POLLS)
    api.sf_factor_subdomains(ctx)
    # solves and a local solve with no polls allowed: abandoned, or (every
    # wait satisfied at once) complete
    api.sf_set_wait_limit(ctx, 0)
    outcomes = []
    for solve in (api.sf_schwarz_solve, api.sf_schwarz_solve_graph):
        U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
        try:
            code, sw, rr = solve(ctx, U, 1e-10, 500)
            outcomes.append(code)
            assert (code, sw, rr) == ref[:3] and np.array_equal(U.cpu().numpy(), ref[3])
        except api.SfError as err:
            assert err.code == api.SF_ERR_DEVICE
            outcomes.append(err.code)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    try:
        api.sf_subdomain_solve(ctx, 4, b, x)
        outcomes.append(api.SF_OK)
        assert torch.equal(x, x_ref)
    except api.SfError as err:
        assert err.code == api.SF_ERR_DEVICE
        outcomes.append(err.code)
    print("outcomes with no polls allowed:", outcomes)

    # the default bound again: the factors stayed usable
    api.sf_set_wait_limit(ctx, DEFAULT_POLLS)
    got = solved(ctx)
    assert got[:3] == ref[:3]
    assert np.array_equal(got[3], ref[3])
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve_graph(ctx, U, 1e-10, 500)
    assert (code, sw, rr) == ref[:3] and np.array_equal(U.cpu().numpy(), ref[3])
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    api.sf_subdomain_solve(ctx, 4, b, x)
    assert torch.equal(x, x_ref)
    # and a refactorisation gives the same factors
    api.sf_factor_subdomains(ctx)
    got = solved(ctx)
    assert got[:3] == ref[:3] and np.array_equal(got[3], ref[3])
    ctx.close()
