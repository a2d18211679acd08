"""GPU parity of the K_rho (rho > 0) data term through the C ABI against the
FP64 oracle (module clg): right-hand side, residual, local solves, RAS
iterates, the error indicator and the alpha update."""
import numpy as np
import pytest

from oracle import adapt, clg, schwarz
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def planes(Uint, W, H):
    return Uint.reshape(H, W, 3).transpose(2, 0, 1).copy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def emax(a, b):
    return max(float(np.abs(a[c] - b[c]).max() / max(np.abs(b[c]).max(), 1e-300)) for c in range(3))


CASES = [
    # (W, H, parts_x, parts_y, overlap, rho, sigma)
    (48, 40, 2, 2, 4, 1.0, 0.0),
    (37, 29, 3, 2, 5, 0.6, 0.0),       # uneven tiles, radius 2
    (72, 56, 3, 3, 8, 2.2, 0.0),       # radius 7: shifts reach across the border clamp
    (40, 34, 2, 2, 4, 1.5, 1.0),       # with presmoothing of the frames
]


@pytest.mark.parametrize("W,H,px,py,d,rho,sigma", CASES)
def test_clg_rhs_residual_solves_iterates_indicator(gpu, W, H, px, py, d, rho, sigma):
    print(f"clg {W}x{H} {px}x{py} overlap {d} rho {rho} sigma {sigma}", flush=True)
    from oracle import variants
    p = synth.make_pair("plain640", 41, W=W, H=H)
    al = synth.random_alpha(W, H, 6)
    f0, f1 = (variants.presmooth(p.I0, sigma), variants.presmooth(p.I1, sigma)) if sigma > 0 else (p.I0, p.I1)
    A, F = clg.assemble_clg(f0, f1, al, 1.0, rho)
    ctx = api.sf_create(W, H, 1, px, py, d, sigma=sigma, rho=rho)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    Fg = torch.empty(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_rhs(ctx, Fg)
    Fo = planes(F, W, H)
    assert np.abs(host(Fg)[0] - Fo).max() <= 1e-13 * np.abs(Fo).max()
    Ur = np.random.default_rng(2).normal(size=A.shape[0])
    rg = torch.empty_like(Fg)
    n2 = api.sf_residual(ctx, dev(planes(Ur, W, H)[None]), rg)
    ro = planes(F - A @ Ur, W, H)
    assert np.abs(host(rg)[0] - ro).max() <= 1e-12 * np.abs(ro).max()
    assert n2[0] == pytest.approx(float(np.sum(ro ** 2)), rel=1e-11)
    api.sf_factor_subdomains(ctx)
    subs = schwarz.decompose(W, H, px, py, d)
    facs = schwarz.factor_subdomains(A, subs)
    rng = np.random.default_rng(3)
    for i, fac in enumerate(facs):
        b = rng.normal(size=fac.sub.n)
        x = torch.empty(fac.sub.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        assert rel(host(x), schwarz.local_solve(fac, b)) <= 1e-12, i
    nsw = 20
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, nsw)
    Uo = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=nsw).U
    assert emax(host(U)[0], planes(Uo, W, H)) <= 1e-10
    eta = torch.empty(ctx.alpha_shape(), dtype=torch.float64, device="cuda")
    api.sf_indicator(ctx, U, eta)
    Ug = np.ascontiguousarray(host(U)[0].transpose(1, 2, 0)).reshape(-1)
    eo = clg.indicator_clg(f0, f1, al, 1.0, rho, Ug)
    assert np.abs(host(eta)[0] - eo).max() <= 1e-11 * eo.max()
    Al = dev(al[None])
    api.sf_update_alpha(ctx, U, Al)
    ao, _ = adapt.update_alpha(al, eo, 1.0, 0.1, 1e-3)
    assert np.abs(host(Al)[0] - ao).max() <= 1e-12 * ao.max()
    ctx.close()


def test_clg_rho_zero_equals_plain_and_adjoint_refused(gpu):
    W, H = 40, 30
    p = synth.make_pair("plain64", 3, W=W, H=H)
    al = dev(synth.constant_alpha(W, H)[None])
    outs = []
    for rho in (0.0, None):
        ctx = api.sf_create(W, H, 1, 2, 2, 4) if rho is None else api.sf_create(W, H, 1, 2, 2, 4, rho=rho)
        api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), al)
        api.sf_factor_subdomains(ctx)
        U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
        api.sf_schwarz_solve(ctx, U, 0.0, 10)
        outs.append(U)
        ctx.close()
    assert torch.equal(outs[0], outs[1])
    ctx = api.sf_create(W, H, 1, 2, 2, 4, rho=1.0)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), al)
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SfError) as e:
        api.sf_adjoint(ctx, U, U, torch.zeros_like(U))
    assert e.value.code == api.SF_ERR_INVALID
    ctx.close()
