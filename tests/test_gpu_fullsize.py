"""GPU parity at the full size of the timed workload: one 640x480 pair of the
plain640 recipe, 4x4 subdomains with an 8-node overlap (the launch shapes the
benchmark times), FP64, against the oracle on the same seeded input.

The oracle assembles the full system and factors all 16 subdomains (seconds),
so the comparisons are element by element: right-hand side, residual, sampled
local solves, Schwarz iterates at equal sweep counts, the sweep count to
1e-8, the error indicator and the alpha update, and the whole timed step (three
alpha passes, four solves to 1e-8) against the oracle's adaptive driver.
Iterates are compared per field as max |difference| / max |oracle value|.
"""
import numpy as np
import pytest

from oracle import adapt, fem, pipeline, schwarz
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

W, H, PX, PY, D = 640, 480, 4, 4, 8


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def interleave(Ufield):
    return np.ascontiguousarray(Ufield.transpose(1, 2, 0)).reshape(-1)


def planes(Uint):
    return Uint.reshape(H, W, 3).transpose(2, 0, 1).copy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def emax(a, b):
    """Largest element-wise difference of field planes [..., 3, H, W] (or any
    array), each field relative to its own largest magnitude."""
    a, b = np.asarray(a), np.asarray(b)
    if a.ndim >= 3 and a.shape[-3] == 3:
        return max(float(np.abs(a[..., c, :, :] - b[..., c, :, :]).max() / max(np.abs(b[..., c, :, :]).max(), 1e-300))
                   for c in range(3))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def full(gpu):
    p = synth.make_pair("plain640", 2)
    al = synth.constant_alpha(W, H)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    subs = schwarz.decompose(W, H, PX, PY, D)
    facs = schwarz.factor_subdomains(A, subs)
    ctx = api.sf_create(W, H, 1, PX, PY, D)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    yield dict(p=p, al=al, A=A, F=F, subs=subs, facs=facs, ctx=ctx)
    ctx.close()


def test_full_size_launch_shape(full):
    # the shapes the benchmark runs: 16 subdomains, two chains of 8 workgroups each
    # (all 256 CUs: ranks 0-3 own one block row of the 12, ranks 4-7 two)
    ctx = full["ctx"]
    assert api.sf_num_subdomains(ctx) == 16
    g = api.sf_subdomain_geometry(ctx, 5)
    assert g["chains"] == 2 and g["P"] == 8


def test_full_size_rhs_and_residual(full):
    ctx, A, F = full["ctx"], full["A"], full["F"]
    Fg = torch.empty(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_rhs(ctx, Fg)
    Fo = planes(F)
    assert np.abs(host(Fg)[0] - Fo).max() <= 1e-14 * np.abs(Fo).max()
    U = np.random.default_rng(3).normal(size=A.shape[0]) * 0.5
    Ug = dev(planes(U)[None])
    rg = torch.empty_like(Ug)
    n2 = api.sf_residual(ctx, Ug, rg)
    ro = planes(F - A @ U)
    assert np.abs(host(rg)[0] - ro).max() <= 1e-13 * np.abs(ro).max()
    assert n2[0] == pytest.approx(float(np.sum(ro ** 2)), rel=1e-12)


@pytest.mark.parametrize("sub", [0, 5, 10, 15])
def test_full_size_local_solves(full, sub):
    # corner, interior and opposite-corner subdomains against LAPACK's banded Cholesky
    ctx, fac = full["ctx"], full["facs"][sub]
    n = fac.sub.n
    b = np.random.default_rng(sub).normal(size=n)
    xo = schwarz.local_solve(fac, b)
    xg = torch.empty(n, dtype=torch.float64, device="cuda")
    api.sf_subdomain_solve(ctx, sub, dev(b), xg)
    assert rel(host(xg), xo) <= 1e-12


def test_full_size_iterates_sweep_count_indicator(full):
    ctx, A, F, facs, p, al = full["ctx"], full["A"], full["F"], full["facs"], full["p"], full["al"]
    # three sweeps from zero, element by element
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, 3)
    o3 = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=3)
    assert emax(host(U)[0], planes(o3.U)) <= 1e-10
    # to 1e-8 as timed: same number of sweeps, same iterate, oracle residual
    U.zero_()
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 2000)
    assert code == api.SF_OK
    ores = schwarz.ras_solve(A, F, facs, rtol=1e-8, max_sweeps=2000)
    assert sw[0] == ores.sweeps
    Ug = interleave(host(U)[0])
    assert emax(host(U)[0], planes(ores.U)) <= 1e-10
    assert np.linalg.norm(F - A @ Ug) <= 1.0001e-8 * np.linalg.norm(F)
    assert rr[0] == pytest.approx(ores.relres, rel=1e-6)
    # error indicator and alpha update on that iterate
    eta = torch.empty(ctx.alpha_shape(), dtype=torch.float64, device="cuda")
    api.sf_indicator(ctx, U, eta)
    eo = adapt.indicator(p.I0, p.I1, al, 1.0, Ug)
    assert np.abs(host(eta)[0] - eo).max() <= 1e-12 * eo.max()
    Al = dev(al[None])
    em = api.sf_update_alpha(ctx, U, Al, kappa=1.0, eta_thr=0.1, alpha_th=1e-3)
    ao, mo = adapt.update_alpha(al, eo, 1.0, 0.1, 1e-3)
    assert em[0] == pytest.approx(mo, rel=1e-12)
    assert np.abs(host(Al)[0] - ao).max() <= 1e-12 * ao.max()


def test_full_size_fp32_tiles_reach_the_same_residual(full):
    # the chosen form at full size: FP32 tiles refined against FP64 residuals
    p, al, A, F = full["p"], full["al"], full["A"], full["F"]
    ctx = api.sf_create(W, H, 1, PX, PY, D, factor_precision=api.SF_FP32)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 2000)
    assert code == api.SF_OK and rr[0] <= 1e-8
    Ug = interleave(host(U)[0])
    assert np.linalg.norm(F - A @ Ug) <= 1.0001e-8 * np.linalg.norm(F)
    ctx.close()


@pytest.mark.timeout(600)
def test_full_size_timed_pipeline_element_by_element(full):
    # The benchmark's step exactly: assemble, factor, solve to 1e-8, then three
    # times (alpha update from the indicator, refactor, warm-started solve),
    # against the oracle's adaptive driver replaying the GPU's sweep counts.
    p, al = full["p"], full["al"]
    ctx = api.sf_create(W, H, 1, PX, PY, D)
    Al = dev(al[None])
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    res = api.run_pipeline(ctx, dev(p.I0[None]), dev(p.I1[None]), Al, U, rtol=1e-8, max_sweeps=2000, passes=3,
                           kappa=1.0, eta_thr=0.1, alpha_th=1e-3)
    ctx.close()
    counts = [s[0] for s in res.sweeps]
    assert res.status == api.SF_OK and all(r[0] <= 1e-8 for r in res.relres)
    o = pipeline.solve_pair(p.I0, p.I1, al, 1.0, PX, PY, D, rtol=0.0, max_sweeps=0, passes=3, kappa=1.0,
                            eta_thr=0.1, alpha_th=1e-3, sweeps_per_solve=counts)
    # the GPU's stopping points are valid for the oracle's iterates too
    assert all(r <= 1.0001e-8 for r in o.relres)
    for rg, ro in zip(res.relres, o.relres):
        assert rg[0] == pytest.approx(ro, rel=1e-6)
    for eg, eo in zip(res.eta_max, o.eta_max):
        assert eg[0] == pytest.approx(eo, rel=1e-10)
    assert emax(host(U)[0], planes(o.U)) <= 1e-10
    assert emax(host(Al)[0], o.alpha) <= 1e-10
