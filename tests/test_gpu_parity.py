"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance (FP64 path): 1e-10 relative, the bar the method is held to; most
quantities agree far closer and are tested tighter.  Iterates are compared at
equal sweep counts.
"""
import numpy as np
import pytest

from oracle import adapt, fem, pipeline, schwarz
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

CASES = {
    "plain64": dict(kind="plain64", seed=1, W=64, H=64, px=2, py=2, d=4),        # 64x64, 2x2, overlap 4
    "ragged": dict(kind="plain64", seed=5, W=37, H=29, px=3, py=2, d=5),         # uneven tiles, odd overlap
    "tall": dict(kind="plain64", seed=6, W=23, H=41, px=2, py=3, d=6),           # line orientation mix
    "noisy": dict(kind="plain640", seed=3, W=72, H=56, px=3, py=3, d=8),         # 640x480 recipe, cropped
    "single": dict(kind="plain64", seed=8, W=9, H=12, px=1, py=1, d=0),          # one line tile (m <= 32)
}
# line matrices above 384 x 384 (13 block rows): the factor's ranks split by column parity
WIDE = dict(kind="plain640", seed=4, W=300, H=136, px=2, py=1, d=8)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def interleave(Ufield):
    """[3, H, W] field planes -> oracle node-interleaved [3N]."""
    return np.ascontiguousarray(Ufield.transpose(1, 2, 0)).reshape(-1)


def planes(Uint, W, H):
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


def setup(case, alpha=None, band_tile=0, lam=1.0):
    p = synth.make_pair(case["kind"], case["seed"], W=case["W"], H=case["H"])
    W, H = case["W"], case["H"]
    al = synth.constant_alpha(W, H) if alpha is None else alpha
    ctx = api.sf_create(W, H, 1, case["px"], case["py"], case["d"], lam=lam, band_tile=band_tile)
    I0, I1, A = dev(p.I0[None]), dev(p.I1[None]), dev(al[None])
    api.sf_assemble(ctx, I0, I1, A)
    return p, al, ctx, (I0, I1, A)


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_and_residual_match_oracle(gpu, name):
    case = CASES[name]
    p, al, ctx, _ = setup(case, alpha=synth.random_alpha(case["W"], case["H"], 3))
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    Fg = torch.empty(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_rhs(ctx, Fg)
    Fo = planes(F, case["W"], case["H"])
    assert np.abs(host(Fg)[0] - Fo).max() <= 1e-14 * np.abs(Fo).max()
    U = np.random.default_rng(7).normal(size=A.shape[0])
    Ug = dev(planes(U, case["W"], case["H"])[None])
    rg = torch.empty_like(Ug)
    n2 = api.sf_residual(ctx, Ug, rg)
    ro = planes(F - A @ U, case["W"], case["H"])
    assert np.abs(host(rg)[0] - ro).max() <= 1e-13 * np.abs(ro).max()
    assert n2[0] == pytest.approx(float(np.sum(ro ** 2)), rel=1e-12)


@pytest.mark.parametrize("name", ["plain64", "ragged", "tall", "single", "wide"])
def test_subdomain_solves_match_lapack(gpu, name):
    case = WIDE if name == "wide" else CASES[name]
    p, al, ctx, _ = setup(case)
    api.sf_factor_subdomains(ctx)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    subs = schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"])
    facs = schwarz.factor_subdomains(A, subs)
    rng = np.random.default_rng(11)
    for i, fac in enumerate(facs):
        b = rng.normal(size=fac.sub.n)
        x = torch.empty(fac.sub.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        xo = schwarz.local_solve(fac, b)
        assert rel(host(x), xo) <= 1e-12, (i, rel(host(x), xo))


@pytest.mark.parametrize("name", list(CASES))
def test_ras_iterates_match_oracle(gpu, name):
    case = CASES[name]
    nsw = 20
    p, al, ctx, _ = setup(case)
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 0.0, nsw)
    assert sw == [nsw] and code == api.SF_NOT_CONVERGED
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"]))
    res = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=nsw)
    Uo = planes(res.U, case["W"], case["H"])
    assert emax(host(U)[0], Uo) <= 1e-10
    assert rr[0] == pytest.approx(res.relres, rel=1e-8)


@pytest.mark.parametrize("name,band_tile", [("ragged", 1), ("ragged", 2), ("plain64", 2), ("plain64", 3),
                                            ("plain64", 4), ("noisy", 3), ("ragged", 9)])
def test_workgroups_per_subdomain_variants(gpu, name, band_tile):
    # P workgroups per subdomain, at most one per 32-row block of a line matrix
    case = CASES[name]
    p, al, ctx, _ = setup(case, band_tile=band_tile)
    nblk = min((3 * min(s.box[1] - s.box[0], s.box[3] - s.box[2]) + 31) // 32
               for s in schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"]))
    assert api.sf_subdomain_geometry(ctx, 0)["P"] == min(band_tile, nblk)
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, 12)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"]))
    res = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=12)
    assert emax(host(U)[0], planes(res.U, case["W"], case["H"])) <= 1e-10


def test_solve_to_tolerance_and_determinism(gpu):
    case = CASES["plain64"]
    p, al, ctx, _ = setup(case)
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 500)
    assert code == api.SF_OK and rr[0] <= 1e-8
    U2 = torch.zeros_like(U)
    code2, sw2, rr2 = api.sf_schwarz_solve(ctx, U2, 1e-8, 500)
    assert sw2 == sw and torch.equal(U, U2)            # bitwise reproducible
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"]))
    res = schwarz.ras_solve(A, F, facs, rtol=1e-8, max_sweeps=500)
    assert abs(res.sweeps - sw[0]) <= 1
    res = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=sw[0])
    assert emax(host(U)[0], planes(res.U, case["W"], case["H"])) <= 1e-10
    # the oracle's own residual of the GPU iterate
    Ug = interleave(host(U)[0])
    assert np.linalg.norm(F - A @ Ug) / np.linalg.norm(F) <= 1.0000001e-8


def test_batch_equals_single(gpu):
    cases = [CASES["ragged"], dict(CASES["ragged"], seed=9)]
    W, H = cases[0]["W"], cases[0]["H"]
    pairs = [synth.make_pair(c["kind"], c["seed"], W=W, H=H) for c in cases]
    als = [synth.random_alpha(W, H, 1), synth.constant_alpha(W, H)]
    ctx = api.sf_create(W, H, 2, 3, 2, 5, band_tile=2)
    I0 = dev(np.stack([q.I0 for q in pairs]))
    I1 = dev(np.stack([q.I1 for q in pairs]))
    Al = dev(np.stack(als))
    api.sf_assemble(ctx, I0, I1, Al)
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-7, 400)
    assert code == api.SF_OK
    for b in range(2):
        c1 = api.sf_create(W, H, 1, 3, 2, 5, band_tile=2)
        api.sf_assemble(c1, I0[b:b + 1].contiguous(), I1[b:b + 1].contiguous(), Al[b:b + 1].contiguous())
        api.sf_factor_subdomains(c1)
        U1 = torch.zeros(c1.field_shape(), dtype=torch.float64, device="cuda")
        _, sw1, rr1 = api.sf_schwarz_solve(c1, U1, 1e-7, 400)
        assert sw1[0] == sw[b] and torch.equal(U1[0], U[b])


@pytest.mark.parametrize("name", ["plain64", "noisy"])
def test_indicator_and_alpha_update(gpu, name):
    case = CASES[name]
    p, al, ctx, (I0, I1, Al) = setup(case, alpha=synth.random_alpha(case["W"], case["H"], 2))
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    Uo = schwarz.dense_solve(A, F) if A.shape[0] < 20000 else np.random.default_rng(1).normal(size=A.shape[0]) * 0.1
    Ug = dev(planes(Uo, case["W"], case["H"])[None])
    eta = torch.empty(ctx.alpha_shape(), dtype=torch.float64, device="cuda")
    api.sf_indicator(ctx, Ug, eta)
    eo = adapt.indicator(p.I0, p.I1, al, 1.0, Uo)
    assert np.abs(host(eta)[0] - eo).max() <= 1e-12 * eo.max()
    em = api.sf_update_alpha(ctx, Ug, Al, kappa=1.0, eta_thr=0.1, alpha_th=1e-3)
    ao, mo = adapt.update_alpha(al, eo, 1.0, 0.1, 1e-3)
    assert em[0] == pytest.approx(mo, rel=1e-12)
    assert np.abs(host(Al)[0] - ao).max() <= 1e-12 * ao.max()


def test_adaptive_pipeline_matches_oracle(gpu):
    case = CASES["plain64"]
    W, H = case["W"], case["H"]
    p = synth.make_pair(case["kind"], case["seed"], W=W, H=H)
    al0 = synth.constant_alpha(W, H)
    ctx = api.sf_create(W, H, 1, case["px"], case["py"], case["d"])
    Al = dev(al0[None])
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    res = api.run_pipeline(ctx, dev(p.I0[None]), dev(p.I1[None]), Al, U, rtol=1e-8, max_sweeps=500, passes=2)
    counts = [s[0] for s in res.sweeps]
    ores = pipeline.solve_pair(p.I0, p.I1, al0, 1.0, case["px"], case["py"], case["d"], 0.0, 0, passes=2,
                               sweeps_per_solve=counts)
    assert emax(host(Al)[0], ores.alpha) <= 1e-10
    assert emax(host(U)[0], planes(ores.U, W, H)) <= 1e-10
    assert all(r <= 1e-8 for r in (rr[0] for rr in res.relres))


def test_identical_frames_zero_flow(gpu):
    case = CASES["ragged"]
    p = synth.make_pair(case["kind"], case["seed"], W=case["W"], H=case["H"])
    ctx = api.sf_create(case["W"], case["H"], 1, case["px"], case["py"], case["d"])
    I0 = dev(p.I0[None])
    api.sf_assemble(ctx, I0, I0.clone(), dev(synth.constant_alpha(case["W"], case["H"])[None]))
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 50)
    assert code == api.SF_OK and sw == [0] and rr == [0.0]
    assert torch.count_nonzero(U).item() == 0


def test_constant_gain_and_linear_fixed_point(gpu):
    W, H = 30, 26
    c = 0.07
    p = synth.gain_pair(W, H, c)
    ctx = api.sf_create(W, H, 1, 2, 2, 4)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(synth.random_alpha(W, H, 4)[None]))
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-12, 2000)
    Uh = host(U)[0]
    assert code == api.SF_OK
    assert np.abs(Uh[:2]).max() < 1e-9 and np.abs(Uh[2] - c).max() < 1e-9
    # translated linear image: the true flow is a fixed point of a sweep
    w = (0.3, 0.45)
    q = synth.linear_pair(W, H, 0.2, 0.1, w=w)
    ctx2 = api.sf_create(W, H, 1, 2, 2, 4)
    api.sf_assemble(ctx2, dev(q.I0[None]), dev(q.I1[None]), dev(synth.constant_alpha(W, H)[None]))
    api.sf_factor_subdomains(ctx2)
    Ut = np.zeros((1, 3, H, W))
    Ut[0, 0], Ut[0, 1] = w
    U2 = dev(Ut)
    api.sf_schwarz_solve(ctx2, U2, 0.0, 1)
    assert np.abs(host(U2) - Ut).max() < 1e-11


def test_error_statuses(gpu):
    W, H = 20, 16
    p = synth.make_pair("plain64", 2, W=W, H=H)
    ctx = api.sf_create(W, H, 1, 2, 2, 4)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SfError) as e:
        api.sf_factor_subdomains(ctx)
    assert e.value.code == api.SF_ERR_STATE
    bad = p.I0.copy()
    bad[3, 4] = np.nan
    with pytest.raises(api.SfError) as e:
        api.sf_assemble(ctx, dev(bad[None]), dev(p.I1[None]), dev(synth.constant_alpha(W, H)[None]))
    assert e.value.code == api.SF_NONFINITE
    al = synth.constant_alpha(W, H)
    al[2, 3, 1] = 0.0
    with pytest.raises(api.SfError) as e:
        api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    assert e.value.code == api.SF_ERR_INVALID
    with pytest.raises(api.SfError) as e:
        api.sf_schwarz_solve(ctx, U, 1e-8, 10)
    assert e.value.code == api.SF_ERR_STATE
    # a flat image with a single subdomain: constants are in the kernel of A
    flat = np.full((1, H, W), 0.5)
    c1 = api.sf_create(W, H, 1, 1, 1, 0)
    api.sf_assemble(c1, dev(flat), dev(flat), dev(synth.constant_alpha(W, H)[None]))
    with pytest.raises(api.SfError) as e:
        api.sf_factor_subdomains(c1)
    assert e.value.code == api.SF_NOT_SPD
    assert e.value.detail["pair"] == 0 and e.value.detail["subdomain"] == 0
    # max_sweeps reached above tolerance: status, iterate still written
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(synth.constant_alpha(W, H)[None]))
    api.sf_factor_subdomains(ctx)
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-14, 1)
    assert code == api.SF_NOT_CONVERGED and sw == [1] and torch.count_nonzero(U).item() > 0
