"""GPU: single-precision storage of the inverse Schur tiles (SF_FP32).

The tiles are computed in FP64, rounded once to FP32 and applied in FP64
arithmetic, so every local solve is inexact; the Schwarz iteration on FP64
residuals removes that error (iterative refinement) and converges to the same
solution U* of A U = F.

Bars:
- a local solve from FP32 tiles agrees with LAPACK's banded Cholesky solve of
  the oracle's subdomain matrix to 1e-5 relative (FP32 rounding, 6e-8, times
  the growth through the line recurrence);
- solved to the same 1e-8 relative residual, the FP32 form's per-field error
  against U* (sparse direct solve of the oracle's A) is at most twice the
  FP64 form's, with at most 2 more sweeps.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, schwarz
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

CASES = {
    "plain64": dict(kind="plain64", seed=1, W=64, H=64, px=2, py=2, d=4),
    "noisy": dict(kind="plain640", seed=3, W=72, H=56, px=3, py=3, d=8),
    # line matrices above 384 x 384 (13 block rows): factor ranks split by column parity
    "wide": dict(kind="plain640", seed=4, W=300, H=136, px=2, py=1, d=8),
    # 170-node lines (16 block rows): one block row per sweep rank
    "wider": dict(kind="plain640", seed=6, W=348, H=170, px=2, py=1, d=8),
}


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def context(case, precision, pivot_tol=0.0):
    p = synth.make_pair(case["kind"], case["seed"], W=case["W"], H=case["H"])
    al = synth.constant_alpha(case["W"], case["H"])
    ctx = api.sf_create(case["W"], case["H"], 1, case["px"], case["py"], case["d"],
                        factor_precision=precision, pivot_tol=pivot_tol)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    return p, al, ctx


@pytest.mark.parametrize("name", ["plain64", "noisy", "wide", "wider"])
def test_fp32_local_solves_match_lapack(gpu, name):
    case = CASES[name]
    p, al, ctx = context(case, api.SF_FP32)
    A, _ = fem.assemble(p.I0, p.I1, al, 1.0)
    subs = schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"])
    facs = schwarz.factor_subdomains(A, subs)
    rng = np.random.default_rng(21)
    worst = 0.0
    for i, fac in enumerate(facs):
        b = rng.normal(size=fac.sub.n)
        x = torch.empty(fac.sub.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        xo = schwarz.local_solve(fac, b)
        worst = max(worst, np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    assert 1e-9 < worst <= 1e-5          # inexact (FP32 storage) but close
    ctx.close()


def field_errors(U, Ustar, W, H):
    Us = Ustar.reshape(H, W, 3).transpose(2, 0, 1)
    return [float(np.linalg.norm(U[c] - Us[c]) / np.linalg.norm(Us[c])) for c in range(3)]


@pytest.mark.parametrize("name", ["plain64", "noisy"])
def test_fp32_refinement_reaches_fp64_accuracy(gpu, name):
    case = CASES[name]
    W, H = case["W"], case["H"]
    p = synth.make_pair(case["kind"], case["seed"], W=W, H=H)
    al = synth.constant_alpha(W, H)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    Ustar = spla.spsolve(A.tocsc(), F)
    out = {}
    for prec in (api.SF_FP64, api.SF_FP32):
        _, _, ctx = context(case, prec)
        U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
        code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 2000)
        assert code == api.SF_OK and rr[0] <= 1e-8
        Ug = U[0].cpu().numpy()
        # the oracle's own residual of the GPU iterate
        r = F - A @ np.ascontiguousarray(Ug.transpose(1, 2, 0)).reshape(-1)
        assert np.linalg.norm(r) / np.linalg.norm(F) <= 1.0000001e-8
        out[prec] = (sw[0], field_errors(Ug, Ustar, W, H))
        ctx.close()
    sw64, e64 = out[api.SF_FP64]
    sw32, e32 = out[api.SF_FP32]
    assert sw32 <= sw64 + 2
    for c in range(3):
        assert e32[c] <= 2.0 * e64[c] + 1e-14, (c, e32, e64)


# ---- the factorisation in FP32 arithmetic (SF_FP32_FACTOR) -----------------

def local_solve_errors(case, ctx):
    p = synth.make_pair(case["kind"], case["seed"], W=case["W"], H=case["H"])
    al = synth.constant_alpha(case["W"], case["H"])
    A, _ = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(case["W"], case["H"], case["px"], case["py"], case["d"]))
    rng = np.random.default_rng(22)
    errs = []
    for i, fac in enumerate(facs):
        b = rng.normal(size=fac.sub.n)
        x = torch.empty(fac.sub.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        xo = schwarz.local_solve(fac, b)
        errs.append(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    return errs


@pytest.mark.parametrize("name", ["plain64", "noisy", "wide", "wider"])
def test_fp32_factor_local_solves(gpu, name):
    # FP32 arithmetic throughout the factorisation: an inexact local solve, a
    # few digits less accurate than FP64 arithmetic with FP32 storage; no
    # subdomain falls back to FP64 on these well-posed pairs
    case = CASES[name]
    _, _, ctx = context(case, api.SF_FP32_FACTOR)
    assert api.sf_factor_fallbacks(ctx) == 0
    errs = local_solve_errors(case, ctx)
    print(name, "FP32 factor local solve errors", max(errs))
    assert 1e-9 < max(errs) <= 1e-3
    ctx.close()


def test_fp32_factor_fallback_to_fp64(gpu):
    # a pivot threshold that every FP32 pivot fails: every subdomain is
    # factored again in FP64 arithmetic, so the local solves have the accuracy
    # of FP32 storage alone
    case = CASES["noisy"]
    _, _, ctx = context(case, api.SF_FP32_FACTOR, pivot_tol=0.999)
    assert api.sf_factor_fallbacks(ctx) == api.sf_num_subdomains(ctx)
    errs = local_solve_errors(case, ctx)
    assert max(errs) <= 1e-5
    ctx.close()


@pytest.mark.parametrize("name", ["plain64", "noisy", "wide"])
def test_fp32_factor_refinement_reaches_fp64_accuracy(gpu, name):
    # at the same 1e-8 relative residual the error against the exact solution
    # is at most twice that of the FP64 form
    case = CASES[name]
    W, H = case["W"], case["H"]
    p = synth.make_pair(case["kind"], case["seed"], W=W, H=H)
    al = synth.constant_alpha(W, H)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    Ustar = spla.spsolve(A.tocsc(), F)
    out = {}
    for prec in (api.SF_FP64, api.SF_FP32_FACTOR):
        _, _, ctx = context(case, prec)
        U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
        code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 2000)
        assert code == api.SF_OK and rr[0] <= 1e-8
        Ug = U[0].cpu().numpy()
        r = F - A @ np.ascontiguousarray(Ug.transpose(1, 2, 0)).reshape(-1)
        assert np.linalg.norm(r) / np.linalg.norm(F) <= 1.0000001e-8
        out[prec] = (sw[0], field_errors(Ug, Ustar, W, H))
        ctx.close()
    sw64, e64 = out[api.SF_FP64]
    sw32, e32 = out[api.SF_FP32_FACTOR]
    print(name, "sweeps", sw64, sw32, "errors", e64, e32)
    assert sw32 <= sw64 + 5
    for c in range(3):
        assert e32[c] <= 2.0 * e64[c] + 1e-14, (c, e32, e64)
