"""GPU: the paper's Gaussian presmoothing of the frames (Section 1) through
the C ABI against the oracle (FP64, 1e-10 relative or tighter)."""
import numpy as np
import pytest

from oracle import adapt, fem, schwarz, variants
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

CASES = [
    dict(kind="plain64", seed=1, W=64, H=64, px=2, py=2, d=4, sigma=1.0),
    dict(kind="plain640", seed=3, W=72, H=56, px=3, py=3, d=8, sigma=2.2),
    dict(kind="plain64", seed=5, W=37, H=29, px=3, py=2, d=5, sigma=0.6),
]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['W']}x{c['H']}-s{c['sigma']}")
def test_presmoothed_rhs_iterates_and_indicator(gpu, case):
    W, H = case["W"], case["H"]
    p = synth.make_pair(case["kind"], case["seed"], W=W, H=H)
    al = synth.random_alpha(W, H, 4)
    ctx = api.sf_create(W, H, 1, case["px"], case["py"], case["d"], sigma=case["sigma"])
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    f0 = variants.presmooth(p.I0, case["sigma"])
    f1 = variants.presmooth(p.I1, case["sigma"])
    A, F = fem.assemble(f0, f1, al, 1.0)
    # right-hand side of the smoothed frames
    Fg = torch.empty(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_rhs(ctx, Fg)
    Fo = F.reshape(H, W, 3).transpose(2, 0, 1)
    assert rel(Fg[0].cpu().numpy(), Fo) <= 1e-13
    # 20 Schwarz sweeps
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, 20)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, case["px"], case["py"], case["d"]))
    Uo = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=20).U
    Ug = np.ascontiguousarray(U[0].cpu().numpy().transpose(1, 2, 0)).reshape(-1)
    d = np.abs(Ug - Uo).reshape(-1, 3).max(axis=0) / np.abs(Uo).reshape(-1, 3).max(axis=0)
    assert d.max() <= 1e-10                      # per field, element by element
    # indicator on the smoothed frames
    eta = torch.empty((1, H - 1, W - 1, 2), dtype=torch.float64, device="cuda")
    api.sf_indicator(ctx, U, eta)
    eo = adapt.indicator(f0, f1, al, 1.0, Ug)
    assert np.abs(eta[0].cpu().numpy() - eo).max() <= 1e-10 * eo.max()
    ctx.close()
