"""GPU: adjoint gradients (sf_adjoint and the autograd wrapper) through the C
ABI against the oracle's adjoint (FP64, 1e-10 relative), plus a central
finite-difference check of the whole differentiable GPU solve."""
import numpy as np
import pytest

from oracle import adjoint, fem, schwarz
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

CASES = [
    dict(kind="plain64", seed=1, W=64, H=64, px=2, py=2, d=4),      # the 64x64 crop
    dict(kind="plain64", seed=1, W=48, H=40, px=2, py=2, d=4),
    dict(kind="plain640", seed=3, W=61, H=37, px=3, py=2, d=5),     # ragged tiles
    dict(kind="plain64", seed=7, W=20, H=26, px=1, py=1, d=0),      # one subdomain
]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def interleave(Ufield):
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


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['W']}x{c['H']}-{c['px']}x{c['py']}")
def test_adjoint_state_and_gradients_match_oracle(gpu, case):
    W, H = case["W"], case["H"]
    p = synth.make_pair(case["kind"], case["seed"], W=W, H=H)
    al = synth.random_alpha(W, H, case["seed"] + 2)
    ctx = api.sf_create(W, H, 1, case["px"], case["py"], case["d"])
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 1e-12, 2000)
    Ug = interleave(host(U)[0])
    w = np.random.default_rng(case["seed"]).normal(scale=0.5, size=(H, W, 2))
    _, G = adjoint.epe_loss(Ug, w)
    # adjoint iterate at an equal sweep count against the oracle's RAS on A P = G
    sweeps = 12
    P = torch.zeros_like(U)
    dI0, dI1 = (torch.empty(ctx.frame_shape(), dtype=torch.float64, device="cuda") for _ in range(2))
    dal = torch.empty(ctx.alpha_shape(), dtype=torch.float64, device="cuda")
    code, sw, _ = api.sf_adjoint(ctx, U, dev(planes(G, W, H)[None]), P, dI0, dI1, dal, 0.0, sweeps)
    assert code == api.SF_NOT_CONVERGED and sw == [sweeps]
    A, _ = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, case["px"], case["py"], case["d"]))
    Po = schwarz.ras_solve(A, G, facs, rtol=0.0, max_sweeps=sweeps).U
    Pg = interleave(host(P)[0])
    assert rel(Pg, Po) <= 1e-10
    # gradients from the same U and P
    o0, o1, oa = adjoint.gradients(p.I0, p.I1, al, 1.0, Ug, Pg)
    assert emax(host(dI0)[0], o0) <= 1e-10
    assert emax(host(dI1)[0], o1) <= 1e-10
    assert emax(host(dal)[0], oa) <= 1e-10
    # a converged adjoint solves A P = G (residual by the oracle's matrix)
    P.zero_()
    code, _, rr = api.sf_adjoint(ctx, U, dev(planes(G, W, H)[None]), P, None, None, None, 1e-12, 4000)
    assert code == api.SF_OK and rr[0] <= 1e-12
    Pc = interleave(host(P)[0])
    assert np.linalg.norm(G - A @ Pc) <= 1e-11 * np.linalg.norm(G)
    ctx.close()


def test_autograd_matches_central_differences(gpu):
    W, H = 24, 18
    p = synth.make_pair("plain64", 2, W=W, H=H)
    al = synth.random_alpha(W, H, 9)
    w = dev(np.random.default_rng(4).normal(scale=0.5, size=(1, 2, H, W)))
    ctx = api.sf_create(W, H, 1, 2, 2, 3)

    def loss(I0, I1, a):
        U = api.schwarz_solve(ctx, I0, I1, a, rtol=1e-13, max_sweeps=5000)
        d = U[:, :2] - w
        return torch.sqrt((d * d).sum(dim=1)).mean()

    I0 = dev(p.I0[None]).requires_grad_()
    I1 = dev(p.I1[None]).requires_grad_()
    A = dev(al[None]).requires_grad_()
    L = loss(I0, I1, A)
    L.backward()
    rng = np.random.default_rng(13)
    h = 1e-6
    with torch.no_grad():
        for name, x, g in (("I0", I0, I0.grad), ("I1", I1, I1.grad), ("alpha", A, A.grad)):
            v = dev(rng.normal(size=tuple(x.shape)))
            if name == "alpha":
                v = v * A                    # relative perturbation keeps alpha > 0
            args = [I0.detach(), I1.detach(), A.detach()]
            k = ("I0", "I1", "alpha").index(name)
            ap, am = list(args), list(args)
            ap[k] = args[k] + h * v
            am[k] = args[k] - h * v
            fd = (float(loss(*ap)) - float(loss(*am))) / (2 * h)
            an = float((g * v).sum())
            assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-2), (name, fd, an)
    ctx.close()


def test_gradients_on_64x64_match_64_central_differences(gpu):
    # 64 random directions per input, h = 1e-6, FP64 solves to 1e-13
    W, H = 64, 64
    p = synth.make_pair("plain64", 1, W=W, H=H)
    al = synth.random_alpha(W, H, 5)
    w = dev(np.random.default_rng(6).normal(scale=0.5, size=(1, 2, H, W)))
    ctx = api.sf_create(W, H, 1, 2, 2, 4)

    def loss(I0, I1, a):
        U = api.schwarz_solve(ctx, I0, I1, a, rtol=1e-13, max_sweeps=5000)
        d = U[:, :2] - w
        return torch.sqrt((d * d).sum(dim=1)).mean()

    I0 = dev(p.I0[None]).requires_grad_()
    I1 = dev(p.I1[None]).requires_grad_()
    A = dev(al[None]).requires_grad_()
    loss(I0, I1, A).backward()
    rng = np.random.default_rng(21)
    h = 1e-6
    worst = 0.0
    with torch.no_grad():
        for k, (x, g) in enumerate(((I0, I0.grad), (I1, I1.grad), (A, A.grad))):
            for _ in range(64):
                v = dev(rng.normal(size=tuple(x.shape)))
                if k == 2:
                    v = v * A
                ap = [I0.detach(), I1.detach(), A.detach()]
                am = list(ap)
                ap[k] = ap[k] + h * v
                am[k] = am[k] - h * v
                fd = (float(loss(*ap)) - float(loss(*am))) / (2 * h)
                an = float((g * v).sum())
                worst = max(worst, abs(fd - an) / max(abs(fd), 1e-2))
    assert worst <= 1e-5, worst
    ctx.close()


def test_fp32_tile_adjoint_agrees_with_fp64(gpu):
    # the FP32-tile form refines against FP64 residuals, so at the same
    # relative residual its gradients agree with the plain form's
    W, H = 96, 80
    p = synth.make_pair("plain640", 4, W=W, H=H)
    al = synth.random_alpha(W, H, 8)
    w = dev(np.random.default_rng(2).normal(scale=0.5, size=(1, 2, H, W)))
    grads = []
    for prec in (api.SF_FP64, api.SF_FP32):
        ctx = api.sf_create(W, H, 1, 3, 2, 6, factor_precision=prec)
        I0 = dev(p.I0[None]).requires_grad_()
        I1 = dev(p.I1[None]).requires_grad_()
        A = dev(al[None]).requires_grad_()
        U = api.schwarz_solve(ctx, I0, I1, A, rtol=1e-12, max_sweeps=5000)
        d = U[:, :2] - w
        torch.sqrt((d * d).sum(dim=1)).mean().backward()
        grads.append([host(t.grad) for t in (I0, I1, A)])
        ctx.close()
    for g64, g32 in zip(*grads):
        assert rel(g32, g64) <= 1e-7


def test_zero_loss_gradient_and_invalid_uses(gpu):
    W, H = 16, 12
    p = synth.make_pair("plain64", 3, W=W, H=H)
    al = synth.constant_alpha(W, H)
    ctx = api.sf_create(W, H, 1, 2, 1, 2)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    P = torch.ones_like(U)
    with pytest.raises(api.SfError):                 # factors are not current
        api.sf_adjoint(ctx, U, torch.zeros_like(U), P)
    api.sf_factor_subdomains(ctx)
    api.sf_schwarz_solve(ctx, U, 1e-12, 500)
    dI0 = torch.full(ctx.frame_shape(), 7.0, dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_adjoint(ctx, U, torch.zeros_like(U), P, dI0)
    assert code == api.SF_OK and sw == [0] and rr == [0.0]
    assert float(P.abs().max()) == 0.0 and float(dI0.abs().max()) == 0.0
    ctx.close()
    smooth = api.sf_create(W, H, 1, 2, 1, 2, sigma=1.0)
    api.sf_assemble(smooth, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(smooth)
    with pytest.raises(api.SfError) as e:
        api.sf_adjoint(smooth, U, torch.zeros_like(U), P)
    assert e.value.code == api.SF_ERR_INVALID
    smooth.close()
