"""GPU edge cases through the C ABI against the oracle: the smallest meshes,
one-pixel-wide parts, overlaps wider than a part, the largest line matrix
the library takes (768 unknowns; and the first one it refuses), and a batch in which one
pair has nothing to solve."""
import numpy as np
import pytest

from oracle import fem, schwarz
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
    """Largest element-wise difference of field planes [..., 3, H, W] (or any
    array), each field relative to its own largest magnitude."""
    a, b = np.asarray(a), np.asarray(b)
    if a.ndim >= 3 and a.shape[-3] == 3:
        return max(float(np.abs(a[..., c, :, :] - b[..., c, :, :]).max() / max(np.abs(b[..., c, :, :]).max(), 1e-300))
                   for c in range(3))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def frames(W, H, seed):
    rng = np.random.default_rng(seed)
    I0 = rng.random((H, W))
    I1 = np.clip(I0 + 0.05 * rng.normal(size=(H, W)), 0.0, 1.0)
    return I0, I1


@pytest.mark.parametrize("W,H,px,py,d", [
    (2, 2, 1, 1, 0),        # one cell, two triangles, four nodes
    (2, 7, 1, 2, 1),        # a two-node-wide strip
    (6, 8, 6, 1, 1),        # one-pixel-wide parts
    (9, 6, 3, 2, 6),        # overlap wider than a part
])
def test_small_and_degenerate_meshes(gpu, W, H, px, py, d):
    I0, I1 = frames(W, H, W * 100 + H)
    al = synth.random_alpha(W, H, 7)
    ctx = api.sf_create(W, H, 1, px, py, d)
    api.sf_assemble(ctx, dev(I0[None]), dev(I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, 6)
    A, F = fem.assemble(I0, I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, px, py, d))
    Uo = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=6).U
    assert emax(host(U)[0], planes(Uo, W, H)) <= 1e-10
    ctx.close()


def test_largest_line_matrix(gpu):
    # lines of 256 nodes: m = 768 unknowns, the largest taken
    W, H = 264, 256
    I0, I1 = frames(W, H, 4)
    al = synth.constant_alpha(W, H)
    ctx = api.sf_create(W, H, 1, 1, 1, 0)
    g = api.sf_subdomain_geometry(ctx, 0)
    assert g["box"] == (0, W, 0, H) and g["cols"]
    api.sf_assemble(ctx, dev(I0[None]), dev(I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    A, F = fem.assemble(I0, I1, al, 1.0)
    fac = schwarz.factor_subdomains(A, schwarz.decompose(W, H, 1, 1, 0))[0]
    b = np.random.default_rng(2).normal(size=fac.sub.n)
    x = torch.empty(fac.sub.n, dtype=torch.float64, device="cuda")
    api.sf_subdomain_solve(ctx, 0, dev(b), x)
    assert rel(host(x), schwarz.local_solve(fac, b)) <= 1e-12
    # one sweep of the single subdomain is the exact solve
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-12, 3)
    assert code == api.SF_OK and sw[0] == 1
    ctx.close()


def test_first_refused_line_matrix(gpu):
    # lines of 257 nodes would need 771 unknowns per line
    with pytest.raises(api.SfError) as e:
        api.sf_create(260, 257, 1, 1, 1, 0)
    assert e.value.code == api.SF_ERR_INVALID


def test_batch_with_a_pair_that_has_nothing_to_solve(gpu):
    W, H = 40, 30
    p = synth.make_pair("plain64", 4, W=W, H=H)
    I0 = dev(np.stack([p.I0, p.I0]))
    I1 = dev(np.stack([p.I1, p.I0]))           # second pair: identical frames, F = 0
    Al = dev(np.stack([synth.constant_alpha(W, H)] * 2))
    ctx = api.sf_create(W, H, 2, 2, 2, 4)
    api.sf_assemble(ctx, I0, I1, Al)
    api.sf_factor_subdomains(ctx)
    U = torch.ones(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-9, 500)
    assert code == api.SF_OK and sw[1] == 0 and rr[1] == 0.0 and sw[0] > 0
    assert float(U[1].abs().max()) == 0.0
    A, F = fem.assemble(p.I0, p.I1, synth.constant_alpha(W, H), 1.0)
    Ug = np.ascontiguousarray(host(U)[0].transpose(1, 2, 0)).reshape(-1)
    assert np.linalg.norm(F - A @ Ug) <= 1.0001e-9 * np.linalg.norm(F)
    ctx.close()
