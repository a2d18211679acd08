"""GPU parity for the wide-line paths: line matrices above 384 (the factor's
split ranks, the one-row fast sweep, up to the largest line of 768 unknowns)
and launches split into chunks of subdomains, through the C ABI against the
FP64 oracle (LAPACK banded Cholesky local solves, RAS iterates)."""
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
    """Largest element-wise difference of field planes [3, H, W], each field
    relative to its own largest magnitude."""
    return max(float(np.abs(a[c] - b[c]).max() / max(np.abs(b[c]).max(), 1e-300)) for c in range(3))


# (W, H, parts_x, parts_y, overlap): nodes per line -> block rows NT of a line matrix
GEOMS = {
    "nt13": (272, 136, 2, 1, 8),     # 136-node lines, m = 408: factor ranks split by column parity, two-row sweep
    "nt16": (348, 170, 2, 1, 8),     # 170-node lines, m = 510: one block row per sweep rank
    "nt24": (256, 516, 1, 2, 8),     # 256-node lines, m = 768: the largest line matrix
}


@pytest.mark.parametrize("name", list(GEOMS))
def test_wide_lines_local_solves_and_iterates(gpu, name):
    W, H, px, py, d = GEOMS[name]
    print(f"wide lines {name}: {W}x{H} {px}x{py} overlap {d}", flush=True)
    p = synth.make_pair("plain640", 21, W=W, H=H)
    al = synth.random_alpha(W, H, 5)
    ctx = api.sf_create(W, H, 1, px, py, d)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    subs = schwarz.decompose(W, H, px, py, d)
    facs = schwarz.factor_subdomains(A, subs)
    rng = np.random.default_rng(3)
    for i, fac in enumerate(facs):
        b = rng.normal(size=fac.sub.n)
        x = torch.empty(fac.sub.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        xg = host(x)
        # the solve itself: backward error at the rounding level of the
        # substitutions; against LAPACK's banded Cholesky the forward
        # difference of two backward-stable solves, which grows with the
        # conditioning of these 100-200 K unknown subdomains (1e-12 measured
        # at 768-unknown lines): the FP64 parity bar
        Ai = schwarz.local_matrix(A, fac.sub)
        assert np.linalg.norm(b - Ai @ xg) <= 1e-13 * np.linalg.norm(b), i
        assert rel(xg, schwarz.local_solve(fac, b)) <= 1e-10, i
    nsw = 20
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, nsw)
    res = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=nsw)
    assert emax(host(U)[0], planes(res.U, W, H)) <= 1e-10
    ctx.close()


def test_chunked_factor_and_sweep_launches(gpu):
    # 256 subdomains: the factor runs in chunks of at most 64 subdomains that
    # reuse workspace slots, the sweep in more than one launch per sweep
    W, H, px, py, d = 128, 128, 16, 16, 4
    p = synth.make_pair("plain64", 31, W=W, H=H)
    al = synth.random_alpha(W, H, 9)
    ctx = api.sf_create(W, H, 1, px, py, d)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    subs = schwarz.decompose(W, H, px, py, d)
    facs = schwarz.factor_subdomains(A, subs)
    rng = np.random.default_rng(4)
    for i in (0, 63, 64, 127, 128, 200, 255):
        b = rng.normal(size=facs[i].sub.n)
        x = torch.empty(facs[i].sub.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        assert rel(host(x), schwarz.local_solve(facs[i], b)) <= 1e-12, i
    nsw = 10
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, nsw)
    res = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=nsw)
    assert emax(host(U)[0], planes(res.U, W, H)) <= 1e-10
    # the graph-replayed loop runs the same chunked launches
    Ug = torch.zeros_like(U)
    api.sf_schwarz_solve_graph(ctx, Ug, 0.0, nsw)
    assert torch.equal(Ug, U)
    ctx.close()


def test_factor_launch_tail(gpu):
    # 164-168-node lines (16 block rows): a subdomain's factor takes 17 co-resident
    # workgroups (16 split ranks and the pivot server), so a launch holds 8
    # subdomains side by side (one XCD each) and the ninth on the workgroups
    # left over, its ranks spread over XCDs.  Every local solve to the FP64
    # backward-error bar, and the solve to 1e-8
    W = H = 480
    p = synth.make_pair("plain640", 23, W=W, H=H)
    al = synth.random_alpha(W, H, 6)
    ctx = api.sf_create(W, H, 1, 3, 3, 8)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    A, _ = fem.assemble(p.I0, p.I1, al, 1.0)
    subs = schwarz.decompose(W, H, 3, 3, 8)
    assert {-(-3 * min(s.box[1] - s.box[0], s.box[3] - s.box[2]) // 32) for s in subs} == {16}
    rng = np.random.default_rng(8)
    for i, s in enumerate(subs):
        b = rng.normal(size=s.n)
        x = torch.empty(s.n, dtype=torch.float64, device="cuda")
        api.sf_subdomain_solve(ctx, i, dev(b), x)
        Ai = schwarz.local_matrix(A, s)
        assert np.linalg.norm(b - Ai @ host(x)) <= 1e-13 * np.linalg.norm(b), i
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, rr = api.sf_schwarz_solve(ctx, U, 1e-8, 500)
    assert code == api.SF_OK and rr[0] <= 1e-8
    ctx.close()


def test_sweep_launch_tail_matches_oracle(gpu):
    # 5x5 subdomains of 6 block rows, 5 sweep workgroups per chain, two
    # chains: 10 co-resident workgroups per subdomain, so a sweep launch holds
    # 24 subdomains side by side in groups of 8 (one XCD each) and the 25th on
    # the workgroups left over, its ranks spread over XCDs (device-scope
    # exchange).  20 RAS iterates element by element against the oracle
    W = H = 280
    p = synth.make_pair("plain640", 29, W=W, H=H)
    al = synth.random_alpha(W, H, 7)
    ctx = api.sf_create(W, H, 1, 5, 5, 4, band_tile=5)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(al[None]))
    api.sf_factor_subdomains(ctx)
    geo = api.sf_subdomain_geometry(ctx, 24)
    assert geo["P"] == 5 and geo["chains"] == 2, geo
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, 5, 5, 4))
    nsw = 20
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    api.sf_schwarz_solve(ctx, U, 0.0, nsw)
    res = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=nsw)
    assert emax(host(U)[0], planes(res.U, W, H)) <= 1e-10
    Ug = torch.zeros_like(U)
    api.sf_schwarz_solve_graph(ctx, Ug, 0.0, nsw)
    assert torch.equal(Ug, U)
    ctx.close()
