"""Pins of the oracle's decomposition and Schwarz iteration (Section 3)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import adapt, fem, schwarz
from paper_1508_02977_amd import synth


def _system(W, H, seed=1, lam=1.0, noise=0.01, alpha=None):
    p = synth.make_pair("plain64", seed, W=W, H=H, noise=noise)
    al = synth.constant_alpha(W, H) if alpha is None else alpha
    A, F = fem.assemble(p.I0, p.I1, al, lam)
    return p, A, F


@pytest.mark.parametrize("W,H,px,py,d", [(64, 64, 2, 2, 4), (37, 29, 3, 2, 5), (40, 17, 4, 1, 2), (23, 41, 2, 3, 6)])
def test_decomposition_partition_and_overlap(W, H, px, py, d):
    subs = schwarz.decompose(W, H, px, py, d)
    owner = np.zeros(W * H, dtype=int)
    for s in subs:
        owner[s.nodes[s.own_mask[0::3]]] += 1
        bx0, bx1, by0, by1 = s.box
        assert s.n == 3 * (bx1 - bx0) * (by1 - by0)
        assert s.ms == min(bx1 - bx0, by1 - by0) or (s.cols and s.ms == by1 - by0)
    assert np.all(owner == 1)
    # neighbours share exactly d node columns/rows
    by_tile = {(s.px, s.py): s for s in subs}
    for (p, q), s in by_tile.items():
        if (p + 1, q) in by_tile:
            t = by_tile[(p + 1, q)]
            assert s.box[1] - t.box[0] == d
        if (p, q + 1) in by_tile:
            t = by_tile[(p, q + 1)]
            assert s.box[3] - t.box[2] == d


def test_local_band_width():
    p, A, F = _system(30, 22, noise=0.02)
    for s in schwarz.decompose(30, 22, 2, 2, 4):
        As = schwarz.local_matrix(A, s).tocoo()
        assert np.abs(As.row - As.col).max() <= s.kd
        # the bound is attained: the diagonal neighbour couples at 3*ms + 3 + 2
        assert np.abs(As.row - As.col).max() == s.kd


def test_band_cholesky_solve_equals_dense():
    p, A, F = _system(26, 20)
    subs = schwarz.decompose(26, 20, 2, 2, 4)
    facs = schwarz.factor_subdomains(A, subs)
    rng = np.random.default_rng(0)
    for fac in facs:
        b = rng.normal(size=fac.sub.n)
        x = schwarz.local_solve(fac, b)
        xd = np.linalg.solve(schwarz.local_matrix(A, fac.sub).toarray(), b)
        assert np.allclose(x, xd, rtol=1e-10, atol=1e-12 * np.abs(xd).max())


def test_ras_equals_dirichlet_schwarz():
    # Equation (schwarz): Dirichlet transmission from the previous iterate, glued
    # by ownership, is the restricted additive Schwarz update.
    p, A, F = _system(24, 21, noise=0.02)
    subs = schwarz.decompose(24, 21, 3, 2, 4)
    facs = schwarz.factor_subdomains(A, subs)
    U = np.random.default_rng(5).normal(size=A.shape[0]) * 0.1
    for _ in range(3):
        U1 = schwarz.ras_sweep(A, F, facs, U)
        U2 = schwarz.dirichlet_sweep(A, F, subs, U)
        assert np.abs(U1 - U2).max() <= 1e-12 * max(1.0, np.abs(U2).max())
        U = U1


def test_ras_converges_to_dense_solution():
    p, A, F = _system(20, 16, noise=0.02)
    subs = schwarz.decompose(20, 16, 2, 2, 4)
    facs = schwarz.factor_subdomains(A, subs)
    res = schwarz.ras_solve(A, F, facs, rtol=1e-13, max_sweeps=2000)
    Ud = schwarz.dense_solve(A, F)
    assert res.relres <= 1e-13
    assert np.linalg.norm(res.U - Ud) <= 1e-9 * np.linalg.norm(Ud)
    # the paper's criterion |U^k - U^{k+1}| goes to zero as well
    assert res.increments[-1] < 1e-8 * res.increments[0]


def test_single_subdomain_is_exact_in_one_sweep():
    p, A, F = _system(18, 14, noise=0.02)
    subs = schwarz.decompose(18, 14, 1, 1, 0)
    facs = schwarz.factor_subdomains(A, subs)
    res = schwarz.ras_solve(A, F, facs, rtol=1e-12, max_sweeps=5)
    assert res.sweeps == 1
    assert np.linalg.norm(res.U - schwarz.dense_solve(A, F)) <= 1e-11 * np.linalg.norm(res.U)


def test_larger_overlap_converges_faster():
    # Section 3.2 / Section 4: the rate improves with the size of the overlap.
    p, A, F = _system(48, 40, noise=0.01)
    counts = []
    for d in (2, 4, 8):
        subs = schwarz.decompose(48, 40, 2, 2, d)
        facs = schwarz.factor_subdomains(A, subs)
        counts.append(schwarz.ras_solve(A, F, facs, rtol=1e-6, max_sweeps=3000).sweeps)
    assert counts[0] > counts[1] > counts[2]


def test_zero_rhs_zero_sweeps():
    p = synth.make_pair("plain64", 2, W=16, H=12)
    A, F = fem.assemble(p.I0, p.I0, synth.constant_alpha(16, 12), 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(16, 12, 2, 2, 4))
    res = schwarz.ras_solve(A, F, facs, rtol=1e-8, max_sweeps=50)
    assert res.sweeps == 0 and np.all(res.U == 0.0)


def test_linear_translation_is_fixed_point_and_normal_flow_recovered():
    # Exact recovery: the true flow of a translated linear image is a fixed point
    # of a sweep; from zero, RAS recovers the flow along the gradient.
    W, H = 12, 10
    w = (0.3, 0.45)
    pq = (0.2, 0.1)
    p = synth.linear_pair(W, H, *pq, w=w)
    A, F = fem.assemble(p.I0, p.I1, synth.constant_alpha(W, H), 1.0)
    subs = schwarz.decompose(W, H, 2, 2, 4)
    facs = schwarz.factor_subdomains(A, subs)
    Ut = np.zeros((H * W, 3))
    Ut[:, 0], Ut[:, 1] = w
    U1 = schwarz.ras_sweep(A, F, facs, Ut.ravel())
    assert np.abs(U1 - Ut.ravel()).max() < 1e-11
    ghat = np.array(pq) / np.hypot(*pq)
    res = schwarz.ras_solve(A, F, facs, rtol=1e-12, max_sweeps=5000)
    assert res.relres <= 1e-12
    Ur = res.U.reshape(-1, 3)
    normal = Ur[:, :2] @ ghat
    tangent = Ur[:, :2] @ np.array([-ghat[1], ghat[0]])
    assert np.allclose(normal, np.dot(w, ghat), atol=1e-8)
    assert np.abs(tangent).max() < 1e-8 and np.abs(Ur[:, 2]).max() < 1e-8


def test_subdomain_matrices_spd_even_if_global_singular():
    # A linear image leaves the tangential flow in the kernel of A (aperture
    # problem); each subdomain has a Dirichlet interface, so its matrix is SPD.
    W, H = 14, 12
    p = synth.linear_pair(W, H, 0.03, 0.02)
    A, F = fem.assemble(p.I0, p.I1, synth.constant_alpha(W, H), 1.0)
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() < 1e-12 * ev.max()
    for s in schwarz.decompose(W, H, 2, 2, 4):
        evs = np.linalg.eigvalsh(schwarz.local_matrix(A, s).toarray())
        assert evs.min() > 0.0


# ---- the adaptive driver (Section 2.3 loop): pins of pipeline.solve_pair -----

def test_solve_pair_without_passes_is_one_ras_solve():
    from oracle import pipeline
    W, H = 14, 12
    p = synth.make_pair("plain64", 21, W=W, H=H, noise=0.01)
    al = synth.random_alpha(W, H, 5)
    res = pipeline.solve_pair(p.I0, p.I1, al, 1.0, 2, 2, 2, rtol=1e-9, max_sweeps=500)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, 2, 2, 2))
    ref = schwarz.ras_solve(A, F, facs, rtol=1e-9, max_sweeps=500)
    assert res.sweeps == [ref.sweeps] and np.array_equal(res.U, ref.U)
    assert np.array_equal(res.alpha, al) and res.eta_max == []


def test_solve_pair_warm_start_continues_the_iteration():
    # kappa = 0 leaves alpha unchanged, so the reassembled system is the same
    # and the warm-started second solve continues the first one's iteration:
    # 3 + 4 sweeps equal 7 sweeps of one solve, bit for bit.
    from oracle import pipeline
    W, H = 13, 11
    p = synth.make_pair("plain64", 22, W=W, H=H, noise=0.01)
    al = synth.random_alpha(W, H, 6)
    res = pipeline.solve_pair(p.I0, p.I1, al, 1.0, 2, 2, 3, rtol=0.0, max_sweeps=0, passes=1,
                              kappa=0.0, sweeps_per_solve=[3, 4])
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, 2, 2, 3))
    ref = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=7)
    assert np.array_equal(res.U, ref.U) and np.array_equal(res.alpha, al)


def test_solve_pair_reassembles_with_the_updated_alpha():
    # A 1x1 split solves exactly in one sweep, so with one sweep per solve each
    # solve returns the solution of the system assembled with the current
    # alpha: after two updates U solves A(alpha_2) U = F, and alpha_2 is the
    # decrease rule applied to the indicators of the two earlier exact solutions.
    from oracle import pipeline
    W, H = 10, 9
    p = synth.make_pair("plain64", 23, W=W, H=H, noise=0.01)
    al0 = synth.constant_alpha(W, H, 0.1)
    kw = dict(kappa=1.0, eta_thr=0.1, alpha_th=1e-3)
    res = pipeline.solve_pair(p.I0, p.I1, al0, 1.0, 1, 1, 0, rtol=0.0, max_sweeps=1, passes=2, **kw)
    al = al0
    for _ in range(2):
        A, F = fem.assemble(p.I0, p.I1, al, 1.0)
        U = schwarz.dense_solve(A, F)
        eta = adapt.indicator(p.I0, p.I1, al, 1.0, U)
        al, _ = adapt.update_alpha(al, eta, kw["kappa"], kw["eta_thr"], kw["alpha_th"])
    A2, F2 = fem.assemble(p.I0, p.I1, al, 1.0)
    U2 = schwarz.dense_solve(A2, F2)
    assert not np.allclose(al, al0)
    assert np.allclose(res.alpha, al, rtol=1e-10, atol=0.0)
    assert np.linalg.norm(res.U - U2) <= 1e-10 * np.linalg.norm(U2)
    assert res.sweeps == [1, 1, 1]
