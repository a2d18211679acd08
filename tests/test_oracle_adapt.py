"""Pins of the oracle's error indicator and alpha rule (Section 2.3) and metrics."""
import numpy as np
import pytest

from oracle import adapt, fem, metrics, schwarz
from paper_1508_02977_amd import synth


def _residual_by_moments(I0, I1, U):
    """int_K (s + f_t)^2 by expanding the square into barycentric moments
    int l0^a l1^b l2^c = 2|K| a! b! c! / (a+b+c+2)! (independent of the rule
    the oracle uses)."""
    H, W = I0.shape
    ed = fem.element_data(I0, I1, W, H)
    K = 0.5
    M, T, Q = (fem.product_table(k, K) for k in (2, 3, 4))
    Uv = np.asarray(U).reshape(-1, 3)[ed["tri"]]
    g, fv, ftv = ed["g"], ed["fv"], ed["ftv"]
    lv = g[:, 0:1] * Uv[:, :, 0] + g[:, 1:2] * Uv[:, :, 1] + ftv
    mv = Uv[:, :, 2]
    return (np.einsum("ei,ij,ej->e", lv, M, lv)
            - 2.0 * np.einsum("ei,ijk,ej,ek->e", lv, T, fv, mv)
            + np.einsum("ei,ej,ijkl,ek,el->e", fv, mv, Q, fv, mv))


def test_element_residual_exact_vs_moment_expansion():
    p = synth.make_pair("plain64", 9, W=11, H=9, noise=0.02)
    U = np.random.default_rng(2).normal(size=3 * 99)
    a = adapt.element_residual_integral(p.I0, p.I1, U)
    b = _residual_by_moments(p.I0, p.I1, U)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-15 * b.max())


def test_indicator_zero_for_identical_frames():
    # Identical frames: F = 0, U = 0, no residual and no gradient anywhere, so
    # eta = 0 exactly and the rule leaves alpha unchanged.
    W, H = 12, 10
    p = synth.make_pair("plain64", 3, W=W, H=H)
    al = synth.random_alpha(W, H, 1)
    eta = adapt.indicator(p.I0, p.I0, al, 1.0, np.zeros(3 * W * H))
    assert np.all(eta == 0.0)
    al2, m = adapt.update_alpha(al, eta, 1.0, 0.1, 1e-3)
    assert m == 0.0 and np.array_equal(al2, al)


def test_indicator_vanishes_for_constant_gain():
    # Constant gain: the exact solution (0, 0, c) fits (OF2) pointwise and has no
    # gradient, so eta is at the rounding level of the pointwise residual.
    W, H = 12, 10
    c = 0.08
    p = synth.gain_pair(W, H, c)
    U = np.zeros((H * W, 3))
    U[:, 2] = c
    eta = adapt.indicator(p.I0, p.I1, synth.random_alpha(W, H, 1), 1.0, U.ravel())
    assert np.abs(eta).max() < 1e-14


def test_jump_term_closed_form_linear_flow():
    # Flat image (no data term): for u1 = a x + b y and constant alpha the flux is
    # constant, interior jumps vanish and border edges carry alpha |grad u1 . n|,
    # so eta_K = 1/2 sum_{border edges} alpha^{1/2} |grad u1 . n| h_e.
    W, H = 7, 6
    a, b, alpha = 0.3, -0.7, 0.05
    z = np.full((H, W), 0.4)
    X, Y = np.meshgrid(np.arange(W), np.arange(H))
    U = np.zeros((H, W, 3))
    U[:, :, 0] = a * X + b * Y
    eta = adapt.indicator(z, z, np.full((H - 1, W - 1, 2), alpha), 1.0, U.ravel())
    expect = np.zeros((H - 1, W - 1, 2))
    s = 0.5 * np.sqrt(alpha)
    expect[0, :, 0] += s * abs(b)          # T0 touches the bottom border (y = 0)
    expect[:, -1, 0] += s * abs(a)         # T0 touches the right border (x = W-1)
    expect[-1, :, 1] += s * abs(b)         # T1 touches the top border (y = H-1)
    expect[:, 0, 1] += s * abs(a)          # T1 touches the left border (x = 0)
    assert np.allclose(eta, expect, atol=1e-14)


def test_jump_term_alpha_interface():
    # Two alpha regions, u1 = x: across the vertical interface the flux jumps by
    # (alpha_R - alpha_L); the interface edges use Lambda_e = max(alpha_L, alpha_R).
    W, H = 6, 5
    z = np.full((H, W), 0.4)
    X, _ = np.meshgrid(np.arange(W), np.arange(H))
    U = np.zeros((H, W, 3))
    U[:, :, 0] = X
    al = np.full((H - 1, W - 1, 2), 0.04)
    al[:, 3:, :] = 0.09
    eta = adapt.indicator(z, z, al, 1.0, U.ravel())
    # interior element T1 of cell column 3 (left edge on the interface x = 3),
    # away from the top/bottom borders
    j = 0.5 * (0.09 - 0.04) / np.sqrt(0.09)
    assert eta[2, 3, 1] == pytest.approx(j, rel=1e-12)
    # T0 of cell column 2 has its right edge on the interface
    assert eta[2, 2, 0] == pytest.approx(j, rel=1e-12)
    # elements away from the interface and the borders have no jump at all
    assert eta[2, 1, 0] == pytest.approx(0.0, abs=1e-14)


def test_update_rule_properties():
    rng = np.random.default_rng(4)
    al = rng.uniform(0.01, 0.2, (5, 6, 2))
    eta = rng.uniform(0.0, 3.0, al.shape)
    kappa, thr, ath = 1.5, 0.2, 0.02
    new, m = adapt.update_alpha(al, eta, kappa, thr, ath)
    assert m == eta.max()
    assert np.all(new <= np.maximum(al, ath)) and np.all(new >= ath)
    keep = eta / m <= thr
    assert keep.any() and np.all(new[keep] == np.maximum(al[keep], ath))
    k = np.unravel_index(np.argmax(eta), eta.shape)
    assert new[k] == pytest.approx(max(al[k] / (1 + kappa * (1 - thr)), ath))


def test_indicator_symmetry_rot180():
    W, H = 10, 8
    p = synth.make_pair("plain64", 12, W=W, H=H, noise=0.02)
    al = synth.random_alpha(W, H, 3)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    U = schwarz.dense_solve(A, F)
    eta = adapt.indicator(p.I0, p.I1, al, 1.0, U)
    Ur = U.reshape(H, W, 3)[::-1, ::-1].copy()
    Ur[:, :, :2] *= -1
    eta_r = adapt.indicator(p.I0[::-1, ::-1].copy(), p.I1[::-1, ::-1].copy(),
                            al[::-1, ::-1, ::-1].copy(), 1.0, Ur.ravel())
    assert np.allclose(eta_r[::-1, ::-1, ::-1], eta, rtol=1e-9, atol=1e-12)


def test_metrics_closed_forms():
    H, W = 4, 5
    ue = np.zeros((2, H, W))
    ue[0] = 1.0
    u = np.zeros((2, H, W))
    u[1] = 1.0
    # (1,0,1) vs (0,1,1): cos = 1/2 -> 60 degrees; endpoint distance sqrt 2
    assert metrics.aae(u, ue) == pytest.approx(60.0)
    assert metrics.ee(u, ue) == pytest.approx(np.sqrt(2.0))
    assert metrics.aae(ue, ue) == pytest.approx(0.0, abs=1e-6)


# ---- closed forms of the element-residual term (Section 2.3, eq. (errind)) ----
# These fix every factor of alpha_K^{-1/2} h_K ||R_K||_{L2(K)}: with a linear
# first frame every element has the same gradient g = (p, q), and with a flow
# field whose gradient vanishes there is no flux jump, so eta_K is the residual
# term alone.  The vertices of the two triangles of cell (x, y) are written out
# here from the mesh definition (T0: (x,y), (x+1,y), (x+1,y+1); T1: (x,y),
# (x+1,y+1), (x,y+1)), and int_K v^2 of a linear v with vertex values v_i is
# |K|/6 (sum v_i^2 + sum_{i<j} v_i v_j).

def _linear_frames(W, H, a, p, q, c):
    X, Y = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    I0 = a + p * X + q * Y
    return I0, I0 + c


def _tri_vertex_values(v):
    """Vertex values [H-1, W-1, 2, 3] of a nodal field v [H, W] on T0 / T1."""
    v00, v10, v11, v01 = v[:-1, :-1], v[:-1, 1:], v[1:, 1:], v[1:, :-1]
    t0 = np.stack([v00, v10, v11], axis=-1)
    t1 = np.stack([v00, v11, v01], axis=-1)
    return np.stack([t0, t1], axis=2)


def test_residual_term_closed_form_shift_no_flow():
    # U = 0: s = 0, f_t = c on every node, int_K f_t^2 = c^2 / 2, so
    # eta_K = sqrt(2) sqrt(p^2 + q^2) (c^2 / 2)^{1/2} / sqrt(alpha_K)
    #       = |c| sqrt(p^2 + q^2) / sqrt(alpha_K).
    W, H = 9, 7
    p, q, c = 0.031, -0.017, 0.2
    I0, I1 = _linear_frames(W, H, 0.4, p, q, c)
    al = synth.random_alpha(W, H, 11)
    eta = adapt.indicator(I0, I1, al, 1.0, np.zeros(3 * W * H))
    expect = abs(c) * np.hypot(p, q) / np.sqrt(al)
    assert np.allclose(eta, expect, rtol=1e-12, atol=0.0)


def test_residual_term_closed_form_constant_flow():
    # U = (u, v, 0) constant: s + f_t = p u + q v + c on every node.
    W, H = 8, 6
    p, q, c, u, v = 0.05, 0.02, -0.03, 0.7, -0.4
    I0, I1 = _linear_frames(W, H, 0.3, p, q, c)
    al = synth.random_alpha(W, H, 12)
    U = np.zeros((H, W, 3))
    U[:, :, 0], U[:, :, 1] = u, v
    eta = adapt.indicator(I0, I1, al, 1.0, U.ravel())
    expect = abs(p * u + q * v + c) * np.hypot(p, q) / np.sqrt(al)
    assert np.allclose(eta, expect, rtol=1e-12, atol=0.0)


def test_residual_term_closed_form_illumination_only():
    # U = (0, 0, mu): s + f_t = c - mu f is linear on K with vertex values
    # c - mu f_i, so ||R_K||^2 = |g|^2 |K|/6 (sum v_i^2 + sum_{i<j} v_i v_j).
    W, H = 8, 7
    p, q, c, mu = 0.04, -0.03, 0.05, 0.3
    I0, I1 = _linear_frames(W, H, 0.6, p, q, c)
    al = synth.random_alpha(W, H, 13)
    U = np.zeros((H, W, 3))
    U[:, :, 2] = mu
    eta = adapt.indicator(I0, I1, al, 1.0, U.ravel())
    vv = _tri_vertex_values(c - mu * I0)                      # [H-1, W-1, 2, 3]
    pair_sum = vv[..., 0] * vv[..., 1] + vv[..., 0] * vv[..., 2] + vv[..., 1] * vv[..., 2]
    int_v2 = 0.5 / 6.0 * (np.sum(vv * vv, axis=-1) + pair_sum)
    expect = np.sqrt(2.0) * np.hypot(p, q) * np.sqrt(int_v2) / np.sqrt(al)
    assert np.allclose(eta, expect, rtol=1e-12, atol=0.0)
