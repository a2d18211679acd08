"""Pins of the oracle's K_rho (combined local-global) data term against what
the paper and the mathematics fix, never against itself: rho = 0 is the
plain assembly, a constant first frame has nothing to smooth, a linear first
frame changes only the illumination blocks by a closed form, the energy
identity against a brute-force quadrature of the shifted data, symmetry,
positive definiteness and the transpose symmetry."""
import numpy as np
import pytest

from oracle import adapt, clg, fem, variants
from paper_1508_02977_amd import synth


def pair(W, H, seed):
    p = synth.make_pair("plain64", seed, W=W, H=H)
    return p.I0, p.I1


def test_rho_zero_is_the_plain_assembly():
    W, H = 13, 11
    I0, I1 = pair(W, H, 3)
    al = synth.random_alpha(W, H, 4)
    A0, F0 = fem.assemble(I0, I1, al, 1.0)
    A, F = clg.assemble_clg(I0, I1, al, 1.0, 0.0)
    assert abs(A - A0).max() <= 1e-15 * abs(A0).max()
    assert np.abs(F - F0).max() <= 1e-15 * np.abs(F0).max()
    U = np.random.default_rng(1).normal(size=3 * W * H)
    e0 = adapt.indicator(I0, I1, al, 1.0, U)
    e = clg.indicator_clg(I0, I1, al, 1.0, 0.0, U)
    assert np.abs(e - e0).max() <= 1e-13 * e0.max()


def test_constant_first_frame_leaves_the_matrix_unchanged():
    # f = const: a = (0, 0, -f) on every element and every shift
    W, H = 12, 9
    I0 = np.full((H, W), 0.7)
    I1 = I0 + 0.05 * np.random.default_rng(2).normal(size=(H, W))
    al = synth.random_alpha(W, H, 5)
    A0, _ = fem.assemble(I0, I1, al, 1.0)
    A, _ = clg.assemble_clg(I0, I1, al, 1.0, 1.3)
    assert abs(A - A0).max() <= 1e-14 * abs(A0).max()


@pytest.mark.parametrize("rho", [0.5, 1.0])
def test_linear_first_frame_closed_form(rho):
    # f = c + p x + q y: grad f = (p, q) everywhere; away from the border the
    # shifted vertex values are f_k - (p s_x + q s_y), so with symmetric weights
    # only int f^2 phi_i phi_j changes, by (p^2 + q^2) sum_k w_k k^2 int phi_i phi_j
    W, H, p, q = 24, 22, 0.03, -0.02
    X, Y = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    I0 = 0.4 + p * X + q * Y
    I1 = I0 + 0.01                                     # constant f_t: the right-hand side is unchanged too
    al = synth.constant_alpha(W, H)
    A0, F0 = fem.assemble(I0, I1, al, 1.0)
    A, F = clg.assemble_clg(I0, I1, al, 1.0, rho)
    w = variants.gaussian_weights(rho)
    R = (len(w) - 1) // 2
    var = float(np.sum(w * np.arange(-R, R + 1) ** 2))
    # mass matrix of the P1 space (the m-field block of a unit data term)
    E = 2 * (W - 1) * (H - 1)
    ed = fem.element_data(np.zeros((H, W)), np.zeros((H, W)), W, H)
    Me = np.zeros((E, 9, 9))
    M = fem.product_table(2, 0.5)
    for i in range(3):
        for j in range(3):
            Me[:, 3 * i + 2, 3 * j + 2] = M[i, j]
    Mg, _ = fem.assemble_elements(ed, Me, np.zeros((E, 9)), W, H)
    # nodes whose six elements are all more than R cells from the border
    x, y = np.meshgrid(np.arange(W), np.arange(H))
    inner = ((x >= R + 2) & (x <= W - R - 3) & (y >= R + 2) & (y <= H - R - 3)).ravel()
    rows = (3 * np.flatnonzero(inner)[:, None] + np.arange(3)).ravel()
    D = (A - A0)[rows].toarray()
    expect = ((p * p + q * q) * var * Mg)[rows].toarray()
    assert np.abs(D - expect).max() <= 1e-12 * np.abs(A0[rows].toarray()).max()
    assert np.abs(expect).max() > 1e-6                  # the change is there
    assert np.abs((F - F0)[rows]).max() <= 1e-14 * np.abs(F0).max()


@pytest.mark.parametrize("rho", [0.6, 1.2])
def test_energy_identity_against_brute_force_quadrature(rho):
    W, H = 10, 8
    I0, I1 = pair(W, H, 6)
    al = synth.random_alpha(W, H, 7)
    A, F = clg.assemble_clg(I0, I1, al, 0.8, rho)
    U = np.random.default_rng(8).normal(size=3 * W * H)
    e = clg.energy_quadrature_clg(I0, I1, al, 0.8, rho, U)
    c = clg.ft_squared_integral_clg(I0, I1, rho)
    assert U @ (A @ U) - 2.0 * F @ U + c == pytest.approx(e, rel=1e-12)


def test_symmetric_positive_definite_and_transpose_symmetry():
    W, H, rho = 9, 7, 1.0
    I0, I1 = pair(W, H, 9)
    al = synth.random_alpha(W, H, 10)
    A, F = clg.assemble_clg(I0, I1, al, 1.0, rho)
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    assert np.linalg.eigvalsh(Ad).min() > 0.0
    # transposing both frames (and swapping T0 <-> T1 of alpha) swaps u1 and u2
    U = np.linalg.solve(Ad, F).reshape(H, W, 3)
    alT = al.transpose(1, 0, 2)[:, :, ::-1].copy()
    At, Ft = clg.assemble_clg(I0.T.copy(), I1.T.copy(), alT, 1.0, rho)
    Ut = np.linalg.solve(At.toarray(), Ft).reshape(W, H, 3)
    assert np.abs(Ut[:, :, 0] - U[:, :, 1].T).max() <= 1e-9 * np.abs(U).max()
    assert np.abs(Ut[:, :, 1] - U[:, :, 0].T).max() <= 1e-9 * np.abs(U).max()
    assert np.abs(Ut[:, :, 2] - U[:, :, 2].T).max() <= 1e-9 * np.abs(U).max()


def test_indicator_residual_term_closed_form_on_a_linear_frame():
    # constant shift I1 = I0 + D of a linear I0 and U = 0: away from the border
    # R_c = sum_s w_s g_c D = g_c D, so the residual term is sqrt(2) |g| |D| sqrt(|K|) / sqrt(alpha)
    W, H, p, q, D, rho = 20, 18, 0.05, 0.02, 0.3, 0.8
    X, Y = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    I0 = 0.2 + p * X + q * Y
    I1 = I0 + D
    al = synth.random_alpha(W, H, 11)
    eta = clg.indicator_clg(I0, I1, al, 1.0, rho, np.zeros(3 * W * H))
    expect = np.sqrt(2.0) * np.hypot(p, q) * D * np.sqrt(0.5) / np.sqrt(al)
    R = (len(variants.gaussian_weights(rho)) - 1) // 2
    inner = (slice(R + 1, H - 1 - R - 1), slice(R + 1, W - 1 - R - 1))
    assert np.abs(eta[inner] - expect[inner]).max() <= 1e-13 * expect.max()
