"""Pins of the oracle's P1 assembly against what the paper and mathematics fix.

Each test would fail for a plausible slip in ``oracle.fem`` (a dropped term, a
wrong sign, a transposed operand or a wrong moment) without restating its
formulas: brute-force quadrature of the functional (BW2), closed-form
solutions, symmetries of the mesh and invariants of the operator.
"""
import itertools

import numpy as np
import pytest

from oracle import fem, schwarz
from paper_1508_02977_amd import synth


def _duffy_rule(order=8):
    xg, wg = np.polynomial.legendre.leggauss(order)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    pts = []
    for a, wa in zip(xg, wg):
        for b, wb in zip(xg, wg):
            pts.append(((1.0 - a - b * (1.0 - a), a, b * (1.0 - a)), wa * wb * (1.0 - a)))
    return pts


@pytest.mark.parametrize("order", [2, 3, 4])
def test_moment_tables_match_quadrature(order):
    # Section 2.2: exact P1 integrals; checked against numerical integration of
    # products of barycentric functions on a triangle of area 1/2.
    P = fem.product_table(order, 0.5)
    rule = _duffy_rule()
    for idx in itertools.product(range(3), repeat=order):
        q = sum(w * np.prod([l[i] for i in idx]) for l, w in rule)   # area-1/2 reference: 2|K| = 1
        assert P[idx] == pytest.approx(q, rel=1e-13, abs=1e-16)


def test_element_stiffness_hand_values():
    # Figure sch-mesh: unit pixel squares cut by the (x,y)-(x+1,y+1) diagonal;
    # the P1 stiffness of those right triangles, worked out by hand.
    tri, xy = fem.mesh(3, 3)
    G, area = fem.barycentric_gradients(tri, xy)
    S = area[:, None, None] * np.einsum("eik,ejk->eij", G, G)
    S_t0 = 0.5 * np.array([[1, -1, 0], [-1, 2, -1], [0, -1, 1]])
    S_t1 = 0.5 * np.array([[1, 0, -1], [0, 1, -1], [-1, -1, 2]])
    assert np.allclose(S[0::2], S_t0, atol=1e-15)
    assert np.allclose(S[1::2], S_t1, atol=1e-15)
    assert np.allclose(area, 0.5)


@pytest.mark.parametrize("lam", [1.0, 0.3])
def test_energy_identity_pins_A_and_F(lam):
    # E(U) of (BW2) by brute-force quadrature equals U^T A U - 2 F^T U + int f_t^2:
    # a quadratic function is fixed by its values, so this pins A and F whole.
    p = synth.make_pair("plain64", 11, W=9, H=7, noise=0.02)
    al = synth.random_alpha(9, 7, 5)
    A, F = fem.assemble(p.I0, p.I1, al, lam)
    c0 = fem.ft_squared_integral(p.I0, p.I1)
    rng = np.random.default_rng(3)
    for _ in range(4):
        U = rng.normal(size=A.shape[0])
        e_quad = fem.energy_quadrature(p.I0, p.I1, al, lam, U)
        e_form = U @ (A @ U) - 2.0 * F @ U + c0
        assert e_form == pytest.approx(e_quad, rel=1e-12)
    assert fem.energy_quadrature(p.I0, p.I1, al, lam, np.zeros(A.shape[0])) == pytest.approx(c0, rel=1e-12)


def test_symmetric_bitwise_and_spd_on_texture():
    # Section 1 theorem (Lax-Milgram): the form is coercive on textured images,
    # so the assembled matrix is symmetric positive definite.
    p = synth.make_pair("plain64", 2, W=14, H=12)
    al = synth.random_alpha(14, 12, 1)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    assert (A != A.T).nnz == 0
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 0.0


def test_stiffness_kernel_constants():
    # No image data: only the regulariser remains; constants are in its kernel
    # (natural Neumann condition, no Dirichlet rows).
    z = np.zeros((6, 8))
    A, F = fem.assemble(z, z, synth.random_alpha(8, 6, 2), 0.8)
    assert np.all(F == 0.0)
    for c in range(3):
        U = np.zeros((48, 3))
        U[:, c] = 1.0
        assert np.abs(A @ U.ravel()).max() < 1e-14
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > -1e-13


def test_stencil_is_seven_point():
    # Stiffness couples axis neighbours only (the hypotenuse coupling of the
    # unit right triangles is zero); the data term adds the diagonal edge.
    W, H = 6, 5
    p = synth.make_pair("plain64", 3, W=W, H=H, noise=0.05)
    A, _ = fem.assemble(p.I0, p.I1, synth.constant_alpha(W, H), 1.0)
    A = A.tocoo()
    ni, nj = A.row // 3, A.col // 3
    dx = nj % W - ni % W
    dy = nj // W - ni // W
    offs = set(zip(dx.tolist(), dy.tolist()))
    assert offs <= {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)}
    assert {(1, 1), (-1, -1)} <= offs


def test_identical_frames_zero_rhs():
    # Identical frames under constant illumination: f_t = 0, so F = 0 exactly
    # and the solution is U = 0.
    p = synth.make_pair("plain64", 4, W=12, H=10)
    A, F = fem.assemble(p.I0, p.I0, synth.constant_alpha(12, 10), 1.0)
    assert np.all(F == 0.0)


@pytest.mark.parametrize("c", [0.05, -0.12])
def test_constant_gain_exact(c):
    # I1 = (1+c) I0: the constraint (OF2) holds with u = 0, m = c, gradients vanish,
    # so E = 0 at U = (0, 0, c): the exact minimiser.
    W, H = 13, 11
    p = synth.gain_pair(W, H, c)
    A, F = fem.assemble(p.I0, p.I1, synth.random_alpha(W, H, 8), 1.0)
    U = np.zeros((H * W, 3))
    U[:, 2] = c
    assert np.linalg.norm(A @ U.ravel() - F) <= 1e-13 * np.linalg.norm(F)
    Ud = schwarz.dense_solve(A, F).reshape(-1, 3)
    assert np.abs(Ud[:, :2]).max() < 1e-12
    assert np.abs(Ud[:, 2] - c).max() < 1e-12


def test_linear_image_translation_exact():
    # Linear intensity under uniform translation: (ofeq) with illumination holds
    # exactly for U = (w, 0), so A U = F to rounding.
    W, H = 11, 9
    p = synth.linear_pair(W, H, 0.03, 0.02, w=(0.4, -0.25))
    A, F = fem.assemble(p.I0, p.I1, synth.constant_alpha(W, H), 1.0)
    U = np.zeros((H * W, 3))
    U[:, 0], U[:, 1] = 0.4, -0.25
    assert np.linalg.norm(A @ U.ravel() - F) <= 1e-13 * np.linalg.norm(F)


def _rot180_alpha(al):
    return al[::-1, ::-1, ::-1].copy()


def _transpose_alpha(al):
    return al.transpose(1, 0, 2)[:, :, ::-1].copy()


def test_transpose_swaps_flow_components():
    W, H = 10, 8
    p = synth.make_pair("plain64", 5, W=W, H=H, noise=0.02)
    al = synth.random_alpha(W, H, 3)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    U = schwarz.dense_solve(A, F).reshape(H, W, 3)
    At, Ft = fem.assemble(p.I0.T.copy(), p.I1.T.copy(), _transpose_alpha(al), 1.0)
    Ut = schwarz.dense_solve(At, Ft).reshape(W, H, 3)
    assert np.allclose(Ut[:, :, 0], U[:, :, 1].T, atol=1e-11)
    assert np.allclose(Ut[:, :, 1], U[:, :, 0].T, atol=1e-11)
    assert np.allclose(Ut[:, :, 2], U[:, :, 2].T, atol=1e-11)


def test_rotation_180_negates_flow():
    W, H = 10, 8
    p = synth.make_pair("plain64", 6, W=W, H=H, noise=0.02)
    al = synth.random_alpha(W, H, 4)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    U = schwarz.dense_solve(A, F).reshape(H, W, 3)
    Ar, Fr = fem.assemble(p.I0[::-1, ::-1].copy(), p.I1[::-1, ::-1].copy(), _rot180_alpha(al), 1.0)
    Ur = schwarz.dense_solve(Ar, Fr).reshape(H, W, 3)[::-1, ::-1]
    assert np.allclose(Ur[:, :, :2], -U[:, :, :2], atol=1e-11)
    assert np.allclose(Ur[:, :, 2], U[:, :, 2], atol=1e-11)


def test_intensity_scaling_invariance():
    # (s I0, s I1, s^2 alpha, s^2 lambda) scales E by s^2: same minimiser.
    W, H = 9, 8
    p = synth.make_pair("plain64", 7, W=W, H=H, noise=0.02)
    al = synth.random_alpha(W, H, 6)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    U = schwarz.dense_solve(A, F)
    s = 3.0
    A2, F2 = fem.assemble(s * p.I0, s * p.I1, s * s * al, s * s)
    U2 = schwarz.dense_solve(A2, F2)
    assert np.allclose(U2, U, atol=1e-10 * np.abs(U).max())
