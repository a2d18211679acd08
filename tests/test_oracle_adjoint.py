"""Pins of the oracle's adjoint gradients: central finite differences of the
loss through a direct solve of the discrete system (no adjoint involved)."""
import numpy as np
import pytest

from oracle import adjoint, fem
from paper_1508_02977_amd import synth


def setup(seed=1, W=11, H=9):
    p = synth.make_pair("plain64", seed, W=W, H=H)
    al = synth.random_alpha(W, H, seed + 3)
    rng = np.random.default_rng(seed)
    w = rng.normal(scale=0.5, size=(H, W, 2))
    return p, al, w


def loss_of(I0, I1, al, w, lam=1.0):
    U = adjoint.solve(I0, I1, al, lam)
    return adjoint.epe_loss(U, w)[0]


@pytest.mark.parametrize("which", ["I0", "I1", "alpha"])
def test_adjoint_gradient_matches_central_differences(which):
    p, al, w = setup()
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    U = adjoint.solve(p.I0, p.I1, al, 1.0)
    L, G = adjoint.epe_loss(U, w)
    P = adjoint.adjoint_state(A, G)
    dI0, dI1, dal = adjoint.gradients(p.I0, p.I1, al, 1.0, U, P)
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(3):
        if which == "I0":
            v = rng.normal(size=p.I0.shape)
            fd = (loss_of(p.I0 + h * v, p.I1, al, w) - loss_of(p.I0 - h * v, p.I1, al, w)) / (2 * h)
            an = float((dI0 * v).sum())
        elif which == "I1":
            v = rng.normal(size=p.I1.shape)
            fd = (loss_of(p.I0, p.I1 + h * v, al, w) - loss_of(p.I0, p.I1 - h * v, al, w)) / (2 * h)
            an = float((dI1 * v).sum())
        else:
            v = rng.normal(size=al.shape) * al          # relative perturbation keeps alpha > 0
            fd = (loss_of(p.I0, p.I1, al + h * v, w) - loss_of(p.I0, p.I1, al - h * v, w)) / (2 * h)
            an = float((dal * v).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (which, fd, an)


@pytest.mark.parametrize("which", ["I0", "I1", "alpha"])
def test_gradient_formula_equals_residual_difference(which):
    # dL/dtheta . v = -P^T dR/dtheta . v with R(U, theta) = A(theta) U - F(theta)
    # at fixed U and P.  R is linear in alpha and I1 and quadratic in I0, so the
    # central difference of the assembled residual is exact for any step: a
    # pin of the closed-form derivatives through the (separately pinned)
    # assembly, free of the conditioning noise of re-solving.
    p, al, w = setup(seed=5, W=10, H=8)
    A, F = fem.assemble(p.I0, p.I1, al, 1.0)
    U = adjoint.solve(p.I0, p.I1, al, 1.0)
    _, G = adjoint.epe_loss(U, w)
    P = adjoint.adjoint_state(A, G)
    dI0, dI1, dal = adjoint.gradients(p.I0, p.I1, al, 1.0, U, P)

    def R(I0, I1, a):
        Ar, Fr = fem.assemble(I0, I1, a, 1.0)
        return Ar @ U - Fr

    rng = np.random.default_rng(11)
    h = 0.5
    if which == "I0":
        v = rng.normal(size=p.I0.shape)
        d = (R(p.I0 + h * v, p.I1, al) - R(p.I0 - h * v, p.I1, al)) / (2 * h)
        an = float((dI0 * v).sum())
    elif which == "I1":
        v = rng.normal(size=p.I1.shape)
        d = (R(p.I0, p.I1 + h * v, al) - R(p.I0, p.I1 - h * v, al)) / (2 * h)
        an = float((dI1 * v).sum())
    else:
        v = rng.normal(size=al.shape) * 0.01
        d = (R(p.I0, p.I1, al + h * v) - R(p.I0, p.I1, al - h * v)) / (2 * h)
        an = float((dal * v).sum())
    ref = -float(P @ d)
    assert abs(an - ref) <= 1e-9 * abs(ref), (which, an, ref)


def test_zero_loss_gradient_gives_zero_gradients():
    p, al, _ = setup(seed=2)
    U = adjoint.solve(p.I0, p.I1, al, 1.0)
    P = np.zeros_like(U)
    for g in adjoint.gradients(p.I0, p.I1, al, 1.0, U, P):
        assert np.abs(g).max() == 0.0
