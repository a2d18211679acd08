"""Gradients of a loss of the solution with respect to the frames and alpha,
by the adjoint method (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The discrete solution U solves A(theta) U = F(theta) (Section 2.2, discrete
form; theta = (I0, I1, alpha) with lambda fixed and no presmoothing).  For a
loss L(U) with G = dL/dU, the adjoint state P solves A^T P = G, and A is
symmetric, so it is the same system with right-hand side G.  Then

    dL/dtheta = -d/dtheta [ P^T (A U - F) ]      at fixed U and P,

and P^T (A U - F) is the functional

    J = sum_K int_K (a.P)(a.U + f_t)
               + alpha_K (grad P1 . grad U1 + grad P2 . grad U2)
               + lambda grad P3 . grad U3,

with a = (f_x, f_y, -f), f the P1 interpolant of the first frame, f_t of
I1 - I0 (Section 1 and 2.2).  Its partial derivatives, with p = a.P and
e = a.U + f_t:

    dJ/dalpha_K = |K| sum_{c=1,2} grad P_c . grad U_c
    dJ/dI1_n    = int p phi_n
    dJ/dI0_n    = int (grad phi_n . (P1, P2) - phi_n P3) e
                      + p (grad phi_n . (U1, U2) - phi_n U3 - phi_n)

(the last integrand has degree 4; it is integrated with the collapsed Gauss
rule that is exact to degree 4).  The finite-difference tests pin all of it.

The loss used by the tests and the autograd wrapper is the mean end-point
error of the flow against a known flow w, EE = mean_n |(u1, u2)_n - w_n|
(Section 4); its gradient is taken as 0 where the error is exactly 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem
from .adapt import _collapsed_gauss


def adjoint_state(A, G: np.ndarray) -> np.ndarray:
    """P with A P = G (A symmetric: the adjoint system is the forward one)."""
    return spla.spsolve(A.tocsc(), G)


def gradients(I0, I1, alpha, lam: float, U: np.ndarray, P: np.ndarray):
    """(dL/dI0 [H, W], dL/dI1 [H, W], dL/dalpha [H-1, W-1, 2]) from U and P.

    ``U`` and ``P`` are node-interleaved [3 W H] vectors (unknown 3 node + c).
    """
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    ed = fem.element_data(I0, I1, W, H)
    tri, G, area = ed["tri"], ed["G"], ed["area"]
    g, fv, ftv = ed["g"], ed["fv"], ed["ftv"]
    Uv = U.reshape(-1, 3)[tri]                     # [E, 3 vertices, 3 fields]
    Pv = P.reshape(-1, 3)[tri]
    # alpha: -|K| sum_c grad P_c . grad U_c
    gU = np.einsum("eik,eic->eck", G, Uv)          # [E, field, 2] gradient of each field
    gP = np.einsum("eik,eic->eck", G, Pv)
    dal = -area * (np.einsum("ek,ek->e", gP[:, 0], gU[:, 0]) + np.einsum("ek,ek->e", gP[:, 1], gU[:, 1]))
    # frames: quadrature of the degree <= 4 integrands
    pts, wts = _collapsed_gauss(3)
    N = W * H
    dI0 = np.zeros(N)
    dI1 = np.zeros(N)
    for lb, w in zip(pts, wts):
        lb = np.asarray(lb)
        fq = fv @ lb
        ftq = ftv @ lb
        Uq = np.einsum("eic,i->ec", Uv, lb)
        Pq = np.einsum("eic,i->ec", Pv, lb)
        p = g[:, 0] * Pq[:, 0] + g[:, 1] * Pq[:, 1] - fq * Pq[:, 2]
        e = g[:, 0] * Uq[:, 0] + g[:, 1] * Uq[:, 1] - fq * Uq[:, 2] + ftq
        wq = 2.0 * area * w
        for i in range(3):
            phi = lb[i]
            gphi = G[:, i, :]                      # [E, 2] gradient of vertex i's basis function
            d1 = p * phi
            d0 = ((gphi[:, 0] * Pq[:, 0] + gphi[:, 1] * Pq[:, 1] - phi * Pq[:, 2]) * e
                  + p * (gphi[:, 0] * Uq[:, 0] + gphi[:, 1] * Uq[:, 1] - phi * Uq[:, 2] - phi))
            np.add.at(dI1, tri[:, i], -wq * d1)
            np.add.at(dI0, tri[:, i], -wq * d0)
    return dI0.reshape(H, W), dI1.reshape(H, W), dal.reshape(H - 1, W - 1, 2)


def epe_loss(U: np.ndarray, w: np.ndarray):
    """Mean end-point error of the flow part of U against w [H, W, 2], and
    its gradient with respect to U (0 where the error vanishes)."""
    Un = U.reshape(-1, 3)
    d = Un[:, :2] - w.reshape(-1, 2)
    r = np.sqrt((d * d).sum(axis=1))
    N = Un.shape[0]
    G = np.zeros_like(Un)
    nz = r > 0
    G[nz, :2] = d[nz] / r[nz, None] / N
    return float(r.mean()), G.reshape(-1)


def solve(I0, I1, alpha, lam: float) -> np.ndarray:
    """U with A U = F by a sparse direct solve (tiny grids)."""
    A, F = fem.assemble(I0, I1, alpha, lam)
    return spla.spsolve(A.tocsc(), F)
