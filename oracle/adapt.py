"""Residual error indicator and adaptive alpha (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper, Section 2.3, equation (errind) and the decrease rule that follows it:

    eta_K = Lambda_K^{-1/2} h_K || R_K ||_{L2(K)^2}
            + 1/2 sum_{e in edges(K)} Lambda_e^{-1/2} h_e^{1/2} || [Lambda grad U . n_e]_e ||_{L2(e)^2}

    alpha_K <- max( alpha_K / (1 + kappa max(eta_K / ||eta||_inf - eta, 0)), alpha_th )

Readings (binding for the oracle and the library alike):

* the norms carry the exponent 2 and alpha is the only adapted parameter, so
  the indicator is taken on the two flow components with Lambda = alpha;
* R_K is the strong residual of the Euler-Lagrange system on K.  For P1 fields
  with element-constant alpha, div(alpha grad u) = 0 inside K, so for the flow
  components R_K = F - A_rho U = -(f_x, f_y) (s + f_t) with
  s = f_x u1 + f_y u2 - f m (the "+" printed before A_rho U is read as the
  residual's "-"); its squared L2(K) norm is |grad f|^2 int_K (s + f_t)^2, a
  degree-4 integral evaluated exactly;
* the degree-4 element integral is evaluated with a positive exact rule
  (weighted sum of squares), not by expanding the square;
* h_K is the element diameter (sqrt 2), h_e the edge length;
* [.]_e is (outside - inside) of alpha grad u_c . n_e for c = 1, 2; on the image
  border the outside flux is zero (natural Neumann condition); Lambda_e is the
  larger alpha of the two elements (the element's own on the border); the
  jump is constant along e, so its L2(e) norm is |J_e| h_e^{1/2};
* ||eta||_inf is the maximum over all elements of the frame pair; if it is 0,
  alpha is left unchanged.

The element residual is pinned against the moment-formula expansion and, with
its weights h_K, |grad f| and alpha_K^{-1/2}, against closed forms on linear
frames (constant shift with zero, constant-flow and constant-illumination
fields, where the flux jumps vanish); the jump term against closed forms of
linear flows and alpha interfaces.  The adapted alpha values on textured pairs
have no printed reference ("parity unpinned" beyond those invariants).
"""
from __future__ import annotations

import numpy as np

from . import fem


def element_edges(tri: np.ndarray, xy: np.ndarray):
    """Edges of every element: vertex pairs, lengths, unit normals, neighbours.

    Returns ``ev`` [E, 3, 2] vertex ids (edge k is opposite vertex k),
    ``length`` [E, 3], ``normal`` [E, 3, 2] and ``nbr`` [E, 3] (element across
    the edge, -1 on the image border).  Neighbours are found by matching the
    sorted vertex pairs of all edges.
    """
    E = tri.shape[0]
    ev = np.stack([tri[:, [1, 2]], tri[:, [2, 0]], tri[:, [0, 1]]], axis=1)
    a = np.minimum(ev[..., 0], ev[..., 1]).ravel().astype(np.int64)
    b = np.maximum(ev[..., 0], ev[..., 1]).ravel().astype(np.int64)
    key = a * (int(b.max()) + 1) + b
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nbr = np.full(3 * E, -1, dtype=np.int64)
    same = np.flatnonzero(ks[1:] == ks[:-1])
    i0, i1 = order[same], order[same + 1]
    nbr[i0] = i1 // 3
    nbr[i1] = i0 // 3
    d = xy[ev[..., 1]] - xy[ev[..., 0]]
    length = np.hypot(d[..., 0], d[..., 1])
    normal = np.stack([d[..., 1], -d[..., 0]], axis=-1) / length[..., None]
    return ev, length, normal, nbr.reshape(E, 3)


def _collapsed_gauss(order: int = 3):
    """Positive-weight rule on the reference triangle (barycentric points).

    Gauss-Legendre in (a, b) on [0,1]^2 mapped by (l1, l2) = (a, b (1 - a)), with
    the Jacobian (1 - a) folded into the weights; ``order = 3`` integrates
    polynomials of degree <= 4 exactly.  Weights sum to 1/2 (the reference area).
    """
    xg, wg = np.polynomial.legendre.leggauss(order)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    pts, wts = [], []
    for a, wa in zip(xg, wg):
        for b, wb in zip(xg, wg):
            pts.append((1.0 - a - b * (1.0 - a), a, b * (1.0 - a)))
            wts.append(wa * wb * (1.0 - a))
    return np.array(pts), np.array(wts)


def _residual_integral(ed: dict, Uv: np.ndarray) -> np.ndarray:
    """int_K (s + f_t)^2 per element, s = f_x u1 + f_y u2 - f m.

    The integrand has degree 4; a positive-weight rule exact to that degree
    evaluates it as a weighted sum of squares, so an exactly fitting field
    gives a residual at the rounding level of s + f_t itself (a moment-table
    expansion would cancel large terms and leave sqrt-of-rounding noise).
    """
    pts, wts = _collapsed_gauss(3)
    g, fv, ftv = ed["g"], ed["fv"], ed["ftv"]
    area = ed["area"]
    out = np.zeros(fv.shape[0])
    for lb, w in zip(pts, wts):
        fq = fv @ lb
        ftq = ftv @ lb
        Uq = np.einsum("eic,i->ec", Uv, lb)
        val = g[:, 0] * Uq[:, 0] + g[:, 1] * Uq[:, 1] - fq * Uq[:, 2] + ftq
        out += w * val * val
    return 2.0 * area * out


def element_residual_integral(I0, I1, U) -> np.ndarray:
    """int_K (s + f_t)^2 per element (flattened element order)."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    ed = fem.element_data(I0, I1, W, H)
    Uv = np.asarray(U, dtype=np.float64).reshape(-1, 3)[ed["tri"]]
    return _residual_integral(ed, Uv)


def indicator(I0, I1, alpha, lam, U) -> np.ndarray:
    """eta_K per element, shape [H-1, W-1, 2] like alpha."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    ed = fem.element_data(I0, I1, W, H)
    tri, g = ed["tri"], ed["g"]
    Uv = np.asarray(U, dtype=np.float64).reshape(-1, 3)[tri]     # [E, 3 vertices, 3 fields]
    al = np.asarray(alpha, dtype=np.float64).reshape(-1)
    quad = _residual_integral(ed, Uv)
    diam = np.sqrt(2.0)
    res_norm = np.sqrt(np.sum(g * g, axis=1) * quad)
    eta = diam * res_norm / np.sqrt(al) + jump_terms(ed, Uv, al)
    return eta.reshape(H - 1, W - 1, 2)


def jump_terms(ed: dict, Uv: np.ndarray, al: np.ndarray) -> np.ndarray:
    """The edge part of eta_K: 1/2 sum_e alpha_e^{-1/2} h_e^{1/2} ||J_e||_{L2(e)},
    J_e the jump of alpha grad u_c . n_e, c = 1, 2 (flattened element order)."""
    tri, xy, G = ed["tri"], ed["xy"], ed["G"]
    eta = np.zeros(tri.shape[0])
    # flux jumps of alpha grad u_c, c = 1, 2
    grad_u = np.einsum("eik,eic->eck", G, Uv[:, :, :2])          # [E, 2 fields, 2]
    flux = al[:, None, None] * grad_u
    ev, length, normal, nbr = element_edges(tri, xy)
    for k in range(3):
        nb = nbr[:, k]
        inner = nb >= 0
        out_flux = np.zeros_like(flux)
        out_flux[inner] = flux[nb[inner]]
        jump = np.einsum("eck,ek->ec", out_flux - flux, normal[:, k, :])
        a_e = al.copy()
        a_e[inner] = np.maximum(al[inner], al[nb[inner]])
        eta += 0.5 * length[:, k] * np.linalg.norm(jump, axis=1) / np.sqrt(a_e)
    return eta


def update_alpha(alpha, eta, kappa: float, eta_thr: float, alpha_th: float):
    """Decrease rule of Section 2.3; returns (new alpha, ||eta||_inf)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    m = float(np.max(eta))
    if m == 0.0:
        return alpha.copy(), m
    fac = 1.0 + kappa * np.maximum(eta / m - eta_thr, 0.0)
    return np.maximum(alpha / fac, alpha_th), m
