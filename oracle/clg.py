"""The combined local-global data term K_rho * (.) (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper, Section 1, functionals (BW) and (BW2) and the Euler-Lagrange system
that follows them: the data term of the model is smoothed by a Gaussian K_rho
of deviation rho,

    A_rho = K_rho * (a a^T),   F = -K_rho * (a f_t),   a = (f_x, f_y, -f),

and Section 2.2 asks only for "a finite element approximation" A_{rho,h} of
A_rho.  Reading taken here (binding for the oracle and the library alike):

* K_rho is the Gaussian sampled at the integer pixel offsets |k| <= ceil(3 rho)
  and normalised to sum 1 (the kernel of the presmoothing K_sigma), and the
  convolution runs over whole-pixel shifts s of the data:
  (K_rho * q)(x) = sum_s w_{s_x} w_{s_y} q(x - s);
* the mesh is invariant under pixel shifts, so on element K the shifted data
  a(x - s), f_t(x - s) are the P1 data of the element K - s of the same type,
  taken at the same barycentric coordinates; a shift that leaves the image
  takes the nearest element of that type (clamp to edge, per axis);
* the element integrals stay exact:
  int_K (K_rho * (a a^T)) U . V = sum_s w_s int_K (a^s . U)(a^s . V), and the
  right-hand side likewise.

With rho = 0 this is exactly the assembly of module ``fem``.  A_rho is a
convex combination of the data terms of shifted images (each positive
semi-definite) plus the stiffness, so it stays symmetric and positive
definite whenever the rho = 0 system is.

The error indicator (Section 2.3, equation (errind)) keeps its form with this
data term: on K the flow components of the strong residual are
R_c = -sum_s w_s f^s_c (a^s . U + f_t^s), c = x, y, a degree-4 polynomial
integrated exactly; the flux jumps are those of module ``adapt``.

Pinned by: rho = 0 is the plain assembly; a constant first frame leaves the
matrix unchanged; a linear first frame changes only the (m, m) blocks of
interior elements, by (p^2 + q^2) sum_k w_k k^2 times the mass matrix; the
energy U^T A U - 2 F^T U + c against a brute-force quadrature of the shifted
data; symmetry, positive definiteness and the transpose symmetry.
"""
from __future__ import annotations

import numpy as np

from . import adapt, fem, variants


def shift_elements(W: int, H: int, sx: int, sy: int) -> np.ndarray:
    """Element ids of K - s for every element K (flattened order), the cell
    index clamped to the cell grid per axis, the element type kept."""
    cx, cy = np.meshgrid(np.arange(W - 1), np.arange(H - 1))
    cx = np.clip(cx - sx, 0, W - 2).ravel()
    cy = np.clip(cy - sy, 0, H - 2).ravel()
    cell = cy * (W - 1) + cx
    return np.stack([2 * cell, 2 * cell + 1], axis=1).reshape(-1)


def shifts(rho: float):
    """(s_x, s_y, weight) of the sampled, normalised Gaussian K_rho."""
    w = variants.gaussian_weights(rho)
    R = (len(w) - 1) // 2
    return [(sx, sy, w[sx + R] * w[sy + R]) for sy in range(-R, R + 1) for sx in range(-R, R + 1)]


def _shifted(ed: dict, idx: np.ndarray) -> dict:
    """Element data with f, f_t and grad f taken from the elements idx."""
    out = dict(ed)
    out["fv"] = ed["fv"][idx]
    out["ftv"] = ed["ftv"][idx]
    out["g"] = ed["g"][idx]
    return out


def element_matrices_clg(ed: dict, alpha: np.ndarray, lam: float, rho: float, W: int, H: int):
    """Local 9x9 matrices and 9-vectors: stiffness of ``fem`` plus the data
    term and right-hand side averaged over the shifts of K_rho."""
    E = ed["tri"].shape[0]
    zero = dict(ed, fv=np.zeros_like(ed["fv"]), ftv=np.zeros_like(ed["ftv"]), g=np.zeros_like(ed["g"]))
    Ae, Fe = fem.element_matrices(zero, alpha, lam)            # stiffness only
    no_reg = np.zeros(E)
    for sx, sy, w in shifts(rho):
        As, Fs = fem.element_matrices(_shifted(ed, shift_elements(W, H, sx, sy)), no_reg, 0.0)
        Ae = Ae + w * As
        Fe = Fe + w * Fs
    return Ae, Fe


def assemble_clg(I0, I1, alpha, lam: float, rho: float):
    """Global system A_rho U = F_rho of one frame pair (CSR matrix, vector)."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    ed = fem.element_data(I0, I1, W, H)
    Ae, Fe = element_matrices_clg(ed, alpha, lam, rho, W, H)
    return fem.assemble_elements(ed, Ae, Fe, W, H)


def residual_integral_clg(ed: dict, Uv: np.ndarray, rho: float, W: int, H: int) -> np.ndarray:
    """int_K (R_x^2 + R_y^2) per element, R_c = sum_s w_s f^s_c (a^s . U + f_t^s),
    by the positive degree-4 rule of module ``adapt``."""
    pts, wts = adapt._collapsed_gauss(3)
    E = ed["tri"].shape[0]
    out = np.zeros(E)
    sh = [(_shifted(ed, shift_elements(W, H, sx, sy)), w) for sx, sy, w in shifts(rho)]
    for lb, wq in zip(pts, wts):
        Uq = np.einsum("eic,i->ec", Uv, lb)
        R = np.zeros((E, 2))
        for e, w in sh:
            val = e["g"][:, 0] * Uq[:, 0] + e["g"][:, 1] * Uq[:, 1] - (e["fv"] @ lb) * Uq[:, 2] + e["ftv"] @ lb
            R += w * e["g"] * val[:, None]
        out += wq * np.sum(R * R, axis=1)
    return 2.0 * ed["area"] * out


def indicator_clg(I0, I1, alpha, lam: float, rho: float, U) -> np.ndarray:
    """eta_K with the K_rho data term, shape [H-1, W-1, 2] like alpha."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    ed = fem.element_data(I0, I1, W, H)
    Uv = np.asarray(U, dtype=np.float64).reshape(-1, 3)[ed["tri"]]
    al = np.asarray(alpha, dtype=np.float64).reshape(-1)
    quad = residual_integral_clg(ed, Uv, rho, W, H)
    eta = np.sqrt(2.0) * np.sqrt(quad) / np.sqrt(al) + adapt.jump_terms(ed, Uv, al)
    return eta.reshape(H - 1, W - 1, 2)


def energy_quadrature_clg(I0, I1, alpha, lam: float, rho: float, U, order: int = 4) -> float:
    """sum_s w_s int (a^s . U + f_t^s)^2 + alpha |grad u|^2 + lambda |grad m|^2,
    by a collapsed Gauss rule on every element with the shifted data evaluated
    at each quadrature point from the shifted element's vertex values (no
    moment tables): pins ``assemble_clg`` through
    E(U) = U^T A U - 2 F^T U + sum_s w_s int (f_t^s)^2."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    tri, xy = fem.mesh(W, H)
    G, area = fem.barycentric_gradients(tri, xy)
    f0 = I0.reshape(-1)
    ft = (np.asarray(I1, dtype=np.float64) - I0).reshape(-1)
    Uv = np.asarray(U, dtype=np.float64).reshape(-1, 3)[tri]
    al = np.asarray(alpha, dtype=np.float64).reshape(-1)
    xg, wg = np.polynomial.legendre.leggauss(order)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    total = 0.0
    for sx, sy, w in shifts(rho):
        idx = shift_elements(W, H, sx, sy)
        fs, fts = f0[tri[idx]], ft[tri[idx]]                    # vertex values of the shifted element
        gs = np.einsum("eik,ei->ek", G[idx], fs)
        for a, wa in zip(xg, wg):
            for b, wb in zip(xg, wg):
                lb = np.array([1.0 - a - b * (1.0 - a), a, b * (1.0 - a)])
                Uq = np.einsum("eic,i->ec", Uv, lb)
                r = gs[:, 0] * Uq[:, 0] + gs[:, 1] * Uq[:, 1] - (fs @ lb) * Uq[:, 2] + fts @ lb
                total += w * np.sum(2.0 * area * wa * wb * (1.0 - a) * r * r)
    gU = np.einsum("eik,eic->eck", G, Uv)
    reg = al * (np.sum(gU[:, 0] ** 2, axis=1) + np.sum(gU[:, 1] ** 2, axis=1)) + lam * np.sum(gU[:, 2] ** 2, axis=1)
    return float(total + np.sum(area * reg))


def ft_squared_integral_clg(I0, I1, rho: float) -> float:
    """sum_s w_s int (f_t^s)^2 (the constant term of the energy)."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    tri, _ = fem.mesh(W, H)
    ft = (np.asarray(I1, dtype=np.float64) - I0).reshape(-1)
    M = fem.product_table(2, 0.5)
    total = 0.0
    for sx, sy, w in shifts(rho):
        v = ft[tri[shift_elements(W, H, sx, sy)]]
        total += w * float(np.einsum("ei,ij,ej->", v, M, v))
    return total
