"""P1 finite-element assembly of the optical-flow system (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Model (paper, Section 1, functional (BW2) with rho = 0, and its Euler-Lagrange
system): minimise over U = (u1, u2, m)

    E(U) = int (f_x u1 + f_y u2 + f_t - m f)^2
               + alpha (|grad u1|^2 + |grad u2|^2) + lambda |grad m|^2

Discretisation (Section 2.2): the pixel grid, each pixel square cut into two
triangles by the diagonal drawn in figure "sch-mesh", continuous P1 elements
for all three unknowns.  Readings taken where the text is silent:

* nodes are pixel centres, node (x, y) has id ``y*W + x``;
* cell (x, y) is split by the diagonal (x,y)-(x+1,y+1) into
  T0 = [(x,y), (x+1,y), (x+1,y+1)] and T1 = [(x,y), (x+1,y+1), (x,y+1)];
  element id ``2*(y*(W-1) + x) + t`` (alpha is stored ``[H-1, W-1, 2]``);
* f = I (no presmoothing), (f_x, f_y) = gradient of the P1 interpolant of the
  first frame (constant per element), f in the third coefficient is the P1
  interpolant of the first frame, f_t = I1 - I0 at the nodes, interpolated P1;
* every integral is computed exactly with the barycentric moment formula
  int_K l0^a l1^b l2^c = 2|K| a! b! c! / (a+b+c+2)!.

Unknown ordering of the global system: ``3*node + c`` with c = 0 (u1),
1 (u2), 2 (m).  The global matrix is returned as scipy CSR.
"""
from __future__ import annotations

import itertools
from math import factorial

import numpy as np
import scipy.sparse as sp


def moment(a: int, b: int, c: int, area: float) -> float:
    """Exact int_K l0^a l1^b l2^c over a triangle of the given area."""
    return 2.0 * area * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)


def product_table(order: int, area: float) -> np.ndarray:
    """Tensor ``P[i1,...,i_order] = int_K prod_k l_{i_k}`` (barycentric l)."""
    P = np.zeros((3,) * order)
    for idx in itertools.product(range(3), repeat=order):
        e = [idx.count(v) for v in range(3)]
        P[idx] = moment(e[0], e[1], e[2], area)
    return P


def mesh(W: int, H: int):
    """Triangles of the pixel mesh.

    Returns ``tri`` [E, 3] node ids and ``xy`` [N, 2] node coordinates
    (x = column, y = row), element order as in the module docstring.
    """
    if W < 2 or H < 2:
        raise ValueError("the mesh needs at least 2x2 nodes")
    xs, ys = np.meshgrid(np.arange(W - 1), np.arange(H - 1))
    xs = xs.ravel()
    ys = ys.ravel()
    n00 = ys * W + xs
    n10 = n00 + 1
    n11 = n00 + W + 1
    n01 = n00 + W
    t0 = np.stack([n00, n10, n11], axis=1)
    t1 = np.stack([n00, n11, n01], axis=1)
    tri = np.stack([t0, t1], axis=1).reshape(-1, 3)
    X, Y = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    return tri, xy


def barycentric_gradients(tri: np.ndarray, xy: np.ndarray):
    """Gradients of the three barycentric functions per element and areas.

    For vertices P0, P1, P2 with Jacobian J = [P1-P0, P2-P0] (columns),
    (l1, l2) = J^{-1} (P - P0), so grad l1, grad l2 are the rows of J^{-1}
    and grad l0 = -grad l1 - grad l2.
    """
    P0 = xy[tri[:, 0]]
    P1 = xy[tri[:, 1]]
    P2 = xy[tri[:, 2]]
    J = np.stack([P1 - P0, P2 - P0], axis=2)          # [E, 2(xy), 2(cols)]
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    Jinv = np.empty_like(J)
    Jinv[:, 0, 0] = J[:, 1, 1] / det
    Jinv[:, 0, 1] = -J[:, 0, 1] / det
    Jinv[:, 1, 0] = -J[:, 1, 0] / det
    Jinv[:, 1, 1] = J[:, 0, 0] / det
    G = np.empty((tri.shape[0], 3, 2))
    G[:, 1, :] = Jinv[:, 0, :]
    G[:, 2, :] = Jinv[:, 1, :]
    G[:, 0, :] = -G[:, 1, :] - G[:, 2, :]
    return G, 0.5 * np.abs(det)


def element_data(I0: np.ndarray, I1: np.ndarray, W: int, H: int):
    """Per-element geometry and image data (flattened frames)."""
    tri, xy = mesh(W, H)
    G, area = barycentric_gradients(tri, xy)
    f0 = np.asarray(I0, dtype=np.float64).reshape(-1)
    ft = (np.asarray(I1, dtype=np.float64) - np.asarray(I0, dtype=np.float64)).reshape(-1)
    fv = f0[tri]                                       # [E, 3] vertex values of f
    ftv = ft[tri]                                      # [E, 3] vertex values of f_t
    g = np.einsum("eik,ei->ek", G, fv)                 # [E, 2] (f_x, f_y) on K
    return dict(tri=tri, xy=xy, G=G, area=area, fv=fv, ftv=ftv, g=g, f0=f0, ft=ft)


def element_matrices(ed: dict, alpha: np.ndarray, lam: float):
    """Local 9x9 matrices and 9-vectors, local index ``3*vertex + field``.

    Stiffness (weak form, first integral): Lambda_c * |K| grad l_i . grad l_j with
    Lambda = (alpha_K, alpha_K, lambda).  Data term: int_K (a.U)(a.V) with
    a = (f_x, f_y, -f), f the P1 interpolant.  Right-hand side: -int_K f_t (a.V)
    with f_t the P1 interpolant (the Euler-Lagrange right-hand side F with
    rho = 0).
    """
    area = ed["area"]
    if not np.allclose(area, area[0]):
        raise ValueError("uniform mesh expected")
    K = area[0]
    M = product_table(2, K)
    T = product_table(3, K)
    Q = product_table(4, K)
    G, g, fv, ftv = ed["G"], ed["g"], ed["fv"], ed["ftv"]
    E = G.shape[0]
    al = np.asarray(alpha, dtype=np.float64).reshape(-1)
    if al.shape[0] != E:
        raise ValueError(f"alpha has {al.shape[0]} entries, mesh has {E} elements")
    stiff = K * np.einsum("eik,ejk->eij", G, G)        # [E, 3, 3]
    Tf = np.einsum("ijk,ek->eij", T, fv)               # int f l_i l_j
    Qff = np.einsum("ijkl,ek,el->eij", Q, fv, fv)      # int f^2 l_i l_j
    Ae = np.zeros((E, 3, 3, 3, 3))                     # [e, i, c, j, d]
    for c in range(2):
        Ae[:, :, c, :, c] += al[:, None, None] * stiff
        for d in range(2):
            Ae[:, :, c, :, d] += (g[:, c] * g[:, d])[:, None, None] * M[None]
        Ae[:, :, c, :, 2] += -g[:, c][:, None, None] * Tf
        Ae[:, :, 2, :, c] += -g[:, c][:, None, None] * Tf
    Ae[:, :, 2, :, 2] += lam * stiff + Qff
    Fe = np.zeros((E, 3, 3))                           # [e, i, c]
    for c in range(2):
        Fe[:, :, c] = -g[:, c][:, None] * np.einsum("ik,ek->ei", M, ftv)
    Fe[:, :, 2] = np.einsum("ikl,ek,el->ei", T, fv, ftv)
    return Ae.reshape(E, 9, 9), Fe.reshape(E, 9)


def assemble(I0: np.ndarray, I1: np.ndarray, alpha: np.ndarray, lam: float):
    """Global system ``A U = F`` of one frame pair.

    ``I0``, ``I1``: [H, W]; ``alpha``: [H-1, W-1, 2].  Returns (A csr [3N, 3N],
    F [3N]).  Symmetric blocks are mirrored so that A equals its transpose
    bit for bit.
    """
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    ed = element_data(I0, I1, W, H)
    Ae, Fe = element_matrices(ed, alpha, lam)
    return assemble_elements(ed, Ae, Fe, W, H)


def assemble_elements(ed: dict, Ae: np.ndarray, Fe: np.ndarray, W: int, H: int):
    """Global CSR matrix and right-hand side from the local 9x9 matrices and
    9-vectors of every element (symmetric blocks mirrored)."""
    Ae = 0.5 * (Ae + Ae.transpose(0, 2, 1))
    gidx = (3 * ed["tri"][:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 9)
    rows = np.repeat(gidx, 9, axis=1).ravel()
    cols = np.tile(gidx, (1, 9)).ravel()
    N3 = 3 * W * H
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(N3, N3)).tocsr()
    A.sum_duplicates()
    A = (0.5 * (A + A.T)).tocsr()
    F = np.zeros(N3)
    np.add.at(F, gidx.ravel(), Fe.ravel())
    return A, F


def energy_quadrature(I0, I1, alpha, lam, U, order: int = 6) -> float:
    """E(U) by brute-force quadrature, independent of the moment tables.

    Collapsed (Duffy) Gauss-Legendre rule on each triangle, exact for the
    degree-4 data term when ``order >= 3``.  Used only to pin ``assemble``:
    E(U) = U^T A U - 2 F^T U + int f_t^2.
    """
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    tri, xy = mesh(W, H)
    G, area = barycentric_gradients(tri, xy)
    f0 = I0.reshape(-1)
    ft = (np.asarray(I1) - I0).reshape(-1)
    U = np.asarray(U, dtype=np.float64).reshape(-1, 3)
    al = np.asarray(alpha).reshape(-1)
    xg, wg = np.polynomial.legendre.leggauss(order)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    # (s, t) in [0,1]^2 -> barycentric (l1, l2) = (s, t (1 - s)), Jacobian (1 - s)
    pts = []
    for a, wa in zip(xg, wg):
        for b, wb in zip(xg, wg):
            l1 = a
            l2 = b * (1.0 - a)
            pts.append((1.0 - l1 - l2, l1, l2, wa * wb * (1.0 - a)))
    gU = np.einsum("eik,eic->eck", G, U[tri])          # [E, 3 fields, 2]
    gf = np.einsum("eik,ei->ek", G, f0[tri])
    total = 0.0
    for l0, l1, l2, wq in pts:
        lam_b = np.array([l0, l1, l2])
        fq = f0[tri] @ lam_b
        ftq = ft[tri] @ lam_b
        Uq = np.einsum("eic,i->ec", U[tri], lam_b)
        res = gf[:, 0] * Uq[:, 0] + gf[:, 1] * Uq[:, 1] + ftq - Uq[:, 2] * fq
        total += np.sum(2.0 * area * wq * res ** 2)
    reg = al * (np.sum(gU[:, 0] ** 2, axis=1) + np.sum(gU[:, 1] ** 2, axis=1)) \
        + lam * np.sum(gU[:, 2] ** 2, axis=1)
    return float(total + np.sum(area * reg))


def ft_squared_integral(I0, I1) -> float:
    """int f_t^2 with f_t the P1 interpolant (constant term of the energy)."""
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    tri, _ = mesh(W, H)
    ft = (np.asarray(I1) - I0).reshape(-1)
    M = product_table(2, 0.5)
    v = ft[tri]
    return float(np.einsum("ei,ij,ej->", v, M, v))
