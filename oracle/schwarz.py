"""Overlapping image decomposition and additive Schwarz (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper, Section 3.1 (one rectangular part of the image per processor, an
overlap between neighbouring parts) and Section 3.2, equation (schwarz): in
sweep k every subdomain solves the full system restricted to its box with the
natural (Neumann) condition on the image border and the Dirichlet condition
U_i^k = U_j^{k-1} on the interface, all subdomains in parallel from the
previous iterate (additive / Jacobi form).

Readings (the paper gives no formula for them):

* tile cuts ``c_k = floor(k W / P)``; tile (p, q) owns nodes
  ``[cx_p, cx_{p+1}) x [cy_q, cy_{q+1})``;
* an overlap of delta nodes is shared by neighbours: each side of a box that is
  interior to the image is pushed out by ``floor(delta/2)`` (left/top) or
  ``ceil(delta/2)`` (right/bottom); image-border sides are not moved;
* the iterate is glued by ownership: a node takes the value computed by the
  subdomain that owns it.  The Dirichlet form of equation (schwarz) glued this
  way is algebraically the restricted additive Schwarz (RAS) update
  ``U[O_i] += (A_i^{-1} r[S_i])[O_i]`` with ``r = F - A U``; both are here
  (``dirichlet_sweep`` and ``ras_sweep``) and the tests check they agree;
* stop test: relative residual ``||F - A U||_2 / ||F||_2 <= rtol`` checked before
  each sweep (the paper monitors the increment |U^k - U^{k+1}|, also returned).

Local ordering of a subdomain (shared with the library's documentation, not
with its code): the box is cut into lines along its shorter side (columns if
``height <= width``, rows otherwise); local unknown ``3*(t*ms + s) + c`` for line
t, position s along the line (ms nodes per line), field c.  With this ordering
the local matrix is banded with half-bandwidth ``kd = 3*ms + 5``.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def cuts(n: int, parts: int) -> list[int]:
    return [(k * n) // parts for k in range(parts + 1)]


@dataclasses.dataclass
class Subdomain:
    px: int
    py: int
    box: tuple          # (x0, x1, y0, y1) half-open, nodes
    own: tuple          # (x0, x1, y0, y1) half-open, nodes
    cols: bool          # lines are columns (True) or rows (False)
    nodes: np.ndarray   # global node ids in local order
    idx: np.ndarray     # global unknown ids in local order (3 per node)
    own_mask: np.ndarray  # bool per local unknown: owned by this subdomain
    ms: int             # nodes per line
    nt: int             # number of lines

    @property
    def n(self) -> int:
        return self.idx.shape[0]

    @property
    def kd(self) -> int:
        return 3 * self.ms + 5


def decompose(W: int, H: int, parts_x: int, parts_y: int, overlap: int) -> list[Subdomain]:
    """Subdomains in row-major tile order (tile (p, q) -> index q*parts_x + p)."""
    if not (1 <= parts_x <= W and 1 <= parts_y <= H):
        raise ValueError("bad split")
    cx = cuts(W, parts_x)
    cy = cuts(H, parts_y)
    lo = overlap // 2
    hi = overlap - lo
    subs = []
    for q in range(parts_y):
        for p in range(parts_x):
            ox0, ox1, oy0, oy1 = cx[p], cx[p + 1], cy[q], cy[q + 1]
            bx0 = ox0 - lo if p > 0 else 0
            bx1 = ox1 + hi if p < parts_x - 1 else W
            by0 = oy0 - lo if q > 0 else 0
            by1 = oy1 + hi if q < parts_y - 1 else H
            bx0, by0 = max(bx0, 0), max(by0, 0)
            bx1, by1 = min(bx1, W), min(by1, H)
            bw, bh = bx1 - bx0, by1 - by0
            cols = bh <= bw
            if cols:
                t_ax = np.arange(bx0, bx1)
                s_ax = np.arange(by0, by1)
                T, S = np.meshgrid(t_ax, s_ax, indexing="ij")
                nodes = (S * W + T).ravel()
                ms, nt = bh, bw
            else:
                t_ax = np.arange(by0, by1)
                s_ax = np.arange(bx0, bx1)
                T, S = np.meshgrid(t_ax, s_ax, indexing="ij")
                nodes = (T * W + S).ravel()
                ms, nt = bw, bh
            nx = nodes % W
            ny = nodes // W
            own_node = (nx >= ox0) & (nx < ox1) & (ny >= oy0) & (ny < oy1)
            idx = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
            own_mask = np.repeat(own_node, 3)
            subs.append(Subdomain(p, q, (bx0, bx1, by0, by1), (ox0, ox1, oy0, oy1),
                                  cols, nodes, idx, own_mask, ms, nt))
    return subs


def local_matrix(A: sp.csr_matrix, sub: Subdomain) -> sp.csr_matrix:
    """Principal submatrix A[S_i, S_i] in the local ordering."""
    return A[sub.idx][:, sub.idx].tocsr()


def to_lower_band(As: sp.spmatrix, kd: int) -> np.ndarray:
    """LAPACK lower band storage ``ab[i - j, j] = A[i, j]`` for ``j <= i <= j + kd``."""
    As = sp.tril(As).tocoo()
    d = As.row - As.col
    if d.size and d.max() > kd:
        raise ValueError(f"matrix bandwidth {d.max()} exceeds kd={kd}")
    ab = np.zeros((kd + 1, As.shape[0]))
    ab[d, As.col] = As.data
    return ab


@dataclasses.dataclass
class Factored:
    sub: Subdomain
    cb: np.ndarray      # lower band Cholesky factor (LAPACK pbtrf layout)


def factor_subdomains(A: sp.csr_matrix, subs: list[Subdomain]) -> list[Factored]:
    """Banded Cholesky A_i = L_i L_i^T of every subdomain matrix (LAPACK pbtrf).

    Raises ``numpy.linalg.LinAlgError`` if a subdomain matrix is not SPD.
    """
    out = []
    for s in subs:
        ab = to_lower_band(local_matrix(A, s), s.kd)
        cb = sla.cholesky_banded(ab, lower=True, check_finite=True)
        out.append(Factored(s, cb))
    return out


def local_solve(fac: Factored, rhs: np.ndarray) -> np.ndarray:
    return sla.cho_solve_banded((fac.cb, True), rhs, check_finite=False)


def ras_sweep(A, F, facs: list[Factored], U: np.ndarray) -> np.ndarray:
    """One restricted additive Schwarz sweep from iterate U (returns U^{k+1})."""
    r = F - A @ U
    Un = U.copy()
    for fac in facs:
        e = local_solve(fac, r[fac.sub.idx])
        m = fac.sub.own_mask
        Un[fac.sub.idx[m]] = U[fac.sub.idx[m]] + e[m]
    return Un


def dirichlet_sweep(A, F, subs: list[Subdomain], U: np.ndarray) -> np.ndarray:
    """Equation (schwarz) as written: every subdomain solves its local problem
    with Dirichlet data from the previous iterate on the nodes outside its box
    that it couples to, Neumann on the image border (natural condition of the
    global assembly); the new iterate takes each node from its owner.
    Dense local solves (tiny grids only)."""
    Un = U.copy()
    N3 = A.shape[0]
    for s in subs:
        inside = np.zeros(N3, dtype=bool)
        inside[s.idx] = True
        A_row = A[s.idx]
        A_ii = A_row[:, s.idx].toarray()
        A_ie = A_row[:, np.flatnonzero(~inside)]
        rhs = F[s.idx] - A_ie @ U[~inside]
        V = np.linalg.solve(A_ii, rhs)
        Un[s.idx[s.own_mask]] = V[s.own_mask]
    return Un


@dataclasses.dataclass
class SolveResult:
    U: np.ndarray
    sweeps: int
    relres: float
    history: list          # relres before each sweep (and the final one)
    increments: list       # ||U^{k+1} - U^k||_2 per sweep


def ras_solve(A, F, facs, U0=None, rtol: float = 0.0, max_sweeps: int = 1000) -> SolveResult:
    """Sweep until ``relres <= rtol`` or ``max_sweeps`` sweeps were done.

    ``relres_k = ||F - A U^k|| / ||F||`` is checked before sweep k; F = 0 gives
    U = 0 after 0 sweeps.  With ``rtol = 0`` exactly ``max_sweeps`` sweeps run.
    """
    N3 = A.shape[0]
    U = np.zeros(N3) if U0 is None else np.array(U0, dtype=np.float64).reshape(-1)
    Fn = np.linalg.norm(F)
    if Fn == 0.0:
        return SolveResult(np.zeros(N3), 0, 0.0, [0.0], [])
    hist, incs = [], []
    k = 0
    while True:
        rel = np.linalg.norm(F - A @ U) / Fn
        hist.append(rel)
        if rel <= rtol or k >= max_sweeps:
            return SolveResult(U, k, rel, hist, incs)
        Un = ras_sweep(A, F, facs, U)
        incs.append(float(np.linalg.norm(Un - U)))
        U = Un
        k += 1


def dense_solve(A, F) -> np.ndarray:
    """Global direct solve (tiny grids): the limit of the Schwarz iteration."""
    return np.linalg.solve(A.toarray(), F)
