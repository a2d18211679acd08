"""End-to-end oracle of one frame pair (FP64): assemble, factor, solve, adapt.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The adaptive loop of Section 2.3 on the fixed pixel mesh (no remeshing):
solve, compute eta, decrease alpha, reassemble with the new alpha, refactor,
solve again warm-started from the previous iterate; ``passes`` alpha updates
give ``passes + 1`` solves.

Pinned by: no passes = one RAS solve; with kappa = 0 the warm start continues
the same iteration; with exact (1x1 split) solves the final iterate solves the
system reassembled with the twice-updated alpha.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import adapt, fem, schwarz


@dataclasses.dataclass
class PairResult:
    U: np.ndarray            # [3N] node-interleaved
    alpha: np.ndarray        # [H-1, W-1, 2] final alpha
    sweeps: list             # sweeps per solve
    relres: list             # final relres per solve
    eta_max: list            # ||eta||_inf per alpha update


def solve_pair(I0, I1, alpha, lam, parts_x, parts_y, overlap, rtol, max_sweeps,
               passes=0, kappa=1.0, eta_thr=0.1, alpha_th=1e-3, sweeps_per_solve=None,
               U0=None) -> PairResult:
    """Run the oracle pipeline on one pair.

    ``sweeps_per_solve`` (list) forces the sweep count of every solve (parity
    at equal sweep counts); otherwise each solve stops at ``rtol``.
    """
    I0 = np.asarray(I0, dtype=np.float64)
    H, W = I0.shape
    subs = schwarz.decompose(W, H, parts_x, parts_y, overlap)
    alpha = np.array(alpha, dtype=np.float64)
    U = None if U0 is None else np.asarray(U0, dtype=np.float64).reshape(-1)
    sweeps, rels, etas = [], [], []
    for it in range(passes + 1):
        A, F = fem.assemble(I0, I1, alpha, lam)
        facs = schwarz.factor_subdomains(A, subs)
        if sweeps_per_solve is not None:
            res = schwarz.ras_solve(A, F, facs, U, rtol=0.0, max_sweeps=sweeps_per_solve[it])
        else:
            res = schwarz.ras_solve(A, F, facs, U, rtol=rtol, max_sweeps=max_sweeps)
        U = res.U
        sweeps.append(res.sweeps)
        rels.append(res.relres)
        if it < passes:
            eta = adapt.indicator(I0, I1, alpha, lam, U)
            alpha, m = adapt.update_alpha(alpha, eta, kappa, eta_thr, alpha_th)
            etas.append(m)
    return PairResult(U, alpha, sweeps, rels, etas)


def fields(U: np.ndarray, W: int, H: int) -> np.ndarray:
    """Node-interleaved [3N] -> field planes [3, H, W]."""
    return np.asarray(U).reshape(H, W, 3).transpose(2, 0, 1).copy()


def interleave(Uf: np.ndarray) -> np.ndarray:
    """Field planes [3, H, W] -> node-interleaved [3N]."""
    Uf = np.asarray(Uf)
    return Uf.transpose(1, 2, 0).reshape(-1).copy()
