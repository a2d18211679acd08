"""Flow accuracy measures of Section 4 (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

AAE: mean over nodes of the angle between (u1, u2, 1) and (u1e, u2e, 1), in
degrees.  EE: mean over nodes of the Euclidean endpoint distance.
"""
from __future__ import annotations

import numpy as np


def aae(u: np.ndarray, ue: np.ndarray) -> float:
    u = np.asarray(u, dtype=np.float64)
    ue = np.asarray(ue, dtype=np.float64)
    num = u[0] * ue[0] + u[1] * ue[1] + 1.0
    den = np.sqrt((u[0] ** 2 + u[1] ** 2 + 1.0) * (ue[0] ** 2 + ue[1] ** 2 + 1.0))
    return float(np.degrees(np.mean(np.arccos(np.clip(num / den, -1.0, 1.0)))))


def ee(u: np.ndarray, ue: np.ndarray) -> float:
    u = np.asarray(u, dtype=np.float64)
    ue = np.asarray(ue, dtype=np.float64)
    return float(np.mean(np.hypot(u[0] - ue[0], u[1] - ue[1])))
