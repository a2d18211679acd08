"""Host check of the twisted block elimination that the library's factor and
sweep kernels implement (no GPU): for a random SPD block-tridiagonal matrix,
eliminating the lines from both ends towards a middle line k and solving in
that order reproduces a dense solve, for every choice of k."""
import numpy as np
import pytest


def twisted_solve(A, B, r, k):
    nt = len(A)
    S = [None] * nt
    for t in range(k):
        S[t] = A[t] - (B[t] @ np.linalg.solve(S[t - 1], B[t].T) if t > 0 else 0)
    for t in range(nt - 1, k, -1):
        S[t] = A[t] - (B[t + 1].T @ np.linalg.solve(S[t + 1], B[t + 1]) if t < nt - 1 else 0)
    S[k] = (A[k] - (B[k] @ np.linalg.solve(S[k - 1], B[k].T) if k > 0 else 0)
            - (B[k + 1].T @ np.linalg.solve(S[k + 1], B[k + 1]) if k < nt - 1 else 0))
    Si = [np.linalg.inv(s) for s in S]
    w = [None] * nt
    for t in range(k):
        w[t] = Si[t] @ (r[t] - (B[t] @ w[t - 1] if t > 0 else 0))
    for t in range(nt - 1, k, -1):
        w[t] = Si[t] @ (r[t] - (B[t + 1].T @ w[t + 1] if t < nt - 1 else 0))
    x = [None] * nt
    x[k] = Si[k] @ (r[k] - (B[k] @ w[k - 1] if k > 0 else 0) - (B[k + 1].T @ w[k + 1] if k < nt - 1 else 0))
    for t in range(k - 1, -1, -1):
        x[t] = w[t] - Si[t] @ (B[t + 1].T @ x[t + 1])
    for t in range(k + 1, nt):
        x[t] = w[t] - Si[t] @ (B[t] @ x[t - 1])
    return np.concatenate(x)


@pytest.mark.parametrize("nt", [1, 2, 3, 7])
def test_twisted_elimination_equals_dense_solve(nt):
    rng = np.random.default_rng(nt)
    m = 5
    A = [a @ a.T + 3 * m * np.eye(m) for a in (rng.normal(size=(m, m)) for _ in range(nt))]
    B = [None] + [rng.normal(size=(m, m)) for _ in range(1, nt)]      # B[t]: rows of line t, cols of line t-1
    K = np.zeros((nt * m, nt * m))
    for t in range(nt):
        K[t * m:(t + 1) * m, t * m:(t + 1) * m] = A[t]
        if t > 0:
            K[t * m:(t + 1) * m, (t - 1) * m:t * m] = B[t]
            K[(t - 1) * m:t * m, t * m:(t + 1) * m] = B[t].T
    r = rng.normal(size=(nt, m))
    xe = np.linalg.solve(K, r.ravel())
    for k in range(nt):
        assert np.abs(twisted_solve(A, B, r, k) - xe).max() < 1e-12
