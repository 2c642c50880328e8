"""Bilinear energy (Gram) matrix of a set of snapshots (oracle; test infrastructure only).

Paper: Sec. II-A, the energies <x^(m), x^(n)>_M := x^(m)T M x^(n) are defined
for two different time indices (a bilinear form).  For K snapshots
x^(1..K) the matrix G[m, n] = sum_i M_ii x_i^(m) x_i^(n) collects all of
them.  Computed here entry by entry with exactly rounded sums (math.fsum).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["gram"]


def gram(X, M) -> np.ndarray:
    """X: (K, n) snapshots as rows; M: (n,) diagonal.  Returns K x K FP64."""
    X = np.asarray(X, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    K = X.shape[0]
    G = np.empty((K, K))
    for a in range(K):
        wa = M * X[a]
        for b in range(a, K):
            G[a, b] = G[b, a] = math.fsum(wa * X[b])
    return G
