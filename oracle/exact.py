"""Exact PPR references, used to pin the oracle (test infrastructure only).

* ``dense_ppr``: the full matrix Pi with rows pi(s, .), from the power-iteration
  fixed point pi_s = alpha e_s + (1 - alpha) pi_s D^-1 A (eqn:powerit), solved
  directly: Pi = alpha (I - (1 - alpha) D^-1 A)^-1 (dense LU, FP64).
* ``power_iteration``: the paper's own ground-truth method (section 8: 100
  iterations of eqn:powerit); L1 error at most (1 - alpha)^iters.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def transition(g) -> sp.csr_matrix:
    """Row-stochastic P = D^-1 A (duplicate edges, if any, add up)."""
    n = g.n
    deg = np.diff(g.rowptr.astype(np.int64)).astype(np.float64)
    data = np.repeat(1.0 / deg, deg.astype(np.int64))
    return sp.csr_matrix((data, g.colidx.astype(np.int64), g.rowptr.astype(np.int64)),
                         shape=(n, n))


def dense_ppr(g, alpha: float) -> np.ndarray:
    n = g.n
    P = transition(g).toarray()
    M = np.eye(n) - (1.0 - alpha) * P
    return alpha * np.linalg.inv(M)


def power_iteration(g, s: int, alpha: float, iters: int = 100) -> np.ndarray:
    P = transition(g)
    PT = P.T.tocsr()
    e = np.zeros(g.n)
    e[s] = 1.0
    pi = e.copy()
    for _ in range(iters):
        pi = alpha * e + (1.0 - alpha) * (PT @ pi)
    return pi
