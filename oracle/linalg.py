"""Normal-equation solve used by every ALS update (test oracle; float64).

Algorithm 1 writes the update as A_new = M Gamma^dagger; the experimental
setup (Section 5) solves it as a symmetric positive definite system.  The
oracle does exactly that: a Cholesky factorisation Gamma = L L^T followed by
two triangular solves per right-hand side row.

Reading where the paper is silent: if the factorisation meets a non-positive
pivot, the oracle retries once with Gamma + delta I, delta = R * 2^-52 *
max(diag Gamma).  The GPU library applies the same rule.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack


def jitter(gamma):
    """The diagonal shift applied after a failed factorisation."""
    r = gamma.shape[0]
    return r * 2.0 ** -52 * float(np.max(np.diag(gamma)))


def cholesky(gamma):
    """Lower Cholesky factor of an SPD matrix, with the single jitter retry.

    Returns (L, status) with status 0 for a clean factorisation and 1 when the
    jittered matrix was used.  Raises numpy.linalg.LinAlgError if both fail.
    """
    try:
        return np.linalg.cholesky(gamma), 0
    except np.linalg.LinAlgError:
        g = gamma + jitter(gamma) * np.eye(gamma.shape[0])
        return np.linalg.cholesky(g), 1


def first_failed_pivot(gamma):
    """0-based index of the first pivot at which the Cholesky factorisation of gamma (no
    shift) meets a non-positive or non-finite value, or -1 if it succeeds.  LAPACK's
    dpotrf reports the order of the first leading minor that is not positive definite;
    the pivot index is that order minus one."""
    g = np.array(gamma, dtype=np.float64, order="F")
    bad = np.argwhere(~np.isfinite(g))
    if bad.size:
        # entry (r, c) of the lower triangle enters pivot max(r, c) (and no earlier one);
        # before it, the leading block decides
        k = int(np.min(np.max(bad, axis=1)))
        p = first_failed_pivot(g[:k, :k]) if k > 0 else -1
        return p if p >= 0 else k
    _, info = lapack.dpotrf(g, lower=1)
    if info < 0:
        raise ValueError(f"dpotrf argument error {info}")
    return int(info) - 1 if info > 0 else -1


def solve_normal(gamma, M):
    """A_new with A_new Gamma = M (rows are independent right-hand sides)."""
    L, status = cholesky(gamma)
    # Gamma A_new^T = M^T  <=>  L (L^T A_new^T) = M^T
    Y = sla.solve_triangular(L, M.T, lower=True)
    Z = sla.solve_triangular(L.T, Y, lower=False)
    return np.ascontiguousarray(Z.T), status
