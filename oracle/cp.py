"""CP model, MTTKRP and CP-ALS (test oracle; float64, plain numpy).

Notation follows Section 2 of the paper: X is an order-N tensor of size
s_1 x ... x s_N stored row-major (last mode fastest); A[n] is the factor
matrix A^(n) of size s_n x R; S[n] = A^(n)T A^(n); modes are 0-based here
(paper mode n is index n-1).
"""
from __future__ import annotations

import dataclasses
import itertools
import string

import numpy as np

from . import linalg

_LET = string.ascii_lowercase


# ---------------------------------------------------------------------------
# Definitions (Section 2.1 notation, Section 2.3 MTTKRP, Section 2.5 intermediates)
# ---------------------------------------------------------------------------

def partial_mttkrp(X, A, keep):
    """Partially contracted MTTKRP intermediate M^(keep) (equation defining the
    dimension-tree intermediates, Section 2.5), elementwise:

        M^(i_1..i_m)(x_i1, .., x_im, k) = sum over the other indices of
            X(x_1, .., x_N) * prod_{r not in keep} A^(r)(x_r, k).

    ``keep`` is a collection of 0-based modes; the output has those modes in
    increasing order followed by the rank index k.  With keep = (n,) this is the
    MTTKRP M^(n) = X_(n) P^(n) of Section 2.3.
    """
    N = X.ndim
    keep = sorted(keep)
    xs = _LET[:N]
    ops, subs = [X], [xs]
    for r in range(N):
        if r not in keep:
            ops.append(A[r])
            subs.append(xs[r] + "z")
    out = "".join(xs[r] for r in keep) + "z"
    return np.einsum(",".join(subs) + "->" + out, *ops, optimize="greedy")


def mttkrp(X, A, n):
    """MTTKRP M^(n)(x_n, k) (Section 2.3 and the elementwise form in Section 2.5)."""
    return partial_mttkrp(X, A, (n,))


def mttkrp_loops(X, A, n):
    """Brute-force MTTKRP with explicit Python loops; tiny tensors only."""
    R = A[0].shape[1]
    M = np.zeros((X.shape[n], R))
    for idx in itertools.product(*[range(s) for s in X.shape]):
        v = X[idx]
        for k in range(R):
            p = v
            for r in range(X.ndim):
                if r != n:
                    p *= A[r][idx[r], k]
            M[idx[n], k] += p
    return M


def unfold(X, n):
    """Mode-n matricization X_(n): rows indexed by x_n, columns by the remaining
    modes in increasing order with the first remaining mode slowest (C order).

    The paper's Kronecker ordering is not pinned down (Section 2.1); this
    unfolding is paired with ``khatri_rao`` below, first matrix slowest, so that
    X_(n) P^(n) reproduces the elementwise definition.
    """
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def khatri_rao(mats):
    """Column-wise Kronecker product a_k (x) b_k (x) ..., first matrix slowest."""
    out = mats[0]
    for m in mats[1:]:
        out = (out[:, None, :] * m[None, :, :]).reshape(-1, m.shape[1])
    return out


def mttkrp_explicit(X, A, n):
    """X_(n) (A^(1) (.) .. A^(n-1) (.) A^(n+1) (.) .. A^(N)) (Section 2.3)."""
    others = [A[r] for r in range(X.ndim) if r != n]
    return unfold(X, n) @ khatri_rao(others)


def gram(a):
    """S = A^T A."""
    return a.T @ a


def hadamard_except(S, n):
    """Gamma^(n) = S^(1) * .. * S^(n-1) * S^(n+1) * .. * S^(N) (Section 2.3)."""
    R = S[0].shape[0]
    g = np.ones((R, R))
    for i, s in enumerate(S):
        if i != n:
            g = g * s
    return g


def cp_full(A):
    """[[A^(1), .., A^(N)]] = sum_r a_r^(1) o .. o a_r^(N) (Section 2.3)."""
    N = len(A)
    xs = _LET[:N]
    return np.einsum(",".join(x + "z" for x in xs) + "->" + xs, *A, optimize="greedy")


# ---------------------------------------------------------------------------
# Fit (Section 5: relative residual r and fitness f = 1 - r)
# ---------------------------------------------------------------------------

def fit_direct(X, A):
    """f = 1 - ||X - [[A]]||_F / ||X||_F, by forming [[A]] densely."""
    return 1.0 - np.linalg.norm(X - cp_full(A)) / np.linalg.norm(X)


def fit_identity(normX2, M_last, A_last, Gamma_last, S_last):
    """Same fit from ||X - [[A]]||^2 = ||X||^2 - 2 <X, [[A]]> + ||[[A]]||^2.

    <X, [[A]]> = sum(M^(N) * A^(N)) with M^(N) the right-hand side of the last
    mode, and ||[[A]]||^2 = 1^T (Gamma^(N) * S^(N)) 1.  In a PP sweep M^(N) is the
    approximated right-hand side that was actually used (reading: the paper
    does not say how fitness is tracked per sweep).
    """
    inner = float(np.sum(M_last * A_last))
    nrm2 = float(np.sum(Gamma_last * S_last))
    r2 = max(0.0, normX2 - 2.0 * inner + nrm2)
    return 1.0 - np.sqrt(r2) / np.sqrt(normX2)


# ---------------------------------------------------------------------------
# CP-ALS sweep (Algorithm 1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SweepRecord:
    kind: str                 # "als", "pp_init" or "pp_approx"
    grad_norm: list           # ||G^(n)||_F per mode
    rel_change: list          # ||dA^(n)||_F / ||A^(n)||_F after the sweep
    chol_status: list         # 0 clean, 1 jittered
    fit_est: float            # identity fit with the right-hand side used
    rhs: list = None          # right-hand sides used (kept for tests)


def als_update(A, S, n, M, step=1.0):
    """One mode update of Algorithm 1 given its right-hand side M.

    Gamma <- Hadamard of the other Grams; A_new <- M Gamma^-1;
    G <- (A - A_new) Gamma; A <- A_new; S <- A^T A.

    ``step`` is the update step size lambda of the variant in Section 5.1:
    A_new = (1 - lambda) A + lambda M Gamma^-1 (lambda = 1 is Algorithm 1).  Reading:
    G stays the gradient at the factor before the update, (A - M Gamma^-1) Gamma,
    whatever lambda is.
    Returns (A_new, Gamma, ||G||_F, chol_status); A and S are updated in place.
    """
    gamma = hadamard_except(S, n)
    a_sol, status = linalg.solve_normal(gamma, M)
    G = (A[n] - a_sol) @ gamma
    a_new = a_sol if step == 1.0 else (1.0 - step) * A[n] + step * a_sol
    A[n] = a_new
    S[n] = gram(a_new)
    return a_new, gamma, float(np.linalg.norm(G)), status


def als_sweep(X, A, S, normX2=None, mttkrp_fn=mttkrp, step=1.0):
    """One Gauss-Seidel sweep over n = 1..N (Algorithm 1, loop body).

    A and S are updated in place.  rel_change[n] = ||A_new - A_old||_F /
    ||A_new||_F, the per-sweep change that Algorithm 3 tests after a regular
    ALS sweep.  ``step``: update step size (see als_update).
    """
    N = X.ndim
    if normX2 is None:
        normX2 = float(np.sum(X * X))
    gn, rc, cs, rhs = [], [], [], []
    gamma = M = None
    for n in range(N):
        M = mttkrp_fn(X, A, n)
        old = A[n].copy()
        a_new, gamma, g, st = als_update(A, S, n, M, step)
        gn.append(g)
        cs.append(st)
        rc.append(float(np.linalg.norm(a_new - old) / np.linalg.norm(a_new)))
        rhs.append(M)
    f = fit_identity(normX2, M, A[N - 1], gamma, S[N - 1])
    return SweepRecord("als", gn, rc, cs, f, rhs)


def cp_als(X, A0, sweeps, step=1.0):
    """Plain CP-ALS for a fixed number of sweeps; returns (A, records)."""
    A = [a.copy() for a in A0]
    S = [gram(a) for a in A]
    normX2 = float(np.sum(X * X))
    recs = [als_sweep(X, A, S, normX2, step=step) for _ in range(sweeps)]
    return A, recs


def objective(X, A):
    """f(A) = 1/2 ||X - [[A]]||_F^2 (Section 2.3)."""
    return 0.5 * float(np.sum((X - cp_full(A)) ** 2))
