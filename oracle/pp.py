"""Pairwise perturbation for CP-ALS (test oracle; float64, plain numpy).

Follows Section 3 of the paper: the pairwise perturbation operators
M_p^(i,n), the approximated right-hand side of the general PP update equation
(Section 3.2.1) and the PP-CP-ALS control flow (Algorithm 3).  Modes are
0-based here.

Readings where the paper is ambiguous:

* The second-order sum in the general PP update runs over unordered pairs
  {i, j} of modes other than n.  The order-3 derivation (Section 3.1) has one
  term X_(1)(dA^(2) (.) dA^(3)); ordered pairs would count it twice.
* V^(n,i,j) uses the current factors A^(i), A^(j), A^(k) and the current
  A^(n) (before its update in this sweep): the term approximates X by the
  current CP model [[A]] (Section 3.1).
* The switching test is strict: ||dA^(i)||_F < eps ||A^(i)||_F with the
  current A^(i), evaluated after complete sweeps.
* The sweep budget counts ALS, PP-initialisation and PP-approximated sweeps
  alike; a "PP-initialisation sweep" is the operator build plus the first
  PP sweep that follows it (Section 5.1).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import cp, linalg


@dataclasses.dataclass
class PPState:
    Ap: list        # factors at operator build time, A_p^(n)
    dA: list        # A^(n) - A_p^(n)
    ops: dict       # (i, j) with i < j  ->  M_p^(i,j), shape s_i x s_j x R
    Mp: list        # M_p^(n), shape s_n x R


def build_operators(X, A):
    """PP initialisation (Algorithm 3, operator build): with A_p = A,
    M_p^(i,j) = X contracted with A_p^(r) over every mode r not in {i, j}
    (the definition accompanying the general PP update), and
    M_p^(n) = MTTKRP of X with A_p (dA <- 0)."""
    N = X.ndim
    Ap = [a.copy() for a in A]
    ops = {}
    for i in range(N):
        for j in range(i + 1, N):
            ops[(i, j)] = cp.partial_mttkrp(X, Ap, (i, j))
    Mp = [cp.mttkrp(X, Ap, n) for n in range(N)]
    dA = [np.zeros_like(a) for a in A]
    return PPState(Ap=Ap, dA=dA, ops=ops, Mp=Mp)


def first_order_term(state, i, n):
    """sum_x M_p^(i,n)(x, y, k) dA^(i)(x, k), with the operator stored once per
    unordered pair (smaller mode index first)."""
    if i < n:
        return np.einsum("xyk,xk->yk", state.ops[(i, n)], state.dA[i])
    return np.einsum("yxk,xk->yk", state.ops[(n, i)], state.dA[i])


def second_order_matrix(A, S, dA, n):
    """W^(n) = sum over unordered pairs {i, j} of modes other than n of
    (A^(i)T dA^(i)) * (A^(j)T dA^(j)) * Hadamard_{k not in {i,j,n}} (A^(k)T A^(k)),
    so that sum_{i<j} V^(n,i,j) = A^(n) W^(n)."""
    N = len(A)
    R = A[0].shape[1]
    W = np.zeros((R, R))
    U = [A[i].T @ dA[i] for i in range(N)]
    for i in range(N):
        for j in range(i + 1, N):
            if n in (i, j):
                continue
            w = U[i] * U[j]
            for k in range(N):
                if k not in (i, j, n):
                    w = w * S[k]
            W += w
    return W


def pp_rhs(state, A, S, n, second_order=True):
    """Approximated MTTKRP, general PP update equation (Section 3.2.1):

        M~^(n) = M_p^(n) + sum_{i != n} M_p^(i,n) x_i dA^(i)
                 + sum_{unordered {i,j} not containing n} V^(n,i,j).
    """
    M = state.Mp[n].copy()
    for i in range(len(A)):
        if i != n:
            M += first_order_term(state, i, n)
    if second_order:
        M += A[n] @ second_order_matrix(A, S, state.dA, n)
    return M


def pp_sweep(state, A, S, normX2, second_order=True, kind="pp_approx", step=1.0):
    """One approximated sweep (Algorithm 3, inner loop body).  A, S and
    state.dA are updated in place; rel_change[n] = ||A^(n) - A_p^(n)||_F /
    ||A^(n)||_F.  ``step``: the update step size of Section 5.1 (cp.als_update)."""
    N = len(A)
    gn, rc, cs, rhs = [], [], [], []
    gamma = M = None
    for n in range(N):
        M = pp_rhs(state, A, S, n, second_order)
        a_new, gamma, g, st = cp.als_update(A, S, n, M, step)
        state.dA[n] = a_new - state.Ap[n]
        gn.append(g)
        cs.append(st)
        rc.append(float(np.linalg.norm(state.dA[n]) / np.linalg.norm(a_new)))
        rhs.append(M)
    f = cp.fit_identity(normX2, M, A[N - 1], gamma, S[N - 1])
    return cp.SweepRecord(kind, gn, rc, cs, f, rhs)


def pp_als(X, A0, eps, sweeps, second_order=True, replay=None, delta=None, step=1.0):
    """PP-CP-ALS control (Algorithm 3) for a budget of ``sweeps`` sweeps.

    Initially dA = A, so the first sweep is a regular ALS sweep.  Whenever every
    ||dA^(i)|| < eps ||A^(i)||, the operators are rebuilt and PP sweeps run
    while the same test holds (dA measured from the build point); a regular
    ALS sweep follows, with dA^(n) taken as its per-sweep change.

    ``replay``: a list of sweep kinds ("als", "pp_init", "pp_approx") to follow
    instead of deciding (used to compare trajectories without threshold
    ties).  ``delta``: optional gradient stopping tolerance
    (sum_i ||G^(i)||_F <= delta ||X||_F stops the run).  ``step``: the update
    step size lambda of Section 5.1, used by ALS and PP sweeps alike.

    Returns (A, records).
    """
    A = [a.copy() for a in A0]
    S = [cp.gram(a) for a in A]
    normX2 = float(np.sum(X * X))
    normX = np.sqrt(normX2)
    recs = []

    if replay is not None:
        state = None
        for kind in replay[:sweeps]:
            if kind == "als":
                recs.append(cp.als_sweep(X, A, S, normX2, step=step))
            elif kind == "pp_init":
                state = build_operators(X, A)
                recs.append(pp_sweep(state, A, S, normX2, second_order, "pp_init", step))
            elif kind == "pp_approx":
                if state is None:
                    raise ValueError("pp_approx before any operator build")
                recs.append(pp_sweep(state, A, S, normX2, second_order, "pp_approx", step))
            else:
                raise ValueError(kind)
        return A, recs

    def small(rc):
        return all(r < eps for r in rc)

    def converged():
        return delta is not None and recs and sum(recs[-1].grad_norm) <= delta * normX

    rel = [1.0] * X.ndim          # dA = A initially: ||dA|| / ||A|| = 1
    while len(recs) < sweeps and not converged():
        if small(rel):
            state = build_operators(X, A)
            kind = "pp_init"
            while len(recs) < sweeps and small(rel) and not converged():
                rec = pp_sweep(state, A, S, normX2, second_order, kind, step)
                recs.append(rec)
                rel = rec.rel_change
                kind = "pp_approx"
            if len(recs) >= sweeps or converged():
                break
        rec = cp.als_sweep(X, A, S, normX2, step=step)
        recs.append(rec)
        rel = rec.rel_change
    return A, recs


def reinterpreted_als(X, A0, sweeps):
    """Pairwise-update form of ALS (Algorithm 5).  Right-hand sides M^(m) are
    kept and, after each mode update delta A^(n), pushed forward with
    M^(m) += M^(m,n) x_n delta A^(n) using intermediates recomputed at the
    current factors (the oracle-like use described in Section 4.1).
    Algebraically identical to Algorithm 1."""
    N = X.ndim
    A = [a.copy() for a in A0]
    S = [cp.gram(a) for a in A]
    M = [cp.mttkrp(X, A, n) for n in range(N)]
    for _ in range(sweeps):
        for n in range(N):
            gamma = cp.hadamard_except(S, n)
            a_new, _ = linalg.solve_normal(gamma, M[n])
            delta = a_new - A[n]
            A[n] = a_new
            S[n] = cp.gram(a_new)
            for m in range(N):
                if m == n:
                    continue
                Mmn = cp.partial_mttkrp(X, A, (m, n))
                if m < n:
                    M[m] += np.einsum("xyk,yk->xk", Mmn, delta)
                else:
                    M[m] += np.einsum("yxk,yk->xk", Mmn, delta)
    return A
