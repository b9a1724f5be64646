"""Tucker decomposition by ALS (HOOI) and by pairwise perturbation (test oracle;
float64, plain numpy).  Modes are 0-based.

Follows the Tucker-ALS procedure (Algorithm 2, Section 2.4) and PP-Tucker-ALS
(Algorithm 4, Section 3.2.2):

* the TTMc Y^(n) = X x_{i != n} A^(i)T keeps mode n in place and replaces every
  other mode i by its rank R_i;
* A^(n) <- the R_n leading left singular vectors of the unfolding Y^(n)_(n),
  computed, as in the paper's implementation, as the eigenvectors of the Gram
  matrix W = Y_(n) Y_(n)^T that belong to its R_n largest eigenvalues;
* the core G = Y^(N) x_N A^(N)T after every sweep and F = G_new - G;
* PP: operators Y_p^(i,n) = X x_{j not in {i,n}} A_p^(j)T and
  Y_p^(n) = X x_{j != n} A_p^(j)T, and the first-order approximation
  Y~^(n) = Y_p^(n) + sum_{i != n} Y_p^(i,n) x_i dA^(i)T.

Readings where the paper is silent:

* Eigenvector order and signs.  Columns are in decreasing eigenvalue order.  A
  new column is oriented so that its inner product with the column it replaces is
  non-negative (the paper relies on its eigensolver keeping signs consistent
  across sweeps; dA = A - A_p needs them consistent).  For the HOSVD start, where
  nothing is replaced, the entry of largest magnitude is made positive (the first
  one on ties).
* HOSVD: the classical one (A^(n) from X_(n) for every n) and the interlaced one
  (Section 2.4: A^(n) from Z^(n)_(n), Z^(n+1) = Z^(n) x_n A^(n)T, Z^(1) = X); the
  paper's error bound for the TTMc assumes the interlaced start.
* Switching (Algorithm 4).  PP is entered after a sweep in which every
  ||dA^(i)||_F < eps ||A^(i)||_F (strict), and PP sweeps run while
  ||F||_F < eps ||X||_F; a build is made only when at least one PP sweep follows
  it, i.e. when both tests pass.  The paper's stopping test ||F|| > Delta ||X||
  is optional here (delta=None runs the full sweep budget).
* "PP-initialisation sweep" is the operator build plus the first PP sweep; the
  sweep budget counts ALS, PP-init and PP-approximated sweeps alike.
* Fit: with orthonormal factors and G the projection of X, ||X - [[G; A]]||^2 =
  ||X||^2 - ||G||^2; the per-sweep fit uses the G the sweep formed (from the
  approximated Y^(N) in PP sweeps).
"""
from __future__ import annotations

import dataclasses
import string

import numpy as np

_LET = string.ascii_lowercase


def ttm(T, A, n):
    """T x_n A^T: mode n of T (size s_n) contracted with A (s_n x R); the result has R
    in position n."""
    N = T.ndim
    xs = _LET[:N]
    out = xs[:n] + "z" + xs[n + 1:]
    return np.einsum(f"{xs},{xs[n]}z->{out}", T, A, optimize=True)


def ttmc(X, A, n):
    """Y^(n) = X x_{i != n} A^(i)T (Section 2.4)."""
    Y = X
    for i in range(X.ndim):
        if i != n:
            Y = ttm(Y, A[i], i)
    return Y


def unfold(T, n):
    """Mode-n unfolding: rows indexed by mode n, the other modes in increasing order
    (C order)."""
    return np.moveaxis(T, n, 0).reshape(T.shape[n], -1)


def leading_eigvecs(Y, n, R, prev=None):
    """The R leading left singular vectors of Y_(n) from the Gram matrix W = Y_(n) Y_(n)^T
    (numpy eigh), decreasing eigenvalues, signs as in the module reading.  Returns
    (A, eigenvalues)."""
    Yn = unfold(Y, n)
    W = Yn @ Yn.T
    lam, V = np.linalg.eigh(W)
    order = np.argsort(lam)[::-1][:R]
    A = np.ascontiguousarray(V[:, order])
    lam = lam[order]
    for k in range(R):
        if prev is not None:
            s = float(A[:, k] @ prev[:, k])
            if s < 0.0:
                A[:, k] = -A[:, k]
        else:
            j = int(np.argmax(np.abs(A[:, k])))
            if A[j, k] < 0.0:
                A[:, k] = -A[:, k]
    return A, lam


def hosvd(X, ranks):
    """Classical HOSVD start (Section 2.4): A^(n) = leading left singular vectors of
    X_(n); the core is X contracted with every A^(n)T."""
    A = [leading_eigvecs(X, n, ranks[n])[0] for n in range(X.ndim)]
    G = X
    for n in range(X.ndim):
        G = ttm(G, A[n], n)
    return A, G


def hosvd_interlaced(X, ranks):
    """Interlaced HOSVD start (Section 2.4): with Z^(1) = X, A^(n) = the leading left
    singular vectors of Z^(n)_(n) and Z^(n+1) = Z^(n) x_n A^(n)T (the truncated
    Sigma V^T of that SVD), so Z^(n) keeps the modes from n on and the ranks of the
    modes before; the core is the last Z.  Signs as in hosvd."""
    A = []
    Z = X
    for n in range(X.ndim):
        a, _ = leading_eigvecs(Z, n, ranks[n])
        A.append(a)
        Z = ttm(Z, a, n)
    return A, Z


@dataclasses.dataclass
class TuckerRecord:
    kind: str                # "als", "pp_init" or "pp_approx"
    fit: float               # 1 - sqrt(max(0, ||X||^2 - ||G||^2)) / ||X||
    core_norm: float         # ||G||_F
    f_norm: float            # ||G_new - G_old||_F
    rel_change: list         # ||dA^(n)||_F / ||A^(n)||_F after the sweep
    rhs: list = None         # the Y^(n) used (kept for tests)


def _finish(kind, X_norm2, A, G_old, Y_last, rel, rhs):
    N = len(A)
    G = ttm(Y_last, A[N - 1], N - 1)
    g2 = float(np.sum(G * G))
    fit = 1.0 - np.sqrt(max(0.0, X_norm2 - g2)) / np.sqrt(X_norm2)
    fn = float(np.linalg.norm(G - G_old)) if G_old is not None else float(np.linalg.norm(G))
    return G, TuckerRecord(kind, float(fit), float(np.sqrt(g2)), fn, rel, rhs)


def tucker_sweep(X, A, G_old, X_norm2=None):
    """One Tucker-ALS sweep (Algorithm 2, loop body): for n = 1..N, Y^(n) from the current
    factors and A^(n) <- its leading left singular vectors; then the core.  A is updated
    in place; returns (G, record, dA) with dA^(n) the change of the sweep."""
    if X_norm2 is None:
        X_norm2 = float(np.sum(X * X))
    N = X.ndim
    rel, rhs, dA = [], [], []
    Y = None
    for n in range(N):
        Y = ttmc(X, A, n)
        new, _ = leading_eigvecs(Y, n, A[n].shape[1], prev=A[n])
        d = new - A[n]
        A[n] = new
        dA.append(d)
        rel.append(float(np.linalg.norm(d) / np.linalg.norm(new)))
        rhs.append(Y)
    G, rec = _finish("als", X_norm2, A, G_old, Y, rel, rhs)
    return G, rec, dA


@dataclasses.dataclass
class PPTuckerState:
    Ap: list                 # factors at the build, A_p^(n)
    dA: list                 # A^(n) - A_p^(n)
    ops: dict                # (i, n) with i < n -> Y_p^(i,n), modes i and n kept in place
    Yp: list                 # Y_p^(n)


def build_operators(X, A):
    """PP-Tucker initialisation (Algorithm 4, operator build): with A_p = A,
    Y_p^(i,n) = X x_{j not in {i,n}} A_p^(j)T (i < n, both modes kept in place) and
    Y_p^(n) = X x_{j != n} A_p^(j)T; dA <- 0."""
    N = X.ndim
    Ap = [a.copy() for a in A]
    ops = {}
    for i in range(N):
        for n in range(i + 1, N):
            Y = X
            for j in range(N):
                if j not in (i, n):
                    Y = ttm(Y, Ap[j], j)
            ops[(i, n)] = Y
    Yp = [ttmc(X, Ap, n) for n in range(N)]
    return PPTuckerState(Ap=Ap, dA=[np.zeros_like(a) for a in A], ops=ops, Yp=Yp)


def pp_rhs(state, n):
    """Y~^(n) = Y_p^(n) + sum_{i != n} Y_p^(i,n) x_i dA^(i)T (Section 3.2.2)."""
    Y = state.Yp[n].copy()
    for i in range(len(state.Ap)):
        if i == n:
            continue
        op = state.ops[(min(i, n), max(i, n))]
        Y = Y + ttm(op, state.dA[i], i)
    return Y


def pp_sweep(state, A, G_old, X_norm2, kind="pp_approx"):
    """One approximated PP-Tucker sweep (Algorithm 4, inner loop body); A and state.dA
    are updated in place.  Returns (G, record)."""
    N = len(A)
    rel, rhs = [], []
    Y = None
    for n in range(N):
        Y = pp_rhs(state, n)
        new, _ = leading_eigvecs(Y, n, A[n].shape[1], prev=A[n])
        A[n] = new
        state.dA[n] = new - state.Ap[n]
        rel.append(float(np.linalg.norm(state.dA[n]) / np.linalg.norm(new)))
        rhs.append(Y)
    return _finish(kind, X_norm2, A, G_old, Y, rel, rhs)


def pp_tucker_als(X, A0, G0, eps, sweeps, replay=None, delta=None):
    """PP-Tucker-ALS control (Algorithm 4) for a budget of ``sweeps`` sweeps, from the
    factors A0 and core G0 (normally the HOSVD).  dA = A initially, so the first sweep
    is a regular one.  ``replay``: a list of sweep kinds to follow instead of deciding.
    ``delta``: optional stopping tolerance ||F|| <= delta ||X||.  Returns (A, G, records)."""
    A = [a.copy() for a in A0]
    G = G0.copy()
    X_norm2 = float(np.sum(X * X))
    X_norm = np.sqrt(X_norm2)
    recs = []
    if replay is not None:
        state = None
        for kind in replay[:sweeps]:
            if kind == "als":
                G, rec, _ = tucker_sweep(X, A, G, X_norm2)
            elif kind == "pp_init":
                state = build_operators(X, A)
                G, rec = pp_sweep(state, A, G, X_norm2, "pp_init")
            elif kind == "pp_approx":
                if state is None:
                    raise ValueError("pp_approx before any operator build")
                G, rec = pp_sweep(state, A, G, X_norm2, "pp_approx")
            else:
                raise ValueError(kind)
            recs.append(rec)
        return A, G, recs

    def stopped():
        return delta is not None and recs and recs[-1].f_norm <= delta * X_norm

    rel = [1.0] * X.ndim          # dA = A initially
    f_norm = float(np.linalg.norm(G))
    while len(recs) < sweeps and not stopped():
        if all(r < eps for r in rel) and f_norm < eps * X_norm:
            state = build_operators(X, A)
            kind = "pp_init"
            while len(recs) < sweeps and f_norm < eps * X_norm and not stopped():
                G, rec = pp_sweep(state, A, G, X_norm2, kind)
                recs.append(rec)
                f_norm = rec.f_norm
                rel = rec.rel_change
                kind = "pp_approx"
            if len(recs) >= sweeps or stopped():
                break
        G, rec, _ = tucker_sweep(X, A, G, X_norm2)
        recs.append(rec)
        rel = rec.rel_change
        f_norm = rec.f_norm
    return A, G, recs


def tucker_als(X, A0, G0, sweeps):
    """Plain Tucker-ALS (Algorithm 2) for a fixed number of sweeps."""
    A = [a.copy() for a in A0]
    G = G0.copy()
    X_norm2 = float(np.sum(X * X))
    recs = []
    for _ in range(sweeps):
        G, rec, _ = tucker_sweep(X, A, G, X_norm2)
        recs.append(rec)
    return A, G, recs


def reconstruct(G, A):
    """[[G; A^(1), .., A^(N)]] = G x_1 A^(1) .. x_N A^(N)."""
    T = G
    for n, a in enumerate(A):
        T = ttm(T, a.T, n)
    return T
