"""Pins for the Tucker part of the oracle: TTMc (Section 2.4), the factor update through
the Gram matrix, HOOI (Algorithm 2) and PP-Tucker-ALS (Algorithm 4, Section 3.2.2)."""
import itertools

import numpy as np
import pytest

import tensorgen
from oracle import tucker as ot


def _ttmc_loops(X, A, n):
    """X x_{i != n} A^(i)T with explicit loops over every index (tiny tensors)."""
    N = X.ndim
    shape = tuple(X.shape[i] if i == n else A[i].shape[1] for i in range(N))
    Y = np.zeros(shape)
    for out in itertools.product(*[range(s) for s in shape]):
        acc = 0.0
        for x in itertools.product(*[range(s) for s in X.shape]):
            if x[n] != out[n]:
                continue
            v = X[x]
            for i in range(N):
                if i != n:
                    v *= A[i][x[i], out[i]]
            acc += v
        Y[out] = acc
    return Y


def test_ttmc_matches_brute_force():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, 4, 2))
    A = [rng.standard_normal((3, 2)), rng.standard_normal((4, 3)), rng.standard_normal((2, 2))]
    for n in range(3):
        np.testing.assert_allclose(ot.ttmc(X, A, n), _ttmc_loops(X, A, n), rtol=1e-13, atol=1e-13)


def test_unfolding_gram_eigenvectors_span_the_leading_singular_subspace():
    """The Gram-matrix route (paper's implementation) gives the same subspace as an SVD of
    the unfolding, with orthonormal columns in decreasing singular-value order."""
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((9, 4, 5))
    for n in range(3):
        A, lam = ot.leading_eigvecs(Y, n, 3)
        U, s, _ = np.linalg.svd(ot.unfold(Y, n), full_matrices=False)
        np.testing.assert_allclose(A @ A.T, U[:, :3] @ U[:, :3].T, atol=1e-12)
        np.testing.assert_allclose(lam, s[:3] ** 2, rtol=1e-12)
        np.testing.assert_allclose(A.T @ A, np.eye(3), atol=1e-13)
        assert all(lam[k] >= lam[k + 1] for k in range(2))


def test_sign_convention():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((8, 3, 3))
    A, _ = ot.leading_eigvecs(Y, 0, 3)
    for k in range(3):
        j = np.argmax(np.abs(A[:, k]))
        assert A[j, k] > 0
    flipped = A * np.array([-1.0, 1.0, -1.0])
    B, _ = ot.leading_eigvecs(Y, 0, 3, prev=flipped)
    for k in range(3):
        assert B[:, k] @ flipped[:, k] >= 0
    np.testing.assert_allclose(np.abs(B), np.abs(A), atol=1e-13)


def test_hosvd_recovers_an_exact_tucker_tensor():
    p = tensorgen.make_tucker_problem((9, 10, 8), (3, 4, 2), seed=3, eta=0.0)
    A, G = ot.hosvd(p.X, p.ranks)
    np.testing.assert_allclose(ot.reconstruct(G, A), p.X, atol=1e-11 * np.abs(p.X).max())
    for a, q in zip(A, p.planted):
        np.testing.assert_allclose(a @ a.T, q @ q.T, atol=1e-12)


def test_interlaced_hosvd_recovers_an_exact_tucker_tensor():
    p = tensorgen.make_tucker_problem((9, 10, 8, 7), (3, 4, 2, 3), seed=5, eta=0.0)
    A, G = ot.hosvd_interlaced(p.X, p.ranks)
    assert G.shape == p.ranks
    np.testing.assert_allclose(ot.reconstruct(G, A), p.X, atol=1e-11 * np.abs(p.X).max())
    for a, q in zip(A, p.planted):
        np.testing.assert_allclose(a @ a.T, q @ q.T, atol=1e-12)


def test_interlaced_hosvd_steps_are_truncated_svds():
    """Each step keeps the leading singular subspace of the current Z's unfolding: the
    kept energy is the sum of the R_n largest squared singular values (numpy's SVD of
    the unfolding, independent of the Gram route), the next Z's mode-n unfolding has
    orthogonal rows of those norms (Sigma V^T), it has the modes from n + 1 on and the
    ranks before (sizes s^(N-n) R^n), and the first factor is the classical one."""
    X = tensorgen.make_tucker_problem((8, 7, 9, 6), (3, 2, 4, 3), seed=6, eta=0.4).X
    ranks = (3, 2, 4, 3)
    A, G = ot.hosvd_interlaced(X, ranks)
    A_cl, _ = ot.hosvd(X, ranks)
    np.testing.assert_allclose(A[0], A_cl[0], atol=1e-12)
    Z = X
    for n in range(X.ndim):
        sv = np.linalg.svd(ot.unfold(Z, n), compute_uv=False)
        Zn = ot.ttm(Z, A[n], n)
        assert Zn.shape == tuple(ranks[:n + 1]) + X.shape[n + 1:]
        gram = ot.unfold(Zn, n) @ ot.unfold(Zn, n).T
        np.testing.assert_allclose(np.diag(gram), sv[:ranks[n]] ** 2, rtol=1e-10)
        off = gram - np.diag(np.diag(gram))
        assert np.abs(off).max() <= 1e-10 * sv[0] ** 2
        Z = Zn
    np.testing.assert_allclose(G, Z, rtol=0, atol=1e-12 * np.abs(Z).max())
    # the residual is the energy dropped at each step
    dropped = 0.0
    Z = X
    for n in range(X.ndim):
        sv = np.linalg.svd(ot.unfold(Z, n), compute_uv=False)
        dropped += float(np.sum(sv[ranks[n]:] ** 2))
        Z = ot.ttm(Z, A[n], n)
    res = float(np.linalg.norm(X - ot.reconstruct(G, A)) ** 2)
    assert abs(res - dropped) <= 1e-10 * float(np.sum(X * X))


def test_hooi_core_norm_never_decreases_and_fit_identity_holds():
    """Each Tucker-ALS factor update maximises ||Y^(n) x_n A^T|| over orthonormal A, so
    ||G|| cannot decrease (the paper states it strictly increases); the fit from ||G||
    equals the fit of the reconstructed model."""
    p = tensorgen.make_tucker_problem((12, 11, 10), (3, 3, 4), seed=4, eta=0.3)
    A0, G0 = ot.hosvd(p.X, (3, 3, 4))
    A, G, recs = ot.tucker_als(p.X, A0, G0, 8)
    norms = [float(np.linalg.norm(G0))] + [r.core_norm for r in recs]
    assert all(b >= a - 1e-12 * a for a, b in zip(norms, norms[1:]))
    fit_direct = 1.0 - np.linalg.norm(p.X - ot.reconstruct(G, A)) / np.linalg.norm(p.X)
    assert abs(recs[-1].fit - fit_direct) < 1e-12


def test_zero_perturbation_gives_the_exact_ttmc():
    p = tensorgen.make_tucker_problem((8, 9, 7, 6), (3, 2, 3, 2), seed=5, eta=0.1)
    A, _ = ot.hosvd(p.X, p.ranks)
    st = ot.build_operators(p.X, A)
    for n in range(4):
        np.testing.assert_allclose(ot.pp_rhs(st, n), ot.ttmc(p.X, A, n), rtol=1e-12, atol=1e-12)


def test_pp_error_is_second_order():
    """Y~^(n) - Y^(n) is the sum of the terms with two or more dA (Section 3.2.2): its
    norm scales as t^2 for dA = t D."""
    p = tensorgen.make_tucker_problem((9, 8, 10), (3, 3, 3), seed=6, eta=0.1)
    A, _ = ot.hosvd(p.X, p.ranks)
    rng = np.random.default_rng(7)
    D = [rng.standard_normal(a.shape) for a in A]
    errs = []
    ts = [1e-2, 1e-3]
    for t in ts:
        st = ot.build_operators(p.X, A)
        At = [a + t * d for a, d in zip(A, D)]
        st.dA = [t * d for d in D]
        errs.append(np.linalg.norm(ot.pp_rhs(st, 0) - ot.ttmc(p.X, At, 0)))
    slope = np.log(errs[0] / errs[1]) / np.log(ts[0] / ts[1])
    assert abs(slope - 2.0) < 0.05, slope
    # and the omitted term is exactly the order-3 second-order term for N = 3
    st = ot.build_operators(p.X, A)
    At = [a + 1e-2 * d for a, d in zip(A, D)]
    st.dA = [1e-2 * d for d in D]
    second = ot.ttm(ot.ttm(p.X, st.dA[1], 1), st.dA[2], 2)
    np.testing.assert_allclose(ot.ttmc(p.X, At, 0) - ot.pp_rhs(st, 0), second, atol=1e-12)


def test_first_pp_sweep_mode_1_is_exact():
    p = tensorgen.make_tucker_problem((10, 9, 8), (3, 2, 3), seed=8, eta=0.2)
    A0, G0 = ot.hosvd(p.X, p.ranks)
    A1, G1, _ = ot.tucker_als(p.X, A0, G0, 2)
    st = ot.build_operators(p.X, A1)
    A_pp = [a.copy() for a in A1]
    _, rec = ot.pp_sweep(st, A_pp, G1, float(np.sum(p.X ** 2)), "pp_init")
    A_als = [a.copy() for a in A1]
    _, ref, _ = ot.tucker_sweep(p.X, A_als, G1)
    np.testing.assert_allclose(rec.rhs[0], ref.rhs[0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(A_pp[0], A_als[0], atol=1e-12)


def test_eps_zero_is_plain_tucker_als_and_replay_reproduces_the_free_run():
    p = tensorgen.make_tucker_problem((12, 10, 11), (3, 3, 3), seed=9, eta=0.05)
    A0, G0 = ot.hosvd(p.X, p.ranks)
    A_a, G_a, r_a = ot.tucker_als(p.X, A0, G0, 6)
    A_b, G_b, r_b = ot.pp_tucker_als(p.X, A0, G0, eps=0.0, sweeps=6)
    assert [r.kind for r in r_b] == ["als"] * 6
    for a, b in zip(A_a, A_b):
        assert np.array_equal(a, b)
    A_c, G_c, r_c = ot.pp_tucker_als(p.X, A0, G0, eps=0.3, sweeps=12)
    kinds = [r.kind for r in r_c]
    assert "pp_approx" in kinds
    A_d, G_d, r_d = ot.pp_tucker_als(p.X, A0, G0, eps=0.3, sweeps=12, replay=kinds)
    for a, b in zip(A_c, A_d):
        assert np.array_equal(a, b)
    # PP tracks Tucker-ALS: the fit after 12 sweeps is within 1e-6 of plain ALS's
    _, _, r_e = ot.tucker_als(p.X, A0, G0, 12)
    assert abs(r_c[-1].fit - r_e[-1].fit) < 1e-6
