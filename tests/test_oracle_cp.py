"""Pins for the float64 oracle: MTTKRP, CP model, normal-equation solve, CP-ALS.

Every check here compares the oracle with something other than itself: brute
force loops, an explicit unfolding x Khatri-Rao product, the paper's perfectly
conditioned tensors (appendix fixtures under tests/golden), closed-form
identities of Section 2.3, or the behaviour of exact block minimisation.
"""
import itertools
import os

import numpy as np
import pytest

import tensorgen
from oracle import cp, linalg

SHAPES = [(3, 5, 7), (2, 3, 4, 5), (2, 3, 2, 3, 2)]


def _rand_factors(shape, R, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((s, R)) for s in shape]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("R", [1, 3, 4])
def test_mttkrp_definition_matches_brute_force(shape, R):
    rng = np.random.default_rng(hash((shape, R)) % 2**32)
    X = rng.standard_normal(shape)
    A = _rand_factors(shape, R, 7)
    for n in range(len(shape)):
        ref = cp.mttkrp_loops(X, A, n)
        np.testing.assert_allclose(cp.mttkrp(X, A, n), ref, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(cp.mttkrp_explicit(X, A, n), ref, rtol=1e-13, atol=1e-13)


def _partial_loops(X, A, keep):
    R = A[0].shape[1]
    out = np.zeros(tuple(X.shape[m] for m in keep) + (R,))
    for idx in itertools.product(*[range(s) for s in X.shape]):
        for k in range(R):
            p = X[idx]
            for r in range(X.ndim):
                if r not in keep:
                    p *= A[r][idx[r], k]
            out[tuple(idx[m] for m in keep) + (k,)] += p
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_partial_intermediates_match_brute_force(shape):
    rng = np.random.default_rng(3)
    X = rng.standard_normal(shape)
    A = _rand_factors(shape, 3, 11)
    N = len(shape)
    for keep in list(itertools.combinations(range(N), 2)) + [tuple(range(N - 1))]:
        np.testing.assert_allclose(cp.partial_mttkrp(X, A, keep), _partial_loops(X, A, keep),
                                   rtol=1e-13, atol=1e-13)


def _load_unit(golden_dir, s):
    T = np.zeros((s, s, s))
    with open(os.path.join(golden_dir, f"unit_condition_s{s}.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            i, j, k, v = line.split()
            T[int(i) - 1, int(j) - 1, int(k) - 1] = float(v)
    return T


@pytest.mark.parametrize("s", [2, 4, 8])
def test_unit_condition_tensors_contract_isometrically(golden_dir, s):
    """Appendix, well-conditioned tensors: ||T x_2 x x_3 y|| = ||x|| ||y||.
    The MTTKRP of mode 1 with R columns applies that map column by column."""
    T = _load_unit(golden_dir, s)
    rng = np.random.default_rng(s)
    R = 5
    A = [np.zeros((s, R)), rng.standard_normal((s, R)), rng.standard_normal((s, R))]
    M = cp.mttkrp(T, A, 0)
    want = np.linalg.norm(A[1], axis=0) * np.linalg.norm(A[2], axis=0)
    np.testing.assert_allclose(np.linalg.norm(M, axis=0), want, rtol=1e-14)


def test_cp_full_matches_independent_reconstruction():
    A = _rand_factors((4, 3, 5), 2, 5)
    full = cp.cp_full(A)
    ref = np.zeros((4, 3, 5))
    for i, j, k, r in itertools.product(range(4), range(3), range(5), range(2)):
        ref[i, j, k] += A[0][i, r] * A[1][j, r] * A[2][k, r]
    np.testing.assert_allclose(full, ref, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(tensorgen.cp_reconstruct(A), ref, rtol=1e-13, atol=1e-13)


def test_solve_normal_matches_dense_solve():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((40, 9))
    gamma = B.T @ B
    M = rng.standard_normal((17, 9))
    a, st = linalg.solve_normal(gamma, M)
    assert st == 0
    np.testing.assert_allclose(a @ gamma, M, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(a, np.linalg.solve(gamma, M.T).T, rtol=1e-10)


def test_solve_normal_jitter_on_singular_gram():
    """A zero factor column makes Gamma singular; the jitter retry kicks in."""
    rng = np.random.default_rng(1)
    B = rng.standard_normal((30, 4))
    B[:, 2] = 0.0
    gamma = B.T @ B
    M = rng.standard_normal((5, 4))
    M[:, 2] = 0.0
    a, st = linalg.solve_normal(gamma, M)
    assert st == 1
    assert np.all(np.isfinite(a))
    assert linalg.jitter(gamma) == 4 * 2.0 ** -52 * np.max(np.diag(gamma))


def test_gradient_identity():
    """Section 2.3: G = A Gamma - X_(n) P = (A - A_new) Gamma."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((6, 7, 8))
    A = _rand_factors(X.shape, 4, 3)
    S = [cp.gram(a) for a in A]
    for n in range(3):
        gamma = cp.hadamard_except(S, n)
        M = cp.mttkrp(X, A, n)
        a_new, _ = linalg.solve_normal(gamma, M)
        np.testing.assert_allclose(A[n] @ gamma - M, (A[n] - a_new) @ gamma, rtol=1e-10, atol=1e-10)
        # G is also the gradient of 1/2 ||X - [[A]]||^2 (finite-difference check on a few entries)
        G = A[n] @ gamma - M
        for (x, k) in [(0, 0), (3, 2), (5, 3)]:
            h = 1e-6
            Ap = [a.copy() for a in A]
            Am = [a.copy() for a in A]
            Ap[n][x, k] += h
            Am[n][x, k] -= h
            fd = (cp.objective(X, Ap) - cp.objective(X, Am)) / (2 * h)
            assert abs(fd - G[x, k]) < 1e-6 * max(1.0, abs(G[x, k]))


def test_als_mode_updates_never_increase_objective():
    """Each mode update is an exact block minimisation (Section 2.3)."""
    p = tensorgen.make_problem((7, 8, 9), 4, seed=4, planted_rank=4, eta=0.1)
    A = [a.copy() for a in p.init]
    S = [cp.gram(a) for a in A]
    f_prev = cp.objective(p.X, A)
    for _ in range(5):
        for n in range(3):
            M = cp.mttkrp(p.X, A, n)
            cp.als_update(A, S, n, M)
            f = cp.objective(p.X, A)
            assert f <= f_prev * (1 + 1e-12) + 1e-14
            f_prev = f


def test_planted_noise_free_recovery():
    """ALS recovers a noise-free planted rank-3 tensor: fit -> 1 and the factors
    match the planted ones up to column permutation and scaling."""
    p = tensorgen.make_problem((10, 11, 12), 3, seed=5, eta=0.0)
    A, recs = cp.cp_als(p.X, p.init, 300)
    assert cp.fit_direct(p.X, A) > 1 - 1e-8
    for n in range(3):
        a = A[n] / np.linalg.norm(A[n], axis=0)
        b = p.planted[n] / np.linalg.norm(p.planted[n], axis=0)
        C = np.abs(a.T @ b)
        assert np.all(np.max(C, axis=1) > 1 - 1e-6)


def test_fit_identity_matches_direct_fit():
    p = tensorgen.make_problem((9, 10, 11), 4, seed=6, eta=1e-2)
    A, recs = cp.cp_als(p.X, p.init, 6)
    assert abs(recs[-1].fit_est - cp.fit_direct(p.X, A)) < 1e-12


def test_fit_identity_order4():
    p = tensorgen.make_problem((5, 6, 4, 7), 3, seed=7, eta=1e-2)
    A, recs = cp.cp_als(p.X, p.init, 4)
    assert abs(recs[-1].fit_est - cp.fit_direct(p.X, A)) < 1e-12


def test_gram_hadamard():
    A = _rand_factors((3, 4, 5, 6), 3, 9)
    S = [cp.gram(a) for a in A]
    g = cp.hadamard_except(S, 2)
    for r in range(3):
        for q in range(3):
            want = 1.0
            for i in (0, 1, 3):
                want *= float(np.dot(A[i][:, r], A[i][:, q]))
            assert abs(g[r, q] - want) < 1e-12 * max(1.0, abs(want))


def test_first_failed_pivot_is_the_first_non_positive_leading_minor():
    """Cholesky runs through column k-1 exactly when the leading minors of orders 1..k are
    positive (a textbook fact): the failing pivot is the first leading minor <= 0."""
    from oracle import linalg as olinalg
    rng = np.random.default_rng(4)
    B = rng.standard_normal((12, 6))
    spd = B.T @ B
    assert olinalg.first_failed_pivot(spd) == -1
    for k in range(6):
        g = spd.copy()
        g[k, :] = 0.0
        g[:, k] = 0.0
        minors = [np.linalg.det(g[:m, :m]) for m in range(1, 7)]
        want = next(m for m, d in enumerate(minors) if d <= 1e-12 * abs(minors[0]))
        assert olinalg.first_failed_pivot(g) == want == k
    ind = np.diag([1.0, 2.0, -1.0, 3.0])
    assert olinalg.first_failed_pivot(ind) == 2


def test_first_failed_pivot_with_non_finite_entries():
    from oracle import linalg as olinalg
    g = np.eye(5) * 2.0
    g[3, 1] = g[1, 3] = np.nan
    assert olinalg.first_failed_pivot(g) == 3
    g = np.eye(5)
    g[2, 2] = -1.0
    g[4, 0] = g[0, 4] = np.inf
    assert olinalg.first_failed_pivot(g) == 2
