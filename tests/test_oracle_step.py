"""Pins of the step-size variant of Section 5.1 in the oracle:
A_new = (1 - lambda) A + lambda M Gamma^-1 (ALS and PP sweeps alike)."""
import numpy as np
import pytest

import tensorgen
from oracle import cp, pp


def _problem(shape=(7, 8, 9), R=3, seed=5, eta=1e-2):
    p = tensorgen.make_problem(shape, R, seed=seed, eta=eta)
    A, _ = cp.cp_als(p.X, p.init, 3)
    return p.X, A


def test_unit_step_is_algorithm_1_bit_for_bit():
    X, A = _problem()
    A1, r1 = cp.cp_als(X, A, 3)
    A2, r2 = cp.cp_als(X, A, 3, step=1.0)
    for a, b in zip(A1, A2):
        assert np.array_equal(a, b)
    assert [r.fit_est for r in r1] == [r.fit_est for r in r2]


@pytest.mark.parametrize("lam", [0.3, 0.7])
def test_damped_update_follows_the_quadratic_along_the_newton_direction(lam):
    """For fixed other factors the objective is a convex quadratic in A^(n) with Hessian
    Gamma (Section 2.3).  With D = (undamped update) - A, moving by lam D lowers it by
    exactly (lam - lam^2/2) <D Gamma, D>.  A step taken from the wrong end,
    (1 - lam) D, gives a different decrease for lam != 1/2."""
    p = tensorgen.make_problem((7, 8, 9), 3, seed=5, eta=1e-2)
    X, A = p.X, p.init          # far from a stationary point in every mode
    for n in range(3):
        S = [cp.gram(a) for a in A]
        M = cp.mttkrp(X, A, n)
        A_full = [a.copy() for a in A]
        cp.als_update(A_full, [s.copy() for s in S], n, M)
        A_lam = [a.copy() for a in A]
        cp.als_update(A_lam, [s.copy() for s in S], n, M, step=lam)
        D = A_full[n] - A[n]
        gamma = cp.hadamard_except(S, n)
        drop = cp.objective(X, A) - cp.objective(X, A_lam)
        want = (lam - lam * lam / 2.0) * float(np.sum(D * (D @ gamma)))
        assert abs(drop - want) <= 1e-9 * abs(want), (n, drop, want)
        assert drop > 0.0


def test_gradient_is_reported_before_the_damped_update():
    """Reading: ||G|| is the gradient norm at the factor before the update, whatever the
    step size (it only depends on A, Gamma and M)."""
    X, A = _problem()
    S = [cp.gram(a) for a in A]
    M = cp.mttkrp(X, A, 1)
    g1 = cp.als_update([a.copy() for a in A], [s.copy() for s in S], 1, M)[2]
    g7 = cp.als_update([a.copy() for a in A], [s.copy() for s in S], 1, M, step=0.7)[2]
    assert g1 == g7
    # the gradient of 1/2 ||X - [[A]]||^2 in A^(1) by central differences
    h = 1e-6
    E = np.zeros_like(A[1])
    E[2, 1] = 1.0
    Ap = [a.copy() for a in A]
    Am = [a.copy() for a in A]
    Ap[1] = A[1] + h * E
    Am[1] = A[1] - h * E
    fd = (cp.objective(X, Ap) - cp.objective(X, Am)) / (2 * h)
    G = A[1] @ cp.hadamard_except(S, 1) - M
    assert abs(fd - G[2, 1]) <= 1e-6 * max(1.0, abs(fd))


def test_first_damped_pp_sweep_order3_modes_1_and_2_equal_damped_als():
    """The first PP sweep after a build equals the ALS sweep in modes 1 and 2 (dA = 0 for
    the modes after them), also with a step size, and the right-hand side of mode 3
    differs from the exact one."""
    X, A = _problem((6, 7, 8), 3, 11)
    st = pp.build_operators(X, A)
    A_pp = [a.copy() for a in A]
    rec = pp.pp_sweep(st, A_pp, [cp.gram(a) for a in A_pp], float(np.sum(X * X)), step=0.7)
    A_als = [a.copy() for a in A]
    ref = cp.als_sweep(X, A_als, [cp.gram(a) for a in A_als], step=0.7)
    for n in (0, 1):
        np.testing.assert_allclose(A_pp[n], A_als[n], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(rec.rhs[n], ref.rhs[n], rtol=1e-11, atol=1e-11)
    assert np.linalg.norm(rec.rhs[2] - ref.rhs[2]) > 0.0


def test_damped_als_converges_on_a_planted_tensor():
    """With lambda = 0.7 the iteration still reaches the planted noise floor."""
    p = tensorgen.make_problem((10, 11, 12), 3, seed=2, eta=1e-4)
    A, recs = cp.cp_als(p.X, p.init, 200, step=0.7)
    assert 1.0 - cp.fit_direct(p.X, A) < 2e-4
    fits = [r.fit_est for r in recs]
    # non-decreasing up to the cancellation of the fit identity at the noise floor
    assert all(b >= a - 1e-10 for a, b in zip(fits[5:], fits[6:]))
