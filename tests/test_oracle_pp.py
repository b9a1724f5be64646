"""Pins for the pairwise-perturbation part of the oracle (Section 3, Algorithm 3,
Section 4.1 and the appendix error bound)."""
import os
from math import comb

import numpy as np
import pytest

import tensorgen
from oracle import cp, pp, tree


def _setup(shape, R, seed, eta=1e-2):
    p = tensorgen.make_problem(shape, R, seed=seed, eta=eta)
    A, _ = cp.cp_als(p.X, p.init, 3)
    return p.X, A


@pytest.mark.parametrize("shape", [(5, 6, 7), (4, 5, 3, 6), (3, 4, 3, 2, 3)])
def test_zero_perturbation_gives_exact_mttkrp(shape):
    """With dA = 0 the PP update reduces to M_p^(n), the exact MTTKRP."""
    X, A = _setup(shape, 3, 1)
    st = pp.build_operators(X, A)
    S = [cp.gram(a) for a in A]
    for n in range(len(shape)):
        np.testing.assert_allclose(pp.pp_rhs(st, A, S, n), cp.mttkrp(X, A, n), rtol=1e-12, atol=1e-12)


def test_order3_exact_cp_model_is_reproduced_exactly():
    """Section 3.1: for N = 3 the only error of the PP right-hand side with the
    second-order correction is (X - [[A]])_(n)(dA (.) dA); if X equals the CP
    model of the current factors, M~^(n) is exact.  This fixes the pair sum to
    unordered pairs: counting ordered pairs doubles V and breaks exactness."""
    rng = np.random.default_rng(0)
    shape, R = (6, 7, 8), 4
    A = [rng.standard_normal((s, R)) for s in shape]
    Ap = [a + 0.05 * rng.standard_normal(a.shape) for a in A]
    X = cp.cp_full(A)
    st = pp.build_operators(X, Ap)
    st.dA = [a - b for a, b in zip(A, Ap)]
    S = [cp.gram(a) for a in A]
    for n in range(3):
        exact = cp.mttkrp(X, A, n)
        approx = pp.pp_rhs(st, A, S, n)
        assert np.linalg.norm(approx - exact) <= 1e-12 * np.linalg.norm(exact)
        # ordered-pair reading: V counted twice
        twice = approx + A[n] @ pp.second_order_matrix(A, S, st.dA, n)
        assert np.linalg.norm(twice - exact) > 1e-4 * np.linalg.norm(exact)
        # without V: an O(t^2) error remains
        first = pp.pp_rhs(st, A, S, n, second_order=False)
        assert np.linalg.norm(first - exact) > 1e-4 * np.linalg.norm(exact)


def test_error_is_second_order_without_correction():
    """Theorem on the PP error without second-order terms: the error of the
    right-hand side scales as O(eps^2) in the perturbation size."""
    X, A0 = _setup((8, 9, 10), 4, 2, eta=0.05)
    rng = np.random.default_rng(3)
    D = [rng.standard_normal(a.shape) for a in A0]
    errs = []
    for t in (1e-1, 1e-2, 1e-3):
        A = [a + t * d for a, d in zip(A0, D)]
        st = pp.build_operators(X, A0)
        st.dA = [a - b for a, b in zip(A, A0)]
        S = [cp.gram(a) for a in A]
        exact = cp.mttkrp(X, A, 0)
        approx = pp.pp_rhs(st, A, S, 0, second_order=False)
        errs.append(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
    slope1 = np.log10(errs[0] / errs[1])
    slope2 = np.log10(errs[1] / errs[2])
    assert 1.9 < slope1 < 2.1 and 1.95 < slope2 < 2.05, errs


def test_correction_error_scales_with_residual():
    """Theorem with second-order corrections: the leading error is proportional
    to how far X is from the CP model; shrinking the noise 100x shrinks it ~100x
    (order-4 case, so terms beyond the pairs also exist at O(eps^3))."""
    rng = np.random.default_rng(4)
    shape, R = (5, 6, 5, 6), 3
    A = [rng.standard_normal((s, R)) for s in shape]
    Ap = [a + 1e-3 * rng.standard_normal(a.shape) for a in A]
    E = rng.standard_normal(shape)
    T = cp.cp_full(A)
    errs = []
    for eta in (1e-1, 1e-3):
        X = T + eta * np.linalg.norm(T) * E / np.linalg.norm(E)
        st = pp.build_operators(X, Ap)
        st.dA = [a - b for a, b in zip(A, Ap)]
        S = [cp.gram(a) for a in A]
        exact = cp.mttkrp(X, A, 0)
        errs.append(np.linalg.norm(pp.pp_rhs(st, A, S, 0) - exact) / np.linalg.norm(exact))
    assert 50 < errs[0] / errs[1] < 200, errs


@pytest.mark.parametrize("s", [4, 8])
def test_unit_condition_error_equals_product_of_relative_perturbations(golden_dir, s):
    """Appendix theorem on the PP-CP error with the tensor condition number: on
    a perfectly conditioned order-3 tensor the column error of the mode-1
    right-hand side without corrections is ||T x da2_k x da3_k|| = ||da2_k|| ||da3_k||
    while ||m_k|| = ||a2_k|| ||a3_k||; the relative error is the product of the
    relative perturbations, within the bound C(3,2) kappa eps^2 with kappa = 1."""
    T = np.zeros((s, s, s))
    for line in open(os.path.join(golden_dir, f"unit_condition_s{s}.txt")):
        if line.startswith("#"):
            continue
        i, j, k, v = line.split()
        T[int(i) - 1, int(j) - 1, int(k) - 1] = float(v)
    rng = np.random.default_rng(s)
    R = 3
    Ap = [rng.standard_normal((s, R)) for _ in range(3)]
    dA = [1e-2 * rng.standard_normal((s, R)) for _ in range(3)]
    A = [a + d for a, d in zip(Ap, dA)]
    st = pp.build_operators(T, Ap)
    st.dA = dA
    S = [cp.gram(a) for a in A]
    exact = cp.mttkrp(T, A, 0)
    approx = pp.pp_rhs(st, A, S, 0, second_order=False)
    rel = np.linalg.norm(approx - exact, axis=0) / np.linalg.norm(exact, axis=0)
    want = (np.linalg.norm(dA[1], axis=0) / np.linalg.norm(A[1], axis=0)
            * np.linalg.norm(dA[2], axis=0) / np.linalg.norm(A[2], axis=0))
    np.testing.assert_allclose(rel, want, rtol=1e-9)
    eps = max(np.max(np.linalg.norm(d, axis=0) / np.linalg.norm(a, axis=0)) for d, a in zip(dA, A))
    assert np.all(rel <= comb(3, 2) * eps ** 2)


def test_first_pp_sweep_order3_modes_1_and_2_are_exact():
    """Right after the build dA = 0: mode 1 is exact, and mode 2 sees a single
    nonzero perturbation, for which the first-order expansion is exact."""
    X, A = _setup((7, 8, 9), 3, 5)
    S = [cp.gram(a) for a in A]
    st = pp.build_operators(X, A)
    A_run = [a.copy() for a in A]
    S_run = [s.copy() for s in S]
    rec = pp.pp_sweep(st, A_run, S_run, float(np.sum(X * X)))
    A_ref = [a.copy() for a in A]
    S_ref = [s.copy() for s in S]
    ref = cp.als_sweep(X, A_ref, S_ref)
    for n in (0, 1):
        np.testing.assert_allclose(rec.rhs[n], ref.rhs[n], rtol=1e-11, atol=1e-11)
    assert np.linalg.norm(rec.rhs[2] - ref.rhs[2]) > 0.0


def test_reinterpreted_als_equals_als():
    """Algorithm 5 is algebraically identical to Algorithm 1."""
    p = tensorgen.make_problem((6, 7, 5), 3, seed=8, eta=1e-2)
    A1, _ = cp.cp_als(p.X, p.init, 4)
    A5 = pp.reinterpreted_als(p.X, p.init, 4)
    for a, b in zip(A1, A5):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-10)


def test_eps_zero_never_uses_pp_and_equals_als():
    p = tensorgen.make_problem((6, 7, 8), 3, seed=9, eta=1e-2)
    A_pp, recs = pp.pp_als(p.X, p.init, eps=0.0, sweeps=8)
    A_als, _ = cp.cp_als(p.X, p.init, 8)
    assert all(r.kind == "als" for r in recs)
    for a, b in zip(A_pp, A_als):
        assert np.array_equal(a, b)


def test_pp_als_tracks_als_fit():
    """PP-ALS reaches the fit of ALS on a planted problem (Section 5.1 reports
    PP fitness as high as ALS) and does use PP sweeps."""
    p = tensorgen.make_problem((20, 21, 22), 5, seed=10, eta=1e-3, collinearity=0.5)
    A_pp, recs = pp.pp_als(p.X, p.init, eps=0.1, sweeps=60)
    A_als, _ = cp.cp_als(p.X, p.init, 60)
    kinds = [r.kind for r in recs]
    assert recs[0].kind == "als"
    assert "pp_init" in kinds and "pp_approx" in kinds
    assert abs(cp.fit_direct(p.X, A_pp) - cp.fit_direct(p.X, A_als)) < 1e-4


def test_replay_reproduces_free_run():
    p = tensorgen.make_problem((9, 10, 11), 3, seed=11, eta=1e-3)
    A1, r1 = pp.pp_als(p.X, p.init, eps=0.2, sweeps=25)
    A2, r2 = pp.pp_als(p.X, p.init, eps=0.2, sweeps=25, replay=[r.kind for r in r1])
    for a, b in zip(A1, A2):
        assert np.array_equal(a, b)


def test_switching_rule_semantics():
    """Algorithm 3: first sweep is ALS; every PP run starts with pp_init right
    after a sweep whose rel_change is below eps for all modes; a PP run continues
    exactly while the accumulated change stays below eps; an ALS sweep follows."""
    p = tensorgen.make_problem((12, 13, 14), 4, seed=12, eta=1e-3, collinearity=0.6)
    eps = 0.1
    A, recs = pp.pp_als(p.X, p.init, eps=eps, sweeps=50)
    assert recs[0].kind == "als"
    for prev, cur in zip(recs, recs[1:]):
        small = all(r < eps for r in prev.rel_change)
        if prev.kind == "als":
            assert cur.kind == ("pp_init" if small else "als")
        else:
            assert cur.kind == ("pp_approx" if small else "als")


@pytest.mark.parametrize("N", [3, 4, 5])
def test_pp_tree_leaves_equal_definition(N):
    shape = (3, 4, 2, 3, 2)[:N]
    rng = np.random.default_rng(N)
    X = rng.standard_normal(shape)
    A = [rng.standard_normal((s, 2)) for s in shape]
    leaves = tree.execute_pp_tree(X, A)
    assert len(leaves) == comb(N, 2)
    for (i, j), v in leaves.items():
        np.testing.assert_allclose(v, cp.partial_mttkrp(X, A, (i - 1, j - 1)), rtol=1e-12, atol=1e-12)


def test_pp_tree_cost_formula():
    """Section 3.2.3: build cost 2R sum C(l+1,2) s^(N-l+2) = 6 s^N R + 12 s^(N-1) R + ..."""
    for N in range(3, 7):
        for s in (7, 40):
            assert tree.pp_tree_build_flops((s,) * N, 5) == tree.pp_build_flops_formula(s, N, 5)
    assert tree.pp_build_flops_formula(10, 3, 1) == 6 * 10 ** 3
    assert tree.pp_build_flops_formula(100, 4, 1) == 6 * 100 ** 4 + 12 * 100 ** 3
    # leading term is 1.5x the dimension-tree ALS sweep (Table 1: 6 s^N R vs 4 s^N R)
    s, N, R = 1000, 3, 1
    assert tree.pp_build_flops_formula(s, N, R) / tree.dt_als_level1_flops((s,) * N, R) == 1.5


def test_pp_tree_children_per_parent_n4():
    nodes = tree.pp_tree(4)
    lvl3 = [(c, p, w) for (l, c, p, w) in nodes if l == 3]
    parents = {}
    for c, p, w in lvl3:
        parents.setdefault(p, []).append((c, w))
    assert parents[(1, 2, 4)] == [((1, 2), 4)]
    assert sorted(parents[(1, 3, 4)]) == [((1, 3), 4), ((1, 4), 3)]
    assert sorted(parents[(2, 3, 4)]) == [((2, 3), 4), ((2, 4), 3), ((3, 4), 2)]
