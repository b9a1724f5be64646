"""GPU parity of the Tucker path (Tucker-ALS, Algorithm 2; PP-Tucker-ALS, Algorithm 4 with
the first-order TTMc of Section 3.2.2) against the float64 oracle, at orders 3 to 8.

Layouts: the library stores Y^(n) as s_n x R^(N-1) with x_n first and the rank indices of
the other modes in increasing mode order (the oracle's ttmc with mode n moved to the
front); the core is (r_1, .., r_N) on both sides.  Tolerances: TTMc and core are contractions of length <= s^2
accumulated in FP64 (relative 1e-12 of the |.|-weighted sum is far above gamma_K u);
factors come from a subspace iteration stopped at a Ritz residual of 1e-12 relative to
the largest eigenvalue, whose eigenvector error is that residual times
lambda_1 / (lambda_R - lambda_{R+1}); the planted problems keep that ratio below 1e3,
so factor entries are compared at 1e-8."""
import numpy as np
import pytest

import tensorgen
from oracle import tucker as ot

from gpu_util import to_dev

pytestmark = pytest.mark.gpu

pk = pytest.importorskip("paper_1811_10573_amd")

def lib_layout(Y, n):
    """Oracle Y^(n) (natural order) -> library layout (x_n first)."""
    return np.ascontiguousarray(np.moveaxis(Y, n, 0))


def host(t, shape=None):
    a = t.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


class TRun:
    def __init__(self, shape, R, seed=0, eta=0.1):
        self.prob = tensorgen.make_tucker_problem(shape, (R,) * len(shape), seed=seed, eta=eta)
        self.shape = tuple(shape)
        self.N = len(shape)
        self.R = R
        self.plan = pk.TuckerPlan(shape, R)
        self.X = to_dev(self.prob.X)
        self.ws = self.plan.workspace(self.X.device)
        self.normX2 = float(np.sum(self.prob.X ** 2))

    def upload(self, A, G):
        self.A = [to_dev(a) for a in A]
        self.G = to_dev(G)

    def factors(self):
        return [host(a, (s, self.R)) for a, s in zip(self.A, self.shape)]

    def core(self):
        return host(self.G, (self.R,) * self.N)

    def ranks(self):
        return (self.R,) * self.N

    def zero_core(self):
        return np.zeros((self.R,) * self.N)

    def zero_y(self, n):
        return np.zeros((self.shape[n],) + (self.R,) * (self.N - 1))


def assert_rel(got, want, tol, what):
    err = np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300)
    assert err <= tol, f"{what}: relative error {err:.3e} > {tol:.1e}"


@pytest.mark.parametrize("shape,R", [((37, 29, 23), 5), ((70, 64, 66), 16), ((96, 80, 72), 64),
                                     ((14, 12, 11, 10), 3), ((9, 8, 7, 8, 6), 3),
                                     ((6, 5, 6, 5, 6, 5), 2), ((5, 4, 5, 4, 5, 4, 3), 2), ((4, 3, 4, 3, 4, 3, 4, 3), 2)])
def test_ttmc_matches_oracle(shape, R):
    """Y^(n) = X x_{i != n} A^(i)T for every mode: ragged sizes, several level-1 tiles,
    the largest rank."""
    r = TRun(shape, R, seed=1)
    rng = np.random.default_rng(2)
    A = [np.linalg.qr(rng.standard_normal((s, R)))[0] for s in shape]
    r.upload(A, r.zero_core())
    for n in range(r.N):
        Y = to_dev(r.zero_y(n))
        pk.tucker_ttmc(r.plan, r.ws, r.X, r.A, n, Y)
        want = lib_layout(ot.ttmc(r.prob.X, A, n), n)
        assert_rel(host(Y, want.shape), want, 1e-12, f"Y^({n})")


@pytest.mark.parametrize("shape,R", [((37, 29, 23), 5), ((96, 80, 72), 64)])
def test_factor_update_matches_eigh(shape, R):
    """Leading eigenvectors of Y_(n) Y_(n)^T, oriented against the previous factor, from a
    TTMc the oracle made (one HOOI step past the HOSVD)."""
    r = TRun(shape, R, seed=3)
    A0, _ = ot.hosvd(r.prob.X, r.ranks())
    A1, _, _ = ot.tucker_als(r.prob.X, A0, ot.hosvd(r.prob.X, r.ranks())[1], 1)
    for n in range(r.N):
        Yn = ot.ttmc(r.prob.X, A1, n)
        want, _ = ot.leading_eigvecs(Yn, n, R, prev=A0[n])
        Y = to_dev(lib_layout(Yn, n))
        prev = to_dev(A0[n])
        out = to_dev(np.zeros_like(A0[n]))
        info = pk.tucker_factor_update(r.plan, r.ws, Y, n, prev, out)
        assert info["converged"] == 1 and info["rr_status"] == 0, info
        np.testing.assert_allclose(host(out, want.shape), want, atol=1e-8, rtol=0)
        # in place (A_out == A_prev)
        pk.tucker_factor_update(r.plan, r.ws, Y, n, prev, prev)
        np.testing.assert_allclose(host(prev, want.shape), want, atol=1e-8, rtol=0)


@pytest.mark.parametrize("shape,R", [((41, 33, 27), 4), ((90, 84, 70), 20), ((14, 12, 11, 10), 3),
                                     ((9, 8, 7, 8, 6), 3), ((5, 4, 5, 4, 5, 4, 3), 2),
                                     ((4, 3, 4, 3, 4, 3, 4, 3), 2), ((600, 20, 18), 4),
                                     ((20, 600, 18), 4), ((20, 18, 16), 1)])
def test_hosvd_matches_oracle(shape, R):
    """HOSVD from random starting bases: factors (largest-magnitude entry positive) and
    core against the oracle's eigh-based HOSVD (the first, inner and last modes' products,
    the inner one on the strided first-level kernel; 600-row modes split k)."""
    r = TRun(shape, R, seed=5)
    A_want, G_want = ot.hosvd(r.prob.X, r.ranks())
    V0 = [to_dev(v) for v in tensorgen.subspace_start(shape, R, seed=6)]
    r.upload([np.zeros_like(a) for a in A_want], r.zero_core())
    info = pk.tucker_hosvd(r.plan, r.ws, r.X, V0, r.A, r.G)
    assert all(i[1] == 1 and i[2] == 0 for i in info), info
    for n, (got, want) in enumerate(zip(r.factors(), A_want)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"A^({n})")
    assert_rel(r.core(), G_want, 1e-8, "core")


@pytest.mark.parametrize("shape,R", [((41, 33, 27), 4), ((90, 84, 70), 20), ((14, 12, 11, 10), 3),
                                     ((9, 8, 7, 8, 6), 3), ((6, 5, 6, 5, 6, 5), 2), ((5, 4, 5, 4, 5, 4, 3), 2), ((4, 3, 4, 3, 4, 3, 4, 3), 2),
                                     ((600, 20, 18), 4)])
def test_interlaced_hosvd_matches_oracle(shape, R):
    """Interlaced HOSVD (each factor from the prefix Z^(n) = X x_0 A^(0)T .. x_(n-1)
    A^(n-1)T, whose first mode is n) against the oracle's."""
    r = TRun(shape, R, seed=5)
    A_want, G_want = ot.hosvd_interlaced(r.prob.X, r.ranks())
    V0 = [to_dev(v) for v in tensorgen.subspace_start(shape, R, seed=6)]
    r.upload([np.zeros_like(a) for a in A_want], r.zero_core())
    info = pk.tucker_hosvd_interlaced(r.plan, r.ws, r.X, V0, r.A, r.G)
    assert all(i[1] == 1 and i[2] == 0 for i in info), info
    for n, (got, want) in enumerate(zip(r.factors(), A_want)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"A^({n})")
    assert_rel(r.core(), G_want, 1e-8, "core")


@pytest.mark.parametrize("shape,R", [((37, 29, 23), 5), ((96, 80, 72), 24), ((14, 12, 11, 10), 3),
                                     ((9, 8, 7, 8, 6), 2), ((1400, 20, 18), 12),
                                     ((120, 20, 20, 20), 16), ((5, 4, 5, 4, 5, 4, 3), 2), ((4, 3, 4, 3, 4, 3, 4, 3), 2)])
def test_als_sweeps_match_oracle(shape, R):
    """Six HOOI sweeps from the oracle's HOSVD: factors, core and every record field.
    W V = Y (Y^T V) runs in one chunked kernel while Y's chunk, V and Y_chunk^T V fit a
    workgroup's LDS, else as two first-level contractions (mode 0 of 1400 x 20 x 18 at
    R = 12).  For R <= 16 and s_n R <= 2048 one workgroup takes the rest of the step,
    adding the chunks itself when there are at most 32 (mode 0 of 120 x 20^3 at R = 16
    has 36, added by a separate launch first)."""
    r = TRun(shape, R, seed=7, eta=0.3)
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    r.upload(A0, G0)
    A_w, G_w, recs_w = ot.tucker_als(r.prob.X, A0, G0, 6)
    for k in range(6):
        rec = pk.tucker_als_sweep(r.plan, r.ws, r.X, r.A, r.G, r.normX2)
        w = recs_w[k]
        assert rec["kind"] == "als"
        assert all(rec["converged"]) and not any(rec["rr_status"]), rec
        assert abs(rec["fit"] - w.fit) <= 1e-10, (k, rec["fit"], w.fit)
        assert abs(rec["core_norm"] - w.core_norm) <= 1e-10 * w.core_norm
        assert abs(rec["f_norm"] - w.f_norm) <= 1e-7 * w.core_norm + 1e-9 * w.f_norm
        np.testing.assert_allclose(rec["rel_change"], w.rel_change, rtol=1e-5, atol=1e-9)
    for n, (got, want) in enumerate(zip(r.factors(), A_w)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"A^({n})")
    assert_rel(r.core(), G_w, 1e-8, "core")


@pytest.mark.parametrize("shape,R", [((60, 52, 47), 8), ((14, 12, 11, 10), 3), ((9, 8, 7, 8, 6), 2),
                                     ((5, 4, 5, 4, 5, 4, 3), 2), ((4, 3, 4, 3, 4, 3, 4, 3), 2),
                                     ((13,) * 6, 6), ((330, 320, 310), 20)])
def test_pp_operators_and_rhs_match_oracle(shape, R):
    """Build at the HOSVD factors, one PP-init sweep (which sets dA), then the
    first-order TTMc of every mode against the oracle's from the same dA.  Small
    operators take the in-place sum of the terms (one launch; 2 to 16 lanes per output
    element, one at 13^6, R = 6); 330 x 320 x 310 at R = 20 (about 8e7 multiply-adds per
    mode) contracts term by term on the first-level kernel."""
    r = TRun(shape, R, seed=9, eta=0.2)
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    A1, G1, _ = ot.tucker_als(r.prob.X, A0, G0, 1)
    r.upload(A1, G1)
    pk.tucker_pp_build(r.plan, r.ws, r.X, r.A)
    st = ot.build_operators(r.prob.X, A1)
    # zero perturbation: the approximated TTMc is the exact one at A_p
    for n in range(r.N):
        Y = to_dev(r.zero_y(n))
        pk.tucker_pp_rhs(r.plan, r.ws, n, Y)
        want = lib_layout(ot.pp_rhs(st, n), n)
        assert_rel(host(Y, want.shape), want, 1e-12, f"Y_p^({n})")
    rec = pk.tucker_pp_sweep(r.plan, r.ws, r.A, r.G, r.normX2, "pp_init")
    A_or = [a.copy() for a in A1]
    _, rec_w = ot.pp_sweep(st, A_or, G1, r.normX2, "pp_init")
    assert rec["kind"] == "pp_init"
    assert abs(rec["fit"] - rec_w.fit) <= 1e-10
    # the oracle's dA and the library's agree to the factor tolerance; compare the rhs
    # with the oracle evaluated at the library's dA
    st.dA = [got - ap for got, ap in zip(r.factors(), A1)]
    for n in range(r.N):
        Y = to_dev(r.zero_y(n))
        pk.tucker_pp_rhs(r.plan, r.ws, n, Y)
        want = lib_layout(ot.pp_rhs(st, n), n)
        assert_rel(host(Y, want.shape), want, 1e-11, f"Y~^({n})")
    for n, (got, want) in enumerate(zip(r.factors(), A_or)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"A^({n})")


@pytest.mark.parametrize("shape,R,sweeps", [((48, 44, 40), 6, 14), ((120, 110, 100), 12, 12),
                                            ((18, 16, 15, 14), 3, 12), ((9, 8, 9, 8, 9), 2, 12),
                                            ((5, 4, 5, 4, 5, 4, 3), 2, 12),
                                            ((4, 3, 4, 3, 4, 3, 4, 3), 2, 12),
                                            ((20, 18, 16), 1, 8), ((9, 8, 7, 8), 1, 8)])
def test_pp_tucker_run_matches_oracle(shape, R, sweeps):
    """Algorithm 4 with eps = 0.3 (the paper's Tucker setting): the library's own
    decisions give the oracle's sweep-kind sequence, and the replayed path ends at the
    oracle's factors and core; every record's fit within 1e-10."""
    r = TRun(shape, R, seed=11, eta=0.05)
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    A_w, G_w, recs_w = ot.pp_tucker_als(r.prob.X, A0, G0, eps=0.3, sweeps=sweeps)
    kinds_w = [w.kind for w in recs_w]
    assert "pp_approx" in kinds_w
    r.upload(A0, G0)
    recs = pk.tucker_run(r.plan, r.ws, r.X, r.A, r.G, eps=0.3, sweeps=sweeps)
    assert [x["kind"] for x in recs] == kinds_w
    for x, w in zip(recs, recs_w):
        assert abs(x["fit"] - w.fit) <= 1e-10, (x, w.fit)
    for n, (got, want) in enumerate(zip(r.factors(), A_w)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"A^({n})")
    assert_rel(r.core(), G_w, 1e-8, "core")
    # replay of the same kinds from the start reproduces the free run
    r.upload(A0, G0)
    recs2 = pk.tucker_run(r.plan, r.ws, r.X, r.A, r.G, eps=0.3, sweeps=sweeps, replay=kinds_w)
    assert [x["kind"] for x in recs2] == kinds_w
    for n, (got, want) in enumerate(zip(r.factors(), A_w)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"replay A^({n})")


@pytest.mark.parametrize("shape,R", [((16, 1031, 1021), 5), ((11, 13, 97, 1001), 3),
                                     ((12, 1101, 999), 8), ((40, 9, 10, 11, 300), 4)])
def test_small_rank_vector_contractions_match_oracle(shape, R):
    """Contractions of more than 2^20 rows over an odd trailing extent at R <= 8 run on the
    vector-unit kernel: the prefix X x_0 A^(0)T at every size (K = 16, 11, 12: steps of 4
    with remainders 0, 3, 0) and at order 4 the first step of mode 0's chain, X x_1
    A^(1)T (K = 13, remainder 1; 11 slices of an odd trailing extent 97097, so a wave's
    rows cross slices); no row count is a multiple of the 1024 rows of a workgroup.  The
    HOSVDs' product X_(0) Z (16, 11 and 12 rows of more than 2^20 contiguous k) and the
    classical HOSVD's X_(n) Z for the inner modes of 13 rows at order 4 and of 9, 10 and 11
    rows at order 5 (row strides 97097, 33000, 3300 and 300) run on the rows kernel (k
    split over workgroups, the parts added in order).  TTMc of every mode,
    two HOOI sweeps, the classical and the interlaced HOSVD and a PP-Tucker run
    (eps = 0.3) against the oracle."""
    r = TRun(shape, R, seed=17, eta=0.05)
    rng = np.random.default_rng(18)
    A = [np.linalg.qr(rng.standard_normal((s, R)))[0] for s in shape]
    r.upload(A, r.zero_core())
    for n in range(r.N):
        Y = to_dev(r.zero_y(n))
        pk.tucker_ttmc(r.plan, r.ws, r.X, r.A, n, Y)
        want = lib_layout(ot.ttmc(r.prob.X, A, n), n)
        assert_rel(host(Y, want.shape), want, 1e-12, f"Y^({n})")
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    A_w, G_w, recs_w = ot.tucker_als(r.prob.X, A0, G0, 2)
    r.upload(A0, G0)
    for k in range(2):
        rec = pk.tucker_als_sweep(r.plan, r.ws, r.X, r.A, r.G, r.normX2)
        assert abs(rec["fit"] - recs_w[k].fit) <= 1e-10, (k, rec["fit"], recs_w[k].fit)
    for n, (got, want) in enumerate(zip(r.factors(), A_w)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"HOOI A^({n})")
    assert_rel(r.core(), G_w, 1e-8, "HOOI core")
    V0 = [to_dev(v) for v in tensorgen.subspace_start(shape, R, seed=19)]
    r.upload([np.zeros_like(a) for a in A0], r.zero_core())
    info = pk.tucker_hosvd(r.plan, r.ws, r.X, V0, r.A, r.G)
    assert all(i[1] == 1 and i[2] == 0 for i in info), info
    for n, (got, want) in enumerate(zip(r.factors(), A0)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"classical HOSVD A^({n})")
    assert_rel(r.core(), G0, 1e-8, "classical HOSVD core")
    A_i, G_i = ot.hosvd_interlaced(r.prob.X, r.ranks())
    V0 = [to_dev(v) for v in tensorgen.subspace_start(shape, R, seed=19)]
    r.upload([np.zeros_like(a) for a in A_i], r.zero_core())
    info = pk.tucker_hosvd_interlaced(r.plan, r.ws, r.X, V0, r.A, r.G)
    assert all(i[1] == 1 and i[2] == 0 for i in info), info
    for n, (got, want) in enumerate(zip(r.factors(), A_i)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"HOSVD A^({n})")
    assert_rel(r.core(), G_i, 1e-8, "HOSVD core")
    A_p, G_p, recs_p = ot.pp_tucker_als(r.prob.X, A0, G0, eps=0.3, sweeps=8)
    kinds = [w.kind for w in recs_p]
    assert "pp_approx" in kinds
    r.upload(A0, G0)
    recs = pk.tucker_run(r.plan, r.ws, r.X, r.A, r.G, eps=0.3, sweeps=8)
    assert [x["kind"] for x in recs] == kinds
    for x, w in zip(recs, recs_p):
        assert abs(x["fit"] - w.fit) <= 1e-10, (x, w.fit)
    for n, (got, want) in enumerate(zip(r.factors(), A_p)):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"PP A^({n})")
    assert_rel(r.core(), G_p, 1e-8, "PP core")


def test_eps_zero_is_hooi():
    shape, R = (40, 38, 36), 5
    r = TRun(shape, R, seed=13, eta=0.1)
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    A_w, G_w, _ = ot.tucker_als(r.prob.X, A0, G0, 5)
    r.upload(A0, G0)
    recs = pk.tucker_run(r.plan, r.ws, r.X, r.A, r.G, eps=0.0, sweeps=5)
    assert [x["kind"] for x in recs] == ["als"] * 5
    for got, want in zip(r.factors(), A_w):
        np.testing.assert_allclose(got, want, atol=1e-8, rtol=0)


def test_pp_sweep_needs_a_build():
    shape, R = (20, 18, 16), 3
    r = TRun(shape, R, seed=15)
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    r.upload(A0, G0)
    with pytest.raises(pk.PPALSError) as e:
        pk.tucker_pp_sweep(r.plan, r.ws, r.A, r.G, r.normX2)
    assert e.value.status == -5


def test_pp_sweeps_through_every_solver_path_match_oracle():
    """PP sweeps run one unchecked subspace iteration per mode first and redo from the
    first mode that did not converge.  A tolerance the first iteration cannot meet forces
    the redo (all modes, capped iteration count); the following sweeps run checked until
    one needs a single iteration in every mode, and the sweep after such a sweep runs
    unchecked again.  Every sweep's factors and fit against the oracle's."""
    shape, R = (60, 52, 47), 8
    r = TRun(shape, R, seed=17, eta=0.2)
    A0, G0 = ot.hosvd(r.prob.X, r.ranks())
    A1, G1, _ = ot.tucker_als(r.prob.X, A0, G0, 2)
    r.upload(A1, G1)
    pk.tucker_pp_build(r.plan, r.ws, r.X, r.A)
    st = ot.build_operators(r.prob.X, A1)
    A_or, G_or = [a.copy() for a in A1], G1.copy()
    plan_iters = []
    for k, tol in enumerate([1e-30, 1e-12, 1e-12, 1e-12, 1e-12]):
        r.plan.set_solver(tol, 4 if tol < 1e-20 else 500, 5000)
        kind = "pp_init" if k == 0 else "pp_approx"
        rec = pk.tucker_pp_sweep(r.plan, r.ws, r.A, r.G, r.normX2, kind)
        G_or, w = ot.pp_sweep(st, A_or, G_or, r.normX2, kind)
        plan_iters.append(rec["iters"])
        assert abs(rec["fit"] - w.fit) <= 1e-10, (k, rec, w.fit)
        for n, (got, want) in enumerate(zip(r.factors(), A_or)):
            np.testing.assert_allclose(got, want, atol=1e-8, rtol=0, err_msg=f"sweep {k} A^({n})")
        assert_rel(r.core(), G_or, 1e-8, f"sweep {k} core")
    assert plan_iters[0] == [4, 4, 4], plan_iters
    # the last sweep follows a sweep with one iteration per mode: the unchecked pass
    assert plan_iters[-2] == [1, 1, 1] and plan_iters[-1] == [1, 1, 1], plan_iters
