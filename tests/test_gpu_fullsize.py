"""GPU parity of the benchmarked kernel branches against the float64 oracle.

* FP32-tier right-hand sides and PP sweeps element by element (the tier the
  benchmark measures), with bounds derived from FP32 accumulation.
* Free PP-ALS runs whose largest mode has 400-800 rows, so that the PP sweeps'
  Gram tiles are split into 2-4 row ranges exchanged between workgroups, with
  sweeps enqueued ahead of the host decision and graph replay (Algorithm 3).
* The 800^3 rank-50 decomposition itself (collinearity 0.9) in FP64 and FP32.
* Ranks above 64 (the general-rank tail) through whole ALS and PP sweeps.

Every oracle input comes from the seeded generators or from the oracle itself;
the GPU's sweep-kind sequence is replayed by the oracle so that a threshold tie
cannot fork the two trajectories (the free oracle's own decisions are checked
where no tie is near).
"""
import numpy as np
import pytest
import torch

import tensorgen
from oracle import cp as ocp
from oracle import pp as opp

from gpu_util import U32, U64, Run, assert_within, dev, fp32_round, oracle_fit, oracle_sensitivity, rel, to_dev

pytestmark = pytest.mark.gpu

pp = pytest.importorskip("paper_1811_10573_amd")


def kinds_of(recs):
    return [x["kind"] for x in recs]


def longest_pp_run(kinds):
    best = cur = 0
    for k in kinds:
        cur = cur + 1 if k == "pp_approx" else 0
        best = max(best, cur)
    return best


# ---------------------------------------------------------------------------
# FP32 tier, element by element
# ---------------------------------------------------------------------------

def f32_operator_unit(dims):
    """Relative accumulation bound of an FP32-tier operator entry, in units of u32: the
    first-level contraction sums at most max(dims) products in FP32 (Higham's gamma_K),
    every later tree level adds one FP32 rounding of its FP64 sum, plus slack."""
    return max(dims) + 2 * len(dims) + 4


@pytest.mark.parametrize("second_order", [True, False])
@pytest.mark.parametrize("dims,R", [((13, 11, 12), 3), ((9, 8, 7, 10), 5), ((400, 30, 28), 8),
                                    ((30, 20, 25), 16), ((6, 5, 7, 5, 4), 3), ((30, 26, 34), 5)])
def test_pp_rhs_f32_matches_oracle(dims, R, second_order):
    """General PP update (Section 3.2.1) in the FP32 tier, every entry of every mode:
    the operators are FP32 sums of FP32-exact inputs (X and A_p rounded to FP32 on both
    sides), the correction weights dA and the second-order term are FP64."""
    prob = tensorgen.make_problem(dims, R, seed=5, eta=1e-2)
    Ap = [fp32_round(a) for a in prob.init]
    r = Run(prob, "f32", second_order, init=Ap)
    pp.pp_build_operators(r.plan, r.X, None, r.A, r.ws)
    st = opp.build_operators(r.Xh, Ap)
    rng = np.random.default_rng(6)
    A = [a + 0.03 * rng.standard_normal(a.shape) for a in Ap]
    st.dA = [a - b for a, b in zip(A, Ap)]
    S = [a.T @ a for a in A]
    Ad = [to_dev(a) for a in A]
    Sd = to_dev(np.stack(S).reshape(-1))
    absX = np.abs(r.Xh)
    absAp = [np.abs(a) for a in Ap]
    K = f32_operator_unit(dims)
    N = len(dims)
    for n in range(N):
        out = torch.empty(dims[n] * R, dtype=torch.float64, device=dev())
        pp.pp_rhs(r.plan, Ad, Sd, n, out, r.ws)
        want = opp.pp_rhs(st, A, S, n, second_order)
        base = ocp.mttkrp(absX, absAp, n)
        for i in range(N):
            if i == n:
                continue
            lo, hi = min(i, n), max(i, n)
            bop = ocp.partial_mttkrp(absX, absAp, (lo, hi))
            sub = "xyk,xk->yk" if i < n else "yxk,xk->yk"
            base = base + np.einsum(sub, bop, np.abs(st.dA[i]))
        fp64 = 64 * U64 * (np.abs(want) + base)
        if second_order:
            fp64 = fp64 + 64 * U64 * np.abs(A[n]) @ np.abs(opp.second_order_matrix(A, S, st.dA, n))
        assert_within(out.cpu().numpy().reshape(dims[n], R), want, K * U32 * base + fp64,
                      f"f32 pp_rhs mode {n} {dims} R={R}")


def perturbed_state(st, Xh, Ap, dims, scale, rng):
    """The oracle's operators with every entry moved by scale * |X| |A_p| contraction *
    N(0,1): the size and sign pattern of FP32 accumulation error, for the sensitivity
    of the oracle's trajectory to it."""
    absX = np.abs(Xh)
    absAp = [np.abs(a) for a in Ap]
    ops = {k: v + scale * ocp.partial_mttkrp(absX, absAp, k) * rng.standard_normal(v.shape)
           for k, v in st.ops.items()}
    Mp = [m + scale * ocp.mttkrp(absX, absAp, n) * rng.standard_normal(m.shape)
          for n, m in enumerate(st.Mp)]
    return opp.PPState(Ap=[a.copy() for a in st.Ap], dA=[d.copy() for d in st.dA], ops=ops, Mp=Mp)


@pytest.mark.parametrize("dims,R", [((23, 19, 21), 4), ((400, 30, 28), 8), ((8, 9, 7, 8), 6),
                                    ((30, 26, 34), 5)])
def test_pp_sweeps_f32_match_oracle(dims, R):
    """Operator build and four PP sweeps in the FP32 tier from the same FP32-exact start on
    both sides (after eight oracle ALS sweeps on float64(float32(X))), every factor entry
    after every sweep.  Bound: 30x the oracle's own response to an operator perturbation
    of FP32-accumulation size (sqrt(K) u32 times the |X| |A| contraction, random sign);
    the 30 covers the worst-case K against the typical sqrt(K) growth."""
    prob = tensorgen.make_problem(dims, R, seed=7, eta=1e-3)
    Xh = fp32_round(prob.X)
    A0, _ = ocp.cp_als(Xh, [fp32_round(a) for a in prob.init], 8)
    A0 = [fp32_round(a) for a in A0]
    r = Run(prob, "f32", init=A0)
    pp.pp_build_operators(r.plan, r.X, None, r.A, r.ws)
    normX2 = float(np.sum(Xh ** 2))
    K = max(dims)
    st0 = opp.build_operators(Xh, A0)
    stp = perturbed_state(st0, Xh, A0, dims, np.sqrt(K) * U32, np.random.default_rng(11))

    def sweeps(state, k):
        st = opp.PPState(Ap=[a.copy() for a in state.Ap], dA=[d.copy() for d in state.dA],
                         ops=state.ops, Mp=state.Mp)
        A = [a.copy() for a in A0]
        S = [a.T @ a for a in A]
        recs = [opp.pp_sweep(st, A, S, normX2, True, "pp_init" if q == 0 else "pp_approx")
                for q in range(k)]
        return A, recs

    for k in range(1, 5):
        pp.pp_sweep(r.plan, r.A, r.S, r.normX2, r.ws, r.rec)
        A_or, recs_or = sweeps(st0, k)
        A_pt, recs_pt = sweeps(stp, k)
        got = pp.read_record(r.rec)
        assert got["kind"] == recs_or[-1].kind
        G = r.factors()
        for n in range(len(dims)):
            sens = max(rel(A_pt[n], A_or[n]), 1e-9 / 30)
            colnorm = np.linalg.norm(A_or[n], axis=0, keepdims=True)
            assert_within(G[n], A_or[n], 30 * sens * colnorm * np.ones_like(A_or[n]),
                          f"f32 PP sweep {k} mode {n} {dims}", slack=1.0)
        fsens = max(abs(recs_pt[-1].fit_est - recs_or[-1].fit_est), 1e-10)
        assert abs(got["fit_est"] - recs_or[-1].fit_est) <= 30 * fsens, (k, got["fit_est"], recs_or[-1].fit_est)


# ---------------------------------------------------------------------------
# Row-range Grams, sweeps enqueued ahead, graph replay (modes of 400-800 rows)
# ---------------------------------------------------------------------------

ROW_RANGE_CASES = [((800, 40, 36), 32, 4), ((600, 40, 36), 32, 3), ((400, 64, 56), 50, 2)]


@pytest.mark.parametrize("tier", ["f64", "f32"])
@pytest.mark.parametrize("dims,R,ranges", ROW_RANGE_CASES)
def test_row_range_gram_runs_match_oracle(dims, R, ranges, tier):
    """Free PP-ALS (eps = 0.1, 40 sweeps) through the driver: ALS and PP-init sweeps from
    graphs, PP sweeps enqueued ahead behind the device-side threshold test, and the
    first mode's Gram tiles split into `ranges` row ranges.  The oracle replays the kind
    sequence.  FP64: factors within the sensitivity bound and the fit estimate of every
    sweep within 1e-10 relative; FP32: final fit within 1e-5 of the FP64 oracle's.
    Collinearity 0.3 lets every case converge (fit 0.999) within the 40 sweeps, so the
    final fit is a property of the problem, not of where a swamp leaves the run."""
    prob = tensorgen.make_problem(dims, R, seed=31, eta=1e-3, collinearity=0.3)
    r = Run(prob, tier)
    d = r.plan.describe()
    assert d["fused_tail"] and d["pp_gram_ranges"][0] == ranges
    recs, _ = r.run(eps=0.1, max_sweeps=40)
    kinds = kinds_of(recs)
    assert longest_pp_run(kinds) >= 3, kinds
    A_or, ref = opp.pp_als(prob.X, prob.init, eps=0.1, sweeps=40, replay=kinds)
    if tier == "f64":
        sens = oracle_sensitivity(
            lambda A: opp.pp_als(prob.X, A, eps=0.1, sweeps=40, replay=kinds)[0], prob.init)
        tol = max(1e-8, 1e3 * sens)
        G = r.factors()
        for n in range(len(dims)):
            assert rel(G[n], A_or[n]) < tol, (n, rel(G[n], A_or[n]), tol)
        for i, (g, o) in enumerate(zip(recs, ref)):
            assert abs(g["fit_est"] - o.fit_est) <= max(1e-10, tol) * abs(o.fit_est), (i, g["fit_est"], o.fit_est)
        # no threshold tie near this run: the free oracle takes the same decisions
        _, free = opp.pp_als(prob.X, prob.init, eps=0.1, sweeps=40)
        assert [x.kind for x in free] == kinds
    else:
        f_gpu = oracle_fit(prob.X, r.factors())
        f_or = oracle_fit(prob.X, A_or)
        assert abs(f_gpu - f_or) <= 1e-5 * abs(f_or), (f_gpu, f_or)


@pytest.mark.parametrize("tier", ["f64", "f32"])
def test_row_range_graph_replay_equals_eager(tier):
    """With per-kernel profiling on, the driver launches every sweep eagerly and decides
    on the host after each one; without it, it replays graphs and enqueues PP sweeps
    ahead.  At 800 rows (four Gram row ranges) both give the same bits."""
    prob = tensorgen.make_problem((800, 40, 36), 32, seed=31, eta=1e-3, collinearity=0.3)
    out = []
    for profiling in (True, False):
        r = Run(prob, tier)
        recs, _ = r.run(eps=0.1, max_sweeps=40, profiling=profiling)
        out.append((kinds_of(recs), [x["fit_est"] for x in recs], r.factors()))
    assert out[0][0] == out[1][0] and longest_pp_run(out[0][0]) >= 3
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][2], out[1][2]):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# The 800^3, rank-50 decomposition (collinearity 0.9, noise 1e-3)
# ---------------------------------------------------------------------------

C2_SWEEPS = 24


@pytest.fixture(scope="module")
def c2_problem():
    return tensorgen.make_problem((800, 800, 800), 50, seed=0, eta=1e-3, collinearity=0.9)


@pytest.mark.parametrize("tier", ["f64", "f32"])
def test_c2_decomposition_matches_oracle(c2_problem, tier):
    """The benchmarked workload for 24 sweeps (ALS, PP-init with the ALS tree's tensor
    reused, at least three PP sweeps in a row, so sweeps enqueued ahead), replayed by
    the oracle.  FP64: every sweep's fit estimate within 1e-10 relative and the factors
    within the sensitivity bound; FP32: final fit within 1e-5 of the FP64 oracle's."""
    prob = c2_problem
    r = Run(prob, tier)
    assert r.plan.describe()["pp_gram_ranges"] == [4, 4, 4]
    recs, _ = r.run(eps=0.1, max_sweeps=C2_SWEEPS)
    kinds = kinds_of(recs)
    assert longest_pp_run(kinds) >= 3 and "pp_init" in kinds, kinds
    G = r.factors()
    del r
    torch.cuda.empty_cache()
    A_or, ref = opp.pp_als(prob.X, prob.init, eps=0.1, sweeps=C2_SWEEPS, replay=kinds)
    if tier == "f64":
        for i, (g, o) in enumerate(zip(recs, ref)):
            assert abs(g["fit_est"] - o.fit_est) <= 1e-10 * abs(o.fit_est), (i, g["fit_est"], o.fit_est)
        sens = oracle_sensitivity(
            lambda A: opp.pp_als(prob.X, A, eps=0.1, sweeps=C2_SWEEPS, replay=kinds)[0], prob.init)
        tol = max(1e-8, 1e3 * sens)
        for n in range(3):
            assert rel(G[n], A_or[n]) < tol, (n, rel(G[n], A_or[n]), tol)
    else:
        f_gpu = oracle_fit(prob.X, G)
        f_or = oracle_fit(prob.X, A_or)
        assert abs(f_gpu - f_or) <= 1e-5 * abs(f_or), (f_gpu, f_or)


# ---------------------------------------------------------------------------
# Ranks above 64: the general-rank tail
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tier", ["f64", "f32"])
@pytest.mark.parametrize("dims,R", [((96, 90, 100), 80), ((140, 130, 136), 128)])
def test_high_rank_sweeps_match_oracle(dims, R, tier):
    """Whole ALS and PP sweeps at R = 80 and 128 (every mode size above R), which take the
    general-rank tail instead of the fused one: a replayed sequence with an operator
    build, PP sweeps, an ALS sweep and a second build, from the factors after six oracle
    ALS sweeps.  FP64: factors and every fit estimate within the sensitivity bound;
    FP32: final fit within 1e-5 of the FP64 oracle's."""
    prob = tensorgen.make_problem(dims, R, seed=13, eta=1e-2)
    A0, _ = ocp.cp_als(prob.X, prob.init, 6)
    r = Run(prob, tier, init=A0)
    assert not r.plan.describe()["fused_tail"]
    kinds = ["als", "pp_init", "pp_approx", "pp_approx", "pp_approx", "als", "pp_init", "pp_approx"]
    recs, _ = r.run(eps=0.2, max_sweeps=len(kinds), replay=kinds)
    assert kinds_of(recs) == kinds
    A_or, ref = opp.pp_als(prob.X, A0, eps=0.2, sweeps=len(kinds), replay=kinds)
    if tier == "f64":
        sens = oracle_sensitivity(
            lambda A: opp.pp_als(prob.X, A, eps=0.2, sweeps=len(kinds), replay=kinds)[0], A0)
        tol = max(1e-9, 1e3 * sens)
        G = r.factors()
        for n in range(3):
            assert rel(G[n], A_or[n]) < tol, (n, rel(G[n], A_or[n]), tol)
        for g, o in zip(recs, ref):
            assert abs(g["fit_est"] - o.fit_est) <= max(1e-10, tol) * abs(o.fit_est)
            for n in range(3):
                assert g["chol_status"][n] == o.chol_status[n]
    else:
        f_gpu = oracle_fit(prob.X, r.factors())
        f_or = oracle_fit(prob.X, A_or)
        assert abs(f_gpu - f_or) <= 1e-5 * abs(f_or), (f_gpu, f_or)


# ---------------------------------------------------------------------------
# A PP sweep after an explicit rewrite of dA
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,R", [((23, 19, 21), 4), ((9, 8, 7, 10), 5)])
def test_pp_sweep_after_pp_rhs_uses_every_correction(dims, R):
    """build -> new factors -> ppals_pp_rhs (which rewrites dA = A - A_p) -> pp_sweep: the
    first sweep after the build must not skip the correction jobs of modes whose dA is
    no longer zero.  Compared with the oracle's PP sweep from the same state."""
    prob = tensorgen.make_problem(dims, R, seed=17, eta=1e-3)
    A0, _ = ocp.cp_als(prob.X, prob.init, 6)
    A1, _ = ocp.cp_als(prob.X, A0, 1)
    r = Run(prob, "f64", init=A0)
    pp.pp_build_operators(r.plan, r.X, None, r.A, r.ws)
    for n in range(len(dims)):
        r.A[n].copy_(to_dev(A1[n]).reshape(r.A[n].shape))
    r.S.copy_(to_dev(np.stack([a.T @ a for a in A1]).reshape(-1)))
    out = torch.empty(dims[0] * R, dtype=torch.float64, device=dev())
    pp.pp_rhs(r.plan, r.A, r.S, 0, out, r.ws)
    pp.pp_sweep(r.plan, r.A, r.S, r.normX2, r.ws, r.rec)
    normX2 = float(np.sum(prob.X ** 2))

    def one(Ain):
        st = opp.build_operators(prob.X, A0)
        A = [a.copy() for a in Ain]
        st.dA = [a - b for a, b in zip(A, A0)]
        rec = opp.pp_sweep(st, A, [a.T @ a for a in A], normX2, True, "pp_init")
        return A, rec

    A_or, rec = one(A1)
    tol = max(1e-10, 1e3 * oracle_sensitivity(lambda A: one(A)[0], A1))
    G = r.factors()
    for n in range(len(dims)):
        assert rel(G[n], A_or[n]) < tol, (n, rel(G[n], A_or[n]), tol)
    assert abs(pp.read_record(r.rec)["fit_est"] - rec.fit_est) < max(1e-11, tol)


# ---------------------------------------------------------------------------
# Shapes of the paper's real-data experiments, scaled down (uniform factors)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tier", ["f64", "f32"])
@pytest.mark.parametrize("dims,R", [((16, 16, 3, 120), 15), ((48, 64, 33, 9), 20),
                                    ((113, 14, 14), 40)])
def test_paper_shaped_runs_match_oracle(dims, R, tier):
    """Non-equidimensional tensors shaped like the image and chemistry experiments of
    Section 5.1 (a mode of 3 below the rank; modes of 33 and 9; rank above two mode
    sizes), planted with U[0,1) factors and 1e-2 noise: free PP-ALS (eps = 0.1, 30
    sweeps) replayed by the oracle.  FP64 within the sensitivity bound.  FP32: final fit
    within max(1e-5, 100 x the oracle's own fit change when its start moves by 2^-24);
    these runs are still in their transient after 30 sweeps (the image-shaped one
    oscillates between PP phases for 80 sweeps), where FP32 rounding at every
    contraction moves the fit further than one rounding of the start does."""
    prob = tensorgen.make_problem(dims, R, seed=51, eta=1e-2, dist="uniform")
    r = Run(prob, tier)
    recs, _ = r.run(eps=0.1, max_sweeps=30)
    kinds = kinds_of(recs)
    A_or, ref = opp.pp_als(prob.X, prob.init, eps=0.1, sweeps=30, replay=kinds)
    if tier == "f64":
        sens = oracle_sensitivity(
            lambda A: opp.pp_als(prob.X, A, eps=0.1, sweeps=30, replay=kinds)[0], prob.init)
        tol = max(1e-8, 1e3 * sens)
        G = r.factors()
        for n in range(len(dims)):
            assert rel(G[n], A_or[n]) < tol, (n, rel(G[n], A_or[n]), tol)
        for g, o in zip(recs, ref):
            assert abs(g["fit_est"] - o.fit_est) <= max(1e-10, tol) * abs(o.fit_est)
    else:
        f_gpu = oracle_fit(prob.X, r.factors())
        f_or = oracle_fit(prob.X, A_or)
        rng = np.random.default_rng(0)
        A_pt, _ = opp.pp_als(prob.X, [a * (1 + U32 * rng.standard_normal(a.shape)) for a in prob.init],
                             eps=0.1, sweeps=30, replay=kinds)
        sens32 = abs(oracle_fit(prob.X, A_pt) - f_or) / abs(f_or)
        assert abs(f_gpu - f_or) <= max(1e-5, 100 * sens32) * abs(f_or), (kinds, f_gpu, f_or, sens32)


@pytest.mark.parametrize("build", ["tree", "direct"])
def test_image_shaped_operators_at_full_size(build):
    """The PP operators of the full-size image-shaped stand-in (128 x 128 x 3 x 7200,
    R = 15, FP32; Section 3.2.3), built by the PP tree (a level-2 node of 7 GB) and
    straight from X (first-level contractions over up to 128 x 7200 strided k), on
    sampled entries (x_i, x_j, :) that include both ends of every mode.  Each entry is
    the oracle's partial MTTKRP of the slice of X through (x_i, x_j).  Bound per entry:
    Higham's gamma_K for the longest FP32 sum of the build, K * u32 times the same
    contraction of |X| and |A|; and over the samples, the relative error within
    30 sqrt(K) u32 (the typical accumulation error)."""
    shape, R = (128, 128, 3, 7200), 15
    prob = tensorgen.make_problem_device(shape, R, seed=7, eta=1e-2, dist="uniform", dtype="f32",
                                         device=dev())
    A = [fp32_round(a) for a in prob.init]
    plan = pp.Plan(shape, R, "f32", "f32", True, pp_build=build)
    assert plan.describe()["pp_build_levels"] == (1 if build == "tree" else 2)
    ws = plan.workspace(dev())
    pp.pp_build_operators(plan, prob.X.reshape(-1), None, [to_dev(a) for a in A], ws)
    torch.cuda.synchronize()
    Xh = prob.X.reshape(shape).cpu().numpy()
    rng = np.random.default_rng(11)
    for i in range(4):
        for j in range(i + 1, 4):
            out = torch.empty(shape[i] * shape[j] * R, dtype=torch.float32, device=dev())
            pp.get_operator(plan, ws, i, j, out)
            op = out.cpu().numpy().astype(np.float64).reshape(shape[i], shape[j], R)
            K = max(shape) if build == "tree" else int(np.prod(shape)) // (shape[i] * shape[j])
            picks = [(0, 0), (shape[i] - 1, shape[j] - 1)] + [
                (int(rng.integers(shape[i])), int(rng.integers(shape[j]))) for _ in range(6)]
            got, want = [], []
            for xi, xj in picks:
                idx = [slice(None)] * 4
                idx[i], idx[j] = slice(xi, xi + 1), slice(xj, xj + 1)
                sub = Xh[tuple(idx)].astype(np.float64)
                Asub = list(A)
                Asub[i], Asub[j] = A[i][xi:xi + 1], A[j][xj:xj + 1]
                ref = ocp.partial_mttkrp(sub, Asub, (i, j)).reshape(R)
                base = ocp.partial_mttkrp(np.abs(sub), [np.abs(a) for a in Asub], (i, j)).reshape(R)
                assert_within(op[xi, xj], ref, (K + 12) * U32 * base,
                              f"{build} operator ({i},{j}) entry ({xi},{xj})")
                got.append(op[xi, xj])
                want.append(ref)
            err = rel(np.array(got), np.array(want))
            assert err < 30 * np.sqrt(K) * U32, (build, i, j, err)
