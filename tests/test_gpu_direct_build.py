"""GPU parity of the combined operator builds of Section 3.2.3: the nodes of tree level
l + 1 are X contracted with the Khatri-Rao product of l factors in one first-level launch
(through strided row and k offsets when the contracted modes are not one contiguous
block), the later levels come from their parents; l = N - 2 computes every operator
M_p^(i,j) from X and stores no O(s^(N-1) R) intermediate.  Operators against their
definition, whole runs against the oracle, and combined against tree builds."""
import numpy as np
import pytest
import torch

import tensorgen
from oracle import cp as ocp
from oracle import pp as opp

from gpu_util import U32, U64, Run, assert_within, dev, fp32_round, oracle_sensitivity, rel

pytestmark = pytest.mark.gpu

pp = pytest.importorskip("paper_1811_10573_amd")


@pytest.mark.parametrize("tier", ["f64", "f32"])
@pytest.mark.parametrize("dims,R,build", [((9, 8, 7, 10), 5, "direct"), ((20, 22, 18, 16), 7, "direct"),
                                          ((5, 4, 6, 5, 4), 3, "direct"), ((5, 4, 6, 5, 4), 3, 2),
                                          ((4, 3, 5, 3, 4, 3), 4, "direct"), ((4, 3, 5, 3, 4, 3), 4, 2),
                                          ((4, 3, 5, 3, 4, 3), 4, 3), ((66, 65, 64, 64), 50, "direct")])
def test_direct_operators_match_definition(tier, dims, R, build):
    """Every operator of a combined build against the definition (partial MTTKRP),
    Higham bound for a K-term sum; strided steps for the non-contiguous contracted sets;
    the full direct build keeps no intermediate."""
    prob = tensorgen.make_problem(dims, R, seed=4, eta=1e-2)
    A = [fp32_round(a) for a in prob.init] if tier == "f32" else prob.init
    r = Run(prob, tier, init=A, pp_build=build)
    d = r.plan.describe()
    want_levels = len(dims) - 2 if build == "direct" else build
    assert d["pp_build_levels"] == want_levels
    if build == "direct":
        assert d["pp_build"] == "direct" and d["pp_build_intermediate_bytes"] == 0
    assert any(o.get("strided") for o in d["pp_build_ops"])
    pp.pp_build_operators(r.plan, r.X, r.Xb, r.A, r.ws)
    st = opp.build_operators(r.Xh, A)
    u = U64 if tier == "f64" else U32
    total = int(np.prod(dims))
    for (i, j), op in st.ops.items():
        out = torch.empty(dims[i] * dims[j] * R, dtype=r.plan.torch_dtype, device=dev())
        pp.get_operator(r.plan, r.ws, i, j, out)
        base = ocp.partial_mttkrp(np.abs(r.Xh), [np.abs(a) for a in A], (i, j))
        K = total // (dims[i] * dims[j])
        assert_within(out.cpu().numpy().reshape(op.shape), op, (K + 4) * u * base,
                      f"{tier} direct operator ({i},{j}) {dims}")


@pytest.mark.parametrize("dims,R,eps,build", [((12, 14, 11, 13), 5, 0.2, "direct"),
                                              ((7, 6, 8, 5, 6), 3, 0.2, "direct"),
                                              ((7, 6, 8, 5, 6), 3, 0.2, 2),
                                              ((6, 5, 4, 5, 4, 5), 3, 0.2, "auto"),
                                              ((40, 36, 34, 32), 12, 0.1, "direct")])
def test_direct_build_run_matches_oracle(dims, R, eps, build):
    """Free PP-ALS with a combined build; the oracle replays the sweep kinds.  Factors
    within the sensitivity bound, last fit within 1e-10; the oracle's free run takes the
    same decisions."""
    prob = tensorgen.make_problem(dims, R, seed=8, eta=1e-3, collinearity=0.5)
    r = Run(prob, pp_build=build)
    recs, _ = pp.run(r.plan, r.X, None, r.A, r.S, r.normX2, r.ws, r.rec, eps=eps, max_sweeps=40)
    kinds = [x["kind"] for x in recs]
    assert "pp_approx" in kinds, kinds
    A_or, ref = opp.pp_als(prob.X, prob.init, eps=eps, sweeps=40, replay=kinds)
    sens = oracle_sensitivity(
        lambda A: opp.pp_als(prob.X, A, eps=eps, sweeps=40, replay=kinds)[0], prob.init)
    tol = max(1e-8, 1e3 * sens)
    for n in range(len(dims)):
        assert rel(r.factors()[n], A_or[n]) < tol, (n, tol)
    assert abs(recs[-1]["fit_est"] - ref[-1].fit_est) <= 1e-10
    _, free = opp.pp_als(prob.X, prob.init, eps=eps, sweeps=40)
    assert [x.kind for x in free] == kinds


@pytest.mark.parametrize("tier", ["f64", "f32"])
def test_direct_and_tree_builds_agree(tier):
    """The same replayed run (ALS, ALS, PP-init with the reused tree tensor, PP sweeps)
    with both builds: factors agree to the tier's rounding level."""
    dims, R = (30, 28, 26, 24), 10
    prob = tensorgen.make_problem(dims, R, seed=12, eta=1e-3, collinearity=0.3)
    kinds = ["als", "als", "pp_init", "pp_approx", "pp_approx", "als"]
    out = {}
    for build in ("tree", "direct"):
        r = Run(prob, tier, pp_build=build)
        recs, _ = pp.run(r.plan, r.X, r.Xb, r.A, r.S, r.normX2, r.ws, r.rec, eps=0.1,
                         max_sweeps=len(kinds), replay=kinds)
        assert [x["kind"] for x in recs] == kinds
        out[build] = (r.factors(), [x["fit_est"] for x in recs])
    tol = 1e-10 if tier == "f64" else 1e-4
    for a, b in zip(out["tree"][0], out["direct"][0]):
        assert rel(a, b) < tol
    for fa, fb in zip(out["tree"][1], out["direct"][1]):
        assert abs(fa - fb) <= (1e-12 if tier == "f64" else 1e-6)
