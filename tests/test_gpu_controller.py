"""GPU parity of the learned PP controller: the network's forward, gradient and Adam
kernels against the float64 oracle, the measured right-hand-side error against the
oracle's PP update and MTTKRP, and the driver's controller mode."""
import math

import numpy as np
import pytest
import torch

import paper_1811_10573_amd as pp
import tensorgen
from gpu_util import dev, to_dev
from oracle import cp as ocp
from oracle import mlp as omlp
from oracle import pp as opp

pytestmark = pytest.mark.gpu


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _net(d, H, B, seed):
    rng = np.random.default_rng(seed)
    p = f32(rng.normal(0.0, 0.6, omlp.n_params(d, H)))
    X = f32(rng.normal(0.0, 1.5, (B, d)))
    t = f32(rng.normal(0.0, 1.0, B))
    return p, X, t


def _run_fwd_bwd(p, X, t, d, H):
    B = X.shape[0]
    pd, Xd, td = (to_dev(a, torch.float32) for a in (p, X, t))
    y = torch.empty(B, dtype=torch.float32, device=dev())
    h = torch.empty(B * H, dtype=torch.float32, device=dev())
    g = torch.empty_like(pd)
    loss = torch.empty(1, dtype=torch.float32, device=dev())
    pp.mlp_forward(pd, d, H, Xd, y, h)
    pp.mlp_backward(pd, d, H, Xd, h, y, td, g, loss)
    torch.cuda.synchronize()
    return (y.cpu().numpy().astype(np.float64), h.cpu().numpy().reshape(B, H).astype(np.float64),
            g.cpu().numpy().astype(np.float64), float(loss.item()))


@pytest.mark.parametrize("d,H,B", [(5, 64, 256), (7, 64, 256), (5, 37, 253), (1, 100, 3), (16, 130, 65)])
def test_forward_and_gradient_match_oracle(d, H, B):
    p, X, t = _net(d, H, B, seed=d * 1000 + H + B)
    y, h, g, L = _run_fwd_bwd(p, X, t, d, H)
    y_or, h_or = omlp.forward(p, X, d, H)
    L_or, g_or = omlp.loss_and_grad(p, X, t, d, H)
    # FP32: |y| error <= ~(d + H) u32 * sum |terms|
    scale_y = np.abs(h_or) @ np.abs(omlp.unpack(p, d, H)[2]) + 1.0
    assert np.all(np.abs(y - y_or) <= 1e-5 * scale_y)
    assert np.max(np.abs(h - h_or)) <= 1e-5
    assert abs(L - L_or) <= 1e-4 * L_or
    assert np.linalg.norm(g - g_or) <= 1e-4 * np.linalg.norm(g_or)


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(3)
    P = 1000
    p, g, m = (f32(rng.normal(size=P)) for _ in range(3))
    v = f32(np.abs(rng.normal(size=P)) * 0.1)
    pd, gd, md, vd = (to_dev(a, torch.float32) for a in (p, g, m, v))
    for step in (1, 7):
        want_p, want_m, want_v = omlp.adam_step(p, g, m, v, step, 1e-2)
        pd2, md2, vd2 = pd.clone(), md.clone(), vd.clone()
        pp.mlp_adam(pd2, gd, md2, vd2, step, 1e-2)
        torch.cuda.synchronize()
        assert np.max(np.abs(pd2.cpu().numpy() - want_p)) <= 1e-6 * (1 + np.max(np.abs(want_p)))
        assert np.max(np.abs(md2.cpu().numpy() - want_m)) <= 1e-6
        assert np.max(np.abs(vd2.cpu().numpy() - want_v)) <= 1e-6


def test_training_loop_on_device_reduces_loss():
    d, H, B = 5, 64, 256
    rng = np.random.default_rng(11)
    X = f32(rng.uniform(-2, 2, (B, d)))
    t = f32(np.sin(X[:, 0]) - 0.5 * X[:, 1] * X[:, 2] + 0.1 * X[:, 3])
    p0 = f32(rng.normal(0, 0.2, omlp.n_params(d, H)))
    pd, Xd, td = (to_dev(a, torch.float32) for a in (p0, X, t))
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    y = torch.empty(B, dtype=torch.float32, device=dev())
    h = torch.empty(B * H, dtype=torch.float32, device=dev())
    g = torch.empty_like(pd)
    loss = torch.empty(1, dtype=torch.float32, device=dev())
    first = None
    for step in range(1, 801):
        pp.mlp_forward(pd, d, H, Xd, y, h)
        pp.mlp_backward(pd, d, H, Xd, h, y, td, g, loss)
        if first is None:
            first = float(loss.item())
        pp.mlp_adam(pd, g, m, v, step, 3e-3)
    pp.mlp_forward(pd, d, H, Xd, y, h)
    pp.mlp_backward(pd, d, H, Xd, h, y, td, g, loss)
    last = float(loss.item())
    assert last < 0.05 * first
    # the oracle agrees on the loss of the trained parameters
    assert abs(omlp.loss(pd.cpu().numpy().astype(np.float64), X, t, d, H) - last) <= 1e-4 * (last + 1e-6)


def _pp_state(dims, R, seed, sweeps_before=6, pp_sweeps=3):
    prob = tensorgen.make_problem(dims, R, seed=seed, eta=1e-2)
    A0, _ = ocp.cp_als(prob.X, prob.init, sweeps_before)
    plan = pp.Plan(dims, R, "f64")
    X = to_dev(prob.X)
    A = [to_dev(a.copy()) for a in A0]
    S = to_dev(np.stack([a.T @ a for a in A0]).reshape(-1))
    ws = plan.workspace(dev())
    rec = pp.new_record(dev())
    nrm = torch.zeros(1, dtype=torch.float64, device=dev())
    pp.tensor_norm2(X, nrm)
    pp.pp_build_operators(plan, X, None, A, ws)
    for _ in range(pp_sweeps):
        pp.pp_sweep(plan, A, S, float(nrm.item()), ws, rec)
    return prob, A0, plan, X, A, S, ws


@pytest.mark.parametrize("dims,R", [((23, 19, 21), 4), ((8, 9, 7, 8), 6), ((6, 5, 7, 4, 5), 3)])
def test_rhs_error_matches_oracle(dims, R):
    prob, A0, plan, X, A, S, ws = _pp_state(dims, R, seed=21)
    err = torch.zeros(1, dtype=torch.float64, device=dev())
    pp.pp_rhs_error(plan, X, None, A, S, ws, err)
    torch.cuda.synchronize()
    Ah = [a.cpu().numpy().reshape(s, R) for a, s in zip(A, dims)]
    st = opp.build_operators(prob.X, A0)
    st.dA = [a - b for a, b in zip(Ah, A0)]
    Sh = [a.T @ a for a in Ah]
    Mt = [opp.pp_rhs(st, Ah, Sh, n) for n in range(len(dims))]
    M = [ocp.mttkrp(prob.X, Ah, n) for n in range(len(dims))]
    want = 10.0 ** omlp.label(Mt, M)
    got = float(err.item())
    assert want > 1e-11
    # e is a difference of two right-hand sides accumulated in different orders:
    # absolute agreement ~ u64 * sqrt(count) relative to ||M||
    assert abs(got - want) <= 1e-6 * want + 1e-13


def test_rhs_error_is_zero_right_after_a_build():
    dims, R = (12, 10, 11), 4
    prob, A0, plan, X, A, S, ws = _pp_state(dims, R, seed=4, pp_sweeps=0)
    err = torch.ones(1, dtype=torch.float64, device=dev())
    pp.pp_rhs_error(plan, X, None, A, S, ws, err)
    torch.cuda.synchronize()
    assert float(err.item()) <= 1e-13


def _controller_run(params, H, log10_tau, check_period, fallback, eps=0.2, sweeps=24, rho_cap=0.6):
    dims, R = (30, 26, 28), 5
    prob = tensorgen.make_problem(dims, R, seed=9, eta=1e-3, collinearity=0.6)
    plan = pp.Plan(dims, R, "f64")
    X = to_dev(prob.X)
    A = [to_dev(a.copy()) for a in prob.init]
    S = torch.zeros(3 * R * R, dtype=torch.float64, device=dev())
    ws = plan.workspace(dev())
    rec = pp.new_record(dev())
    nrm = torch.zeros(1, dtype=torch.float64, device=dev())
    pp.tensor_norm2(X, nrm)
    pp.set_controller(plan, params, hidden=H, log10_tau=log10_tau, rho_cap=rho_cap,
                      check_period=check_period, fallback_factor=fallback)
    recs, _ = pp.run(plan, X, None, A, S, float(nrm.item()), ws, rec, eps=eps, max_sweeps=sweeps)
    pp.set_controller(plan, None)
    return recs


def test_controller_predictions_and_decisions():
    d, H = 5, 16
    rng = np.random.default_rng(2)
    p = f32(rng.normal(0, 0.5, omlp.n_params(d, H)))
    pd = to_dev(p, torch.float32)
    tau = -1.0
    recs = _controller_run(pd, H, tau, check_period=0, fallback=10.0)
    kinds = [r["kind"] for r in recs]
    assert "pp_init" in kinds
    for i, r in enumerate(recs):
        if r["kind"] == "als":
            assert math.isnan(r["ctrl_pred"]) and r["ctrl_leave"] == -1
            continue
        x = f32(omlp.features(r["rel_change"], i, r["fit_est"]))
        y, _ = omlp.forward(p, x[None, :], d, H)
        assert abs(r["ctrl_pred"] - y[0]) <= 1e-5 * (1 + abs(y[0]))
        assert r["ctrl_leave"] == (1 if r["ctrl_pred"] >= tau else 0)
        if i + 1 < len(recs):
            stay = r["ctrl_leave"] == 0 and max(r["rel_change"]) < 0.6
            assert recs[i + 1]["kind"] == ("pp_approx" if stay else "als")


def test_controller_falls_back_after_a_failed_check():
    d, H = 5, 8
    # b2 = -30 and zero weights: the network always predicts an error of 1e-30,
    # so only the fallback can end its PP phases
    p = np.zeros(omlp.n_params(d, H))
    p[-1] = -30.0
    pd = to_dev(p, torch.float32)
    recs = _controller_run(pd, H, -2.0, check_period=2, fallback=1e-20)
    pp_idx = [i for i, r in enumerate(recs) if r["kind"] != "als"]
    assert len(pp_idx) >= 2
    second = pp_idx[1]
    assert recs[second]["ctrl_true_err"] > 0.0
    assert all(r["ctrl_fallback"] == 0 for r in recs[:second])
    assert all(r["ctrl_fallback"] == 1 for r in recs[second:])
    # after the fallback the threshold rule decides (eps = 0.2)
    for i in range(second, len(recs) - 1):
        if recs[i]["kind"] != "als":
            small = max(recs[i]["rel_change"]) < 0.2
            assert recs[i + 1]["kind"] == ("pp_approx" if small else "als")


def test_learned_controller_end_to_end_small():
    """Labels from the method, training on the device, a threshold from the training
    split and the controller against the threshold rule on held-out seeds (a small
    version of the order-3 experiment; the full-size run is reported separately).

    What the network itself gains is measured against the ablation that keeps the rest
    of the controller (leaving at rho_cap = 3 eps, periodic exact checks, fallback) and
    replaces the network by a constant that never asks to leave.  At full size that
    share is a loss of 1-2% at both orders (the gain at order 5 comes from rho_cap and
    the checks): a prediction of the right-hand-side error does not tell when leaving
    the PP phase pays, because staying costs less than a rebuild until rho_cap.  The
    test asserts that this absence holds here too: the network's share stays below
    1.10 (geometric mean over the held-out runs both arms bring to the target)."""
    from paper_1811_10573_amd import controller as ctl
    res, params = ctl.experiment(3, list(range(0, 40)), list(range(40, 50)), list(range(2000, 2008)),
                                 shape=(60, 60, 60), max_sweeps=150, steps=1500, progress_every=10,
                                 tau_search_runs=6, target=0.95)
    print({k: v for k, v in res.items() if k != "per_run"})
    assert res["labels"]["train"] >= 100 and res["labels"]["val"] >= 20
    # the network explains most of the label variance on held-out runs
    assert res["val_r2"] is not None and res["val_r2"] > 0.5
    ev = res["eval"]
    assert ev["runs"] == 8
    # tau comes from the search on training problems: its training-split gain is the
    # best of the candidates
    assert res["log10_tau"] in [t for t, _ in res["tau_search"]]
    assert max(g for _, g in res["tau_search"]) == dict(res["tau_search"])[res["log10_tau"]]
    share = ev["network_vs_capped"]
    assert share["both_reached"] >= 3, ev
    assert share["speedup_geomean"] < 1.10, share
    # the ablation arm never leaves on a prediction: it keeps more PP sweeps than the
    # threshold rule wherever rho stays below rho_cap
    assert sum(e["pp_capped"] >= e["pp_fixed"] for e in res["per_run"]) >= len(res["per_run"]) // 2
