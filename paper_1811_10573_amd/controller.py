"""Learned controller for leaving the PP phase of PP-CP-ALS.

Algorithm 3 leaves the PP phase when some ||dA^(i)|| / ||A^(i)|| reaches eps; the
paper names other switching schemes as future work (Section 6).  This module
trains a small network (the library's `ppals_mlp_*` kernels, FP32 on the GPU)
to predict log10 of the PP right-hand-side error

    e = max_n ||M~^(n) - M^(n)||_F / ||M^(n)||_F

from the state of the iteration (per-mode relative changes, sweep index, fit),
on pairs the method itself generates, and evaluates the driver's controller
mode (`ppals_set_controller`) against the threshold rule on time to a target
fit.  Every step runs through the C ABI; this module only orchestrates.

Workload (order-3 300^3 and order-5 40^5 FP32 tensors, planted rank 20..40,
collinearity U[0.5, 0.95], noise 1e-3): one network per order.

Run as `python -m paper_1811_10573_amd.controller --help`.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import Plan, mlp_adam, mlp_backward, mlp_forward, mlp_n_params, new_record, \
    pp_build_operators, pp_rhs_error, pp_sweep, cp_als_sweep, read_record, run, set_controller, \
    tensor_norm2

SHAPES = {3: (300, 300, 300), 5: (40, 40, 40, 40, 40)}


def log(msg):
    print(f"[controller {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def problem_spec(order, seed):
    """Rank ~ U{20..40} and collinearity ~ U[0.5, 0.95] for one seeded run."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), int(order), 7]))
    return int(rng.integers(20, 41)), float(rng.uniform(0.5, 0.95))


def features(rel_change, sweep, fit):
    rc = [math.log10(float(r) + 1e-12) for r in rel_change]
    return rc + [math.log1p(float(sweep)), -math.log10(1.0 - float(fit) + 1e-16)]


class Session:
    """Device buffers and a plan for one decomposition problem."""

    def __init__(self, shape, rank, seed, collinearity, eta=1e-3, device="cuda"):
        import tensorgen
        self.dev = torch.device(device)
        prob = tensorgen.make_problem_device(shape, rank, seed, eta=eta, collinearity=collinearity,
                                             dtype="f32", device=device)
        self.shape = tuple(shape)
        self.rank = rank
        self.plan = Plan(self.shape, rank, "f32", "f32", True)
        self.X = prob.X.reshape(-1)
        self.init = prob.init
        self.A = [torch.from_numpy(a.copy()).to(self.dev) for a in prob.init]
        self.S = torch.zeros(len(shape) * rank * rank, dtype=torch.float64, device=self.dev)
        self.ws = self.plan.workspace(self.dev)
        self.rec = new_record(self.dev)
        nrm = torch.zeros(1, dtype=torch.float64, device=self.dev)
        tensor_norm2(self.X, nrm)
        self.normX2 = float(nrm.item())
        self.err = torch.zeros(1, dtype=torch.float64, device=self.dev)

    def reset(self):
        """Initial factors back in place; the driver with a zero sweep budget only
        forms the Grams S^(n) = A^(n)T A^(n)."""
        for a, a0 in zip(self.A, self.init):
            a.copy_(torch.from_numpy(a0))
        run(self.plan, self.X, None, self.A, self.S, self.normX2, self.ws, self.rec, eps=0.0,
            max_sweeps=0)


def collect(session, eps_gen, max_sweeps):
    """Run Algorithm 3 with threshold eps_gen and record, after every PP sweep, the
    controller features and the measured log10 right-hand-side error."""
    s = session
    s.reset()
    N = len(s.shape)
    rel = [1.0] * N
    prev = None
    feats, labels = [], []
    for it in range(max_sweeps):
        small = all(r < eps_gen for r in rel)
        if small and prev in (None, "als"):
            pp_build_operators(s.plan, s.X, None, s.A, s.ws)
            kind = "pp_init"
        elif small:
            kind = "pp_approx"
        else:
            kind = "als"
        if kind == "als":
            cp_als_sweep(s.plan, s.X, None, s.A, s.S, s.normX2, s.ws, s.rec)
        else:
            pp_sweep(s.plan, s.A, s.S, s.normX2, s.ws, s.rec)
        r = read_record(s.rec)
        rel = r["rel_change"][:N]
        if kind != "als":
            pp_rhs_error(s.plan, s.X, None, s.A, s.S, s.ws, s.err)
            e = float(s.err.item())
            if e > 0.0 and math.isfinite(e):
                feats.append(features(rel, it, r["fit_est"]))
                labels.append(math.log10(e))
        prev = kind
        if r["fit_est"] > 1.0 - 1e-9:
            break
    return feats, labels


def train(X, y, hidden=64, steps=3000, lr=3e-3, batch=256, seed=0, device="cuda", Xval=None,
          yval=None):
    """Fit the network on standardised inputs with the device kernels (minibatch Adam).
    Returns (params for raw inputs, history)."""
    dev = torch.device(device)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = X.shape[1]
    mu = X.mean(axis=0)
    sd = X.std(axis=0) + 1e-6
    Xs = ((X - mu) / sd).astype(np.float32)
    rng = np.random.default_rng(seed)
    P = mlp_n_params(d, hidden)
    p0 = np.concatenate([rng.normal(0, 1.0 / math.sqrt(d), hidden * d), np.zeros(hidden),
                         rng.normal(0, 1.0 / math.sqrt(hidden), hidden), [float(y.mean())]])
    p = torch.tensor(p0, dtype=torch.float32, device=dev)
    m = torch.zeros(P, dtype=torch.float32, device=dev)
    v = torch.zeros(P, dtype=torch.float32, device=dev)
    g = torch.zeros(P, dtype=torch.float32, device=dev)
    Xd = torch.from_numpy(Xs).to(dev)
    yd = torch.from_numpy(y.astype(np.float32)).to(dev)
    n = Xs.shape[0]
    B = min(batch, n)
    yb = torch.empty(B, dtype=torch.float32, device=dev)
    hb = torch.empty(B * hidden, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    hist = []
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (B,), generator=gen).to(dev)
        xb = Xd.index_select(0, idx).contiguous()
        tb = yd.index_select(0, idx).contiguous()
        mlp_forward(p, d, hidden, xb, yb, hb)
        mlp_backward(p, d, hidden, xb, hb, yb, tb, g, loss)
        mlp_adam(p, g, m, v, step, lr)
        if step % 500 == 0 or step == steps:
            hist.append((step, float(loss.item())))
    # fold the standardisation into the first layer: W1' = W1 / sd, b1' = b1 - W1' mu
    ph = p.cpu().numpy().astype(np.float64)
    W1 = ph[:hidden * d].reshape(hidden, d) / sd
    b1 = ph[hidden * d:hidden * d + hidden] - W1 @ mu
    raw = np.concatenate([W1.ravel(), b1, ph[hidden * d + hidden:]])
    return raw.astype(np.float32), hist


def predict(params, X, hidden, device="cuda"):
    dev = torch.device(device)
    X = np.asarray(X, dtype=np.float32)
    d = X.shape[1]
    pd = torch.from_numpy(np.asarray(params, dtype=np.float32)).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    y = torch.empty(X.shape[0], dtype=torch.float32, device=dev)
    mlp_forward(pd, d, hidden, Xd, y)
    return y.cpu().numpy().astype(np.float64)


def choose_log10_tau(X, y, eps, q=0.9):
    """tau: the q-quantile of the errors the threshold rule accepts (iterates whose
    relative changes are all below eps)."""
    X = np.asarray(X)
    y = np.asarray(y)
    N = X.shape[1] - 2
    ok = np.all(X[:, :N] < math.log10(eps), axis=1)
    pool = y[ok] if ok.sum() >= 10 else y
    return float(np.quantile(pool, q))


def time_to_fit(recs, ms, target):
    t = 0.0
    for r, m in zip(recs, ms):
        t += m
        if r["fit_est"] >= target:
            return t
    return None


def run_fixed(session, eps, max_sweeps):
    s = session
    s.reset()
    return run(s.plan, s.X, None, s.A, s.S, s.normX2, s.ws, s.rec, eps=eps, max_sweeps=max_sweeps)


def run_controlled(session, params, hidden, log10_tau, eps, rho_cap, check_period,
                   fallback_factor, max_sweeps):
    s = session
    s.reset()
    pd = torch.from_numpy(np.asarray(params, dtype=np.float32)).to(s.dev)
    set_controller(s.plan, pd, hidden=hidden, log10_tau=log10_tau, rho_cap=rho_cap,
                   check_period=check_period, fallback_factor=fallback_factor)
    try:
        return run(s.plan, s.X, None, s.A, s.S, s.normX2, s.ws, s.rec, eps=eps,
                   max_sweeps=max_sweeps)
    finally:
        set_controller(s.plan, None)


def constant_params(d, hidden, value=-1e30):
    """Parameters of a network whose output is `value` for every input: the controller
    then never leaves on its prediction, only on rho_cap or after a failed periodic check
    (the ablation that removes the network and keeps the rest of the controller)."""
    p = np.zeros(mlp_n_params(d, hidden), dtype=np.float32)
    p[-1] = value
    return p


def compare(fixed, ctrl, target, capped=None):
    recs0, ms0 = fixed
    recs1, ms1 = ctrl
    kinds0 = [r["kind"] for r in recs0]
    kinds1 = [r["kind"] for r in recs1]
    out = {
        "t_fixed_ms": time_to_fit(recs0, ms0, target), "t_ctrl_ms": time_to_fit(recs1, ms1, target),
        "builds_fixed": kinds0.count("pp_init"), "builds_ctrl": kinds1.count("pp_init"),
        "pp_fixed": sum(k != "als" for k in kinds0), "pp_ctrl": sum(k != "als" for k in kinds1),
        "fallback": int(any(r["ctrl_fallback"] for r in recs1)),
        "fit_fixed": recs0[-1]["fit_est"], "fit_ctrl": recs1[-1]["fit_est"],
    }
    if capped is not None:
        recs2, ms2 = capped
        kinds2 = [r["kind"] for r in recs2]
        out.update({"t_capped_ms": time_to_fit(recs2, ms2, target),
                    "builds_capped": kinds2.count("pp_init"),
                    "pp_capped": sum(k != "als" for k in kinds2),
                    "fallback_capped": int(any(r["ctrl_fallback"] for r in recs2)),
                    "fit_capped": recs2[-1]["fit_est"]})
    return out


def evaluate(session, params, hidden, log10_tau, eps, rho_cap, check_period, fallback_factor,
             max_sweeps, target, ablation=True):
    """Time to the target fit with the threshold rule, with the controller and (ablation)
    with the controller's rho_cap and periodic checks but a constant network."""
    fixed = run_fixed(session, eps, max_sweeps)
    ctrl = run_controlled(session, params, hidden, log10_tau, eps, rho_cap, check_period,
                          fallback_factor, max_sweeps)
    capped = None
    if ablation:
        d = len(session.shape) + 2
        capped = run_controlled(session, constant_params(d, hidden), hidden, log10_tau, eps,
                                rho_cap, check_period, fallback_factor, max_sweeps)
    return compare(fixed, ctrl, target, capped)


def search_log10_tau(sessions, params, hidden, candidates, eps, rho_cap, check_period,
                     fallback_factor, max_sweeps, target):
    """Pick tau on training problems: the candidate with the best geometric-mean
    speed-up in time to the target fit over the threshold rule (runs where either
    misses the target count as a ratio of the sweep budgets' times)."""
    fixed = [run_fixed(s, eps, max_sweeps) for s in sessions]
    best, table = None, []
    for lt in candidates:
        logs = []
        for s, f in zip(sessions, fixed):
            c = run_controlled(s, params, hidden, lt, eps, rho_cap, check_period, fallback_factor,
                               max_sweeps)
            t0 = time_to_fit(f[0], f[1], target) or sum(f[1])
            t1 = time_to_fit(c[0], c[1], target) or sum(c[1])
            logs.append(math.log(t0 / t1))
        g = math.exp(float(np.mean(logs)))
        table.append((float(lt), g))
        if best is None or g > best[1]:
            best = (float(lt), g)
    return best[0], table


def _ratio_stats(evals, num, den):
    """Speed-up t_num / t_den over the runs where both reached the target."""
    ratios = [e[num] / e[den] for e in evals if e.get(num) is not None and e.get(den) is not None]
    out = {
        "both_reached": len(ratios),
        "first_only": sum(e.get(num) is not None and e.get(den) is None for e in evals),
        "second_only": sum(e.get(num) is None and e.get(den) is not None for e in evals),
    }
    if ratios:
        q1, med, q3 = np.quantile(ratios, [0.25, 0.5, 0.75])
        out.update({"speedup_median": float(med), "speedup_q1": float(q1), "speedup_q3": float(q3),
                    "speedup_geomean": float(np.exp(np.mean(np.log(ratios))))})
    return out


def summarize(evals):
    """Controller against the threshold rule (as before: both_reached, fixed_only,
    ctrl_only, speed-ups); with the ablation arm also the capped controller against the
    threshold rule and the network's own share (capped time over controller time)."""
    r = _ratio_stats(evals, "t_fixed_ms", "t_ctrl_ms")
    out = {
        "runs": len(evals),
        "both_reached": r["both_reached"], "fixed_only": r["first_only"], "ctrl_only": r["second_only"],
        "fallback_fraction": float(np.mean([e["fallback"] for e in evals])) if evals else None,
    }
    out.update({k: v for k, v in r.items() if k.startswith("speedup")})
    if evals and "t_capped_ms" in evals[0]:
        out["capped_vs_fixed"] = _ratio_stats(evals, "t_fixed_ms", "t_capped_ms")
        out["network_vs_capped"] = _ratio_stats(evals, "t_capped_ms", "t_ctrl_ms")
        out["capped_fallback_fraction"] = float(np.mean([e["fallback_capped"] for e in evals]))
    return out


def experiment(order, train_seeds, val_seeds, eval_seeds, shape=None, eps=0.1, eps_gen=(0.05, 0.5),
               max_sweeps=100, hidden=64, steps=4000, target=0.99, check_period=10,
               fallback_factor=10.0, rho_cap_factor=3.0, progress_every=50, tau_search_runs=20):
    """Label generation, training, threshold choice and held-out evaluation for one
    order.  Returns a JSON-ready summary."""
    shape = SHAPES[order] if shape is None else tuple(shape)
    t_start = time.time()
    data = {}
    for split, seeds in (("train", train_seeds), ("val", val_seeds)):
        Xs, ys = [], []
        for k, sd in enumerate(seeds):
            rank, coll = problem_spec(order, sd)
            rng = np.random.default_rng(np.random.SeedSequence([int(sd), int(order), 11]))
            eg = float(rng.uniform(*eps_gen))
            sess = Session(shape, rank, sd, coll)
            f, l = collect(sess, eg, max_sweeps)
            Xs += f
            ys += l
            del sess
            if (k + 1) % progress_every == 0:
                log(f"order {order} {split}: {k + 1}/{len(seeds)} runs, {len(ys)} labels "
                    f"({time.time() - t_start:.0f} s)")
        data[split] = (np.array(Xs), np.array(ys))
    Xtr, ytr = data["train"]
    Xva, yva = data["val"]
    params, hist = train(Xtr, ytr, hidden=hidden, steps=steps)
    pva = predict(params, Xva, hidden)
    ptr = predict(params, Xtr, hidden)
    var = float(np.var(yva))
    mse_va = float(np.mean((pva - yva) ** 2))
    base_tau = choose_log10_tau(Xtr, ytr, eps)
    cands = sorted(set([round(base_tau, 3)] + [round(float(c), 3) for c in
                       np.quantile(ytr, [0.5, 0.75, 0.9, 0.97])] + [-3.5, -3.0, -2.5, -2.0]))
    search_sessions = []
    for sd in list(train_seeds)[:tau_search_runs]:
        rank, coll = problem_spec(order, sd)
        search_sessions.append(Session(shape, rank, sd, coll))
    log10_tau, tau_table = search_log10_tau(search_sessions, params, hidden, cands, eps,
                                            rho_cap_factor * eps, check_period, fallback_factor,
                                            max_sweeps, target)
    del search_sessions
    log(f"order {order}: {len(ytr)} train / {len(yva)} val labels, val MSE {mse_va:.4f} "
        f"(label variance {var:.4f}); tau search {tau_table} -> log10 tau {log10_tau:.3f}")
    evals = []
    for k, sd in enumerate(eval_seeds):
        rank, coll = problem_spec(order, sd)
        sess = Session(shape, rank, sd, coll)
        evals.append(evaluate(sess, params, hidden, log10_tau, eps, rho_cap_factor * eps,
                              check_period, fallback_factor, max_sweeps, target))
        del sess
        if (k + 1) % max(1, progress_every // 5) == 0:
            log(f"order {order} eval: {k + 1}/{len(eval_seeds)} runs ({time.time() - t_start:.0f} s)")
    return {
        "order": order, "shape": list(shape),
        "labels": {"train": int(len(ytr)), "val": int(len(yva))},
        "train_mse": float(np.mean((ptr - ytr) ** 2)), "val_mse": mse_va, "val_label_var": var,
        "val_r2": 1.0 - mse_va / var if var > 0 else None,
        "loss_history": hist, "log10_tau": log10_tau, "tau_search": tau_table,
        "eval": summarize(evals), "per_run": evals,
        "seconds": time.time() - t_start,
    }, params


def main():
    ap = argparse.ArgumentParser(description="learned PP controller: labels, training, gain")
    ap.add_argument("--orders", type=int, nargs="+", default=[3, 5])
    ap.add_argument("--train-runs", type=int, default=800)
    ap.add_argument("--val-runs", type=int, default=200)
    ap.add_argument("--eval-runs", type=int, default=50)
    ap.add_argument("--max-sweeps", type=int, default=100)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--size", type=int, default=None, help="override the mode size")
    ap.add_argument("--save", default=None, help="write the trained parameters (.npz)")
    args = ap.parse_args()
    results = {}
    saved = {}
    if args.train_runs + args.val_runs > 2000:
        raise SystemExit("training and validation seeds must stay below the held-out seeds (2000+)")
    for order in args.orders:
        # seeds 0..1999 train/validate, 2000.. are held out; a problem depends on (seed,
        # order), so the orders share the seed ranges without sharing problems
        tr = list(range(0, args.train_runs))
        va = list(range(args.train_runs, args.train_runs + args.val_runs))
        ev = list(range(2000, 2000 + args.eval_runs))
        shape = None if args.size is None else (args.size,) * order
        res, params = experiment(order, tr, va, ev, shape=shape, max_sweeps=args.max_sweeps,
                                 steps=args.steps)
        res.pop("per_run")
        results[str(order)] = res
        saved[f"order{order}"] = params
        print(json.dumps({"order": order, **res}), flush=True)
    if args.save:
        np.savez(args.save, **saved)


if __name__ == "__main__":
    main()
