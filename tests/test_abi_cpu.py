"""Host-side checks of the C ABI (no GPU): the shared library loads and exports
every entry point declared in include/ppals.h, argument validation returns the
documented status codes without touching a device, and the host plans follow
the dimension-tree schedules and cost formulas of Sections 2.5 and 3.2.3."""
import ctypes
import os
import re

import pytest

from oracle import tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppals.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1811_10573_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1811_10573_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "typedef")))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    from paper_1811_10573_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def _desc(dims, rank, tdt=0, l1=0, so=1):
    from paper_1811_10573_amd import _lib
    d = _lib.Desc()
    d.order = len(dims)
    d.rank = rank
    for i, s in enumerate(dims):
        d.dims[i] = s
    d.tensor_dtype, d.level1_dtype, d.use_second_order = tdt, l1, so
    return d


def _create(lib, *a, **k):
    h = ctypes.c_void_p()
    st = lib.ppals_plan_create(ctypes.byref(_desc(*a, **k)), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("dims,rank,tdt,l1,want", [
    ((5, 6), 3, 0, 0, -2),               # order 2
    ((2,) * 9, 3, 0, 0, -2),             # order 9 (dims beyond 8 are not even representable)
    ((5, 6, 7), 0, 0, 0, -2),
    ((5, 6, 7), 129, 0, 0, -2),
    ((5, 0, 7), 3, 0, 0, -1),
    ((5, 6, 7), 3, 0, 1, -2),            # FP64 tensor with FP32 first level
    ((5, 6, 7), 3, 0, 2, -2),            # FP64 tensor with BF16 first level
    ((5, 6, 7), 3, 1, 0, -2),
])
def test_plan_argument_errors(lib, dims, rank, tdt, l1, want):
    if len(dims) > 8:
        d = _desc(dims[:8], rank, tdt, l1)
        d.order = 9
        h = ctypes.c_void_p()
        st = lib.ppals_plan_create(ctypes.byref(d), ctypes.byref(h))
    else:
        st, h = _create(lib, dims, rank, tdt, l1)
    assert st == want
    assert not h.value
    assert len(lib.ppals_last_error()) > 0


@pytest.mark.parametrize("step,want", [(0.0, 0), (0.7, 0), (1.0, 0), (1.5, -1), (-0.2, -1),
                                       (float("nan"), -1)])
def test_plan_step_size_range(lib, step, want):
    """The update step size of the step-size variant must lie in (0, 1]; 0 reads as 1."""
    d = _desc((5, 6, 7), 3, 0, 0)
    d.step_size = step
    h = ctypes.c_void_p()
    st = lib.ppals_plan_create(ctypes.byref(d), ctypes.byref(h))
    assert st == want
    if h.value:
        lib.ppals_plan_destroy(h)
    assert bool(h.value) == (want == 0)


def test_null_arguments_fail_before_any_device_work(lib):
    st, h = _create(lib, (6, 7, 8), 4)
    assert st == 0
    try:
        nul = ctypes.c_void_p()
        arr = (ctypes.c_void_p * 3)(1, 2, 3)
        assert lib.cp_als_sweep(h, nul, nul, arr, nul, 1.0, nul, nul, nul) == -1
        assert lib.cp_als_sweep(h, ctypes.c_void_p(8), nul, arr, ctypes.c_void_p(8), 1.0, nul,
                                ctypes.c_void_p(8), nul) == -4
        assert lib.pp_sweep(h, arr, ctypes.c_void_p(8), 1.0, ctypes.c_void_p(8),
                            ctypes.c_void_p(8), nul) == -4     # workspace not 256-byte aligned
        assert lib.pp_sweep(h, arr, ctypes.c_void_p(8), 1.0, ctypes.c_void_p(4096),
                            ctypes.c_void_p(8), nul) == -5     # no operators built
        assert lib.pp_build_operators(h, nul, nul, arr, ctypes.c_void_p(8), nul) == -1
        assert lib.gram_solve(0, 5, nul, nul, 0, nul, nul, nul, nul, nul) == -2
        assert lib.gram_solve(4, 5, nul, nul, 0, nul, nul, nul, nul, nul) == -1
        assert lib.ppals_tensor_norm2(nul, 0, 10, nul, nul, nul) == -1
        assert lib.ppals_cast_bf16(nul, nul, 10, nul) == -1
        assert lib.ppals_cast_bf16(ctypes.c_void_p(8), ctypes.c_void_p(8), 0, nul) == 0
        ws = ctypes.c_void_p(4096)
        assert lib.ppals_mttkrp(h, ctypes.c_void_p(8), nul, arr, 7, ctypes.c_void_p(8),
                                ws, nul) == -1
        assert lib.ppals_level1(h, ctypes.c_void_p(8), nul, arr, 0b101, ctypes.c_void_p(8),
                                ws, nul) == -1  # not contiguous
        assert lib.ppals_level1(h, ctypes.c_void_p(8), nul, arr, 0b111, ctypes.c_void_p(8),
                                ws, nul) == -1  # all modes
        assert lib.ppals_get_operator(h, ws, 0, 1, ctypes.c_void_p(8), nul) == -5
        assert lib.ppals_get_operator(h, ws, 1, 0, ctypes.c_void_p(8), nul) == -1
    finally:
        lib.ppals_plan_destroy(h)


def test_bf16_tier_requires_bf16_copy(lib):
    st, h = _create(lib, (6, 7, 8), 4, 1, 2)
    assert st == 0
    try:
        arr = (ctypes.c_void_p * 3)(1, 2, 3)
        nul = ctypes.c_void_p()
        assert lib.pp_build_operators(h, ctypes.c_void_p(8), nul, arr, ctypes.c_void_p(8), nul) == -1
    finally:
        lib.ppals_plan_destroy(h)


def _describe(lib, dims, rank, tdt=0, l1=0):
    import json
    st, h = _create(lib, dims, rank, tdt, l1)
    assert st == 0
    buf = ctypes.create_string_buffer(1 << 20)
    assert lib.ppals_plan_describe(h, buf, len(buf)) == 0
    small = ctypes.create_string_buffer(8)
    assert lib.ppals_plan_describe(h, small, len(small)) == -1
    ws = lib.ppals_workspace_bytes(h)
    lib.ppals_plan_destroy(h)
    return json.loads(buf.value.decode()), ws


@pytest.mark.parametrize("N,s,R", [(3, 40, 5), (3, 800, 50), (4, 160, 64), (5, 40, 40), (6, 9, 3),
                                   (8, 3, 2)])
def test_plan_costs_match_the_paper(lib, N, s, R):
    d, ws = _describe(lib, (s,) * N, R)
    assert ws > 0
    # Section 2.5: all MTTKRPs of one sweep cost 4 s^N R to leading order (two first-level
    # contractions of 2 s^N R each)
    assert d["dt_level1_flops"] == 4 * s ** N * R
    assert d["dt_ttv_flops"] < d["dt_level1_flops"]
    # Section 3.2.3: operator build 2R sum_{l=2}^{N-1} C(l+1,2) s^(N-l+2)
    assert d["pp_build_level1_flops"] + d["pp_build_tree_ttv_flops"] == \
        tree.pp_build_flops_formula(s, N, R)
    assert d["pp_build_level1_flops"] == 6 * s ** N * R
    # Table 1, first-order part of the approximated step: N(N-1) operator contractions
    assert d["pp_approx_first_order_flops"] == 2 * N * (N - 1) * s * s * R


@pytest.mark.parametrize("dims", [(7, 5, 9), (4, 6, 5, 3), (3, 4, 2, 5, 3), (2, 3, 2, 2, 3, 2, 2)])
def test_dt_schedule_solves_every_mode_once_in_order(lib, dims):
    d, _ = _describe(lib, dims, 3)
    solves = [o["mode"] for o in d["dt_ops"] if o["op"] == "solve"]
    assert solves == list(range(len(dims)))
    # every TTV that feeds a solve keeps exactly that mode
    ops = d["dt_ops"]
    for a, b in zip(ops, ops[1:]):
        if b["op"] == "solve":
            assert a["op"] == "ttv" and a["kept"] == [b["mode"]]


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_pp_build_schedule_matches_oracle_tree(lib, N):
    d, _ = _describe(lib, (4,) * N, 2)
    ops = d["pp_build_ops"]
    nodes = tree.pp_tree(N)
    assert len(ops) == len(nodes)
    for o, (l, child, parent, w) in zip(ops, nodes):
        assert o["kept"] == [m - 1 for m in child]
        if l == 2:
            assert o["op"] == "level1" and o["contract"] == [w - 1, w]
        else:
            assert o["op"] == "ttv" and o["src"] == [m - 1 for m in parent]
            assert o["src"][o["contract_pos"][0]] == w - 1


@pytest.mark.parametrize("N", [3, 4, 5])
def test_pp_build_reuse_after_als(lib, N):
    # an ALS sweep of order 3 ends with X contracted with the final first factor, the build's
    # first-level step that keeps modes 2 and 3 (1-based); the trees of higher orders
    # contract two or more modes at their first level, which no build step does
    d, _ = _describe(lib, (5,) * N, 3)
    reused = d["pp_build_reused_after_als"]
    if N == 3:
        assert reused == [0, 1]
        dt_l1 = [o for o in d["dt_ops"] if o["op"] == "level1"]
        last = dt_l1[-1]
        assert last["contract"] == reused and last["kept"] == [1, 2]
        k = d["dt_ops"].index(last)
        assert {"op": "solve", "mode": 0} in d["dt_ops"][:k]
        assert any(o["op"] == "level1" and o["contract"] == reused and o["kept"] == [1, 2]
                   for o in d["pp_build_ops"])
    else:
        assert reused is None


def test_controller_entry_points_validate_arguments(lib):
    from paper_1811_10573_amd import _lib
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    E_ARG, E_UNS, E_STATE = _lib.PPALS_E_ARG, _lib.PPALS_E_UNSUPPORTED, _lib.PPALS_E_STATE
    assert lib.ppals_mlp_forward(None, 5, 64, fake, 4, fake, None, None) == E_ARG
    assert lib.ppals_mlp_forward(fake, 0, 64, fake, 4, fake, None, None) == E_UNS
    assert lib.ppals_mlp_forward(fake, 17, 64, fake, 4, fake, None, None) == E_UNS
    assert lib.ppals_mlp_forward(fake, 5, 1025, fake, 4, fake, None, None) == E_UNS
    assert lib.ppals_mlp_forward(fake, 5, 64, fake, -1, fake, None, None) == E_ARG
    assert lib.ppals_mlp_backward(fake, 5, 64, fake, None, fake, fake, 4, fake, None, None) == E_ARG
    assert lib.ppals_mlp_backward(fake, 5, 64, fake, fake, fake, fake, 0, fake, None, None) == E_ARG
    assert lib.ppals_mlp_adam(fake, fake, fake, fake, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == E_ARG
    assert lib.ppals_mlp_adam(fake, fake, fake, fake, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None) == E_ARG
    assert lib.ppals_mlp_adam(fake, None, fake, fake, 10, 1, 1e-3, 0.9, 0.999, 1e-8, None) == E_ARG
    st, h = _create(lib, [6, 5, 7], 3)
    assert st == 0
    try:
        ptrs = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)
        # no operators built yet
        assert lib.ppals_pp_rhs_error(h, fake, None, ptrs, fake, fake, fake, None) == E_STATE
        assert lib.ppals_pp_rhs_error(h, fake, None, ptrs, None, fake, fake, None) == E_ARG
        c = _lib.Controller(params=0x1000, hidden=64, check_period=5, log10_tau=-2.0, rho_cap=0.3,
                            fallback_factor=10.0)
        assert lib.ppals_set_controller(h, ctypes.byref(c)) == 0
        assert lib.ppals_set_controller(h, None) == 0
        bad = [dict(params=None), dict(hidden=0), dict(hidden=2048), dict(check_period=-1),
               dict(rho_cap=0.0), dict(fallback_factor=0.0)]
        for b in bad:
            kw = dict(params=0x1000, hidden=64, check_period=5, log10_tau=-2.0, rho_cap=0.3,
                      fallback_factor=10.0)
            kw.update(b)
            c = _lib.Controller(**kw)
            assert lib.ppals_set_controller(h, ctypes.byref(c)) != 0, b
    finally:
        lib.ppals_plan_destroy(h)


def test_batch_create_validates_and_describes(lib):
    import json
    from paper_1811_10573_amd import _lib
    h = ctypes.c_void_p()
    arr = (_lib.BatchProblem * 2)()
    arr[0].dims[:] = [10, 20, 30]
    arr[0].rank = 5
    arr[1].dims[:] = [40, 8, 9]
    arr[1].rank = 64
    assert lib.ppals_batch_create(arr, 0, 10, ctypes.byref(h)) == _lib.PPALS_E_ARG
    assert lib.ppals_batch_create(arr, 2, 0, ctypes.byref(h)) == _lib.PPALS_E_ARG
    assert lib.ppals_batch_create(None, 2, 10, ctypes.byref(h)) == _lib.PPALS_E_ARG
    arr[1].rank = 65
    assert lib.ppals_batch_create(arr, 2, 10, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    arr[1].rank = 64
    arr[1].dims[1] = 257
    assert lib.ppals_batch_create(arr, 2, 10, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    arr[1].dims[1] = 8
    assert lib.ppals_batch_create(arr, 2, 10, ctypes.byref(h)) == 0
    try:
        ws = lib.ppals_batch_workspace_bytes(h)
        # at least the three FP32 operators of every problem
        assert ws >= 4 * (10 * 20 + 10 * 30 + 20 * 30) * 5 + 4 * (40 * 8 + 40 * 9 + 8 * 9) * 64
        buf = ctypes.create_string_buffer(4096)
        assert lib.ppals_batch_describe(h, buf, 4096) == 0
        info = json.loads(buf.value.decode())
        assert info["count"] == 2 and info["max_rank"] == 64 and info["max_dim"] == 40
        assert not info["tuned"]
        # nothing bound yet: the device entry points refuse before touching a device
        fake = ctypes.c_void_p(0x1000)
        assert lib.ppals_batch_sweep(h, fake, None) == _lib.PPALS_E_STATE
        assert lib.ppals_batch_run(h, fake, 1, 1, None) == _lib.PPALS_E_STATE
        assert lib.ppals_batch_autotune(h, fake, 1, None) == _lib.PPALS_E_STATE
    finally:
        lib.ppals_batch_destroy(h)


def test_tucker_plan_validates_and_refuses_before_device_work(lib):
    """Tucker plan limits (1 <= R <= 64, R <= every s_n) and the entry points' host
    checks: null arguments, workspace alignment, PP sweeps or right-hand sides before an
    operator build, unknown kinds."""
    from paper_1811_10573_amd import _lib
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 3)(30, 20, 10)
    assert lib.tucker_plan_create(3, dims, 0, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    assert lib.tucker_plan_create(3, dims, 65, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    assert lib.tucker_plan_create(3, dims, 11, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    assert lib.tucker_plan_create(2, dims, 3, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    assert lib.tucker_plan_create(9, dims, 3, ctypes.byref(h)) == _lib.PPALS_E_UNSUPPORTED
    bad = (ctypes.c_int64 * 3)(30, 0, 10)
    assert lib.tucker_plan_create(3, bad, 3, ctypes.byref(h)) == _lib.PPALS_E_ARG
    assert lib.tucker_plan_create(3, dims, 10, ctypes.byref(h)) == 0
    try:
        R = 10
        ws_bytes = lib.tucker_workspace_bytes(h)
        # at least the three pairwise operators and the three Y_p^(n)
        assert ws_bytes >= 8 * ((30 * 20 + 30 * 10 + 20 * 10) * R + (30 + 20 + 10) * R * R)
        assert lib.tucker_set_solver(h, 0.0, 10, 10) == _lib.PPALS_E_ARG
        assert lib.tucker_set_solver(h, 1e-10, 0, 10) == _lib.PPALS_E_ARG
        assert lib.tucker_set_solver(h, 1e-12, 500, 5000) == 0
        fake = ctypes.c_void_p(0x1000)
        arr = (ctypes.c_void_p * 3)(0x2000, 0x3000, 0x4000)
        rec = _lib.TuckerRecord()
        nul = ctypes.c_void_p()
        assert lib.tucker_pp_sweep(h, fake, arr, fake, 1.0, 2, ctypes.byref(rec), nul) == _lib.PPALS_E_STATE
        assert lib.tucker_pp_rhs(h, fake, 0, fake, nul) == _lib.PPALS_E_STATE
        assert lib.tucker_pp_sweep(h, fake, arr, fake, 1.0, 0, ctypes.byref(rec), nul) == _lib.PPALS_E_ARG
        assert lib.tucker_pp_sweep(h, ctypes.c_void_p(0x1008), arr, fake, 1.0, 2, ctypes.byref(rec),
                                   nul) == _lib.PPALS_E_WORKSPACE
        assert lib.tucker_ttmc(h, fake, fake, arr, 3, fake, nul) == _lib.PPALS_E_ARG  # mode 3 of 3
        assert lib.tucker_als_sweep(h, fake, nul, arr, fake, 1.0, ctypes.byref(rec), nul) == _lib.PPALS_E_ARG
        assert lib.tucker_als_sweep(h, fake, fake, arr, fake, 0.0, ctypes.byref(rec), nul) == _lib.PPALS_E_ARG
        part = (ctypes.c_void_p * 3)(0x2000, None, 0x4000)
        assert lib.tucker_pp_build(h, fake, fake, part, nul) == _lib.PPALS_E_ARG
        n_out = ctypes.c_int32()
        assert lib.tucker_run(h, fake, fake, arr, fake, -1.0, 5, 0.0, None, 0, ctypes.byref(rec),
                              ctypes.byref(n_out), nul) == _lib.PPALS_E_ARG
    finally:
        lib.tucker_plan_destroy(h)


def test_direct_build_plan(lib):
    """The direct operator build keeps no tree intermediate, contracts each of the
    N(N-1)/2 operators from X (2 s^N R flops each), refuses the BF16 first level, and
    leaves order 3 as it is."""
    import json
    from paper_1811_10573_amd import _lib

    def describe(dims, R, tdt, l1, direct):
        d = _desc(dims, R, tdt, l1)
        d.pp_build_levels = direct
        h = ctypes.c_void_p()
        st = lib.ppals_plan_create(ctypes.byref(d), ctypes.byref(h))
        if st != 0:
            return st, None
        buf = ctypes.create_string_buffer(1 << 20)
        assert lib.ppals_plan_describe(h, buf, len(buf)) == 0
        lib.ppals_plan_destroy(h)
        return 0, json.loads(buf.value.decode())

    s, R = 20, 6
    st, tree = describe((s,) * 4, R, 0, 0, 0)
    st2, direct = describe((s,) * 4, R, 0, 0, 2)
    assert st == 0 and st2 == 0
    assert tree["pp_build"] == "tree" and direct["pp_build"] == "direct"
    assert tree["pp_build_intermediate_bytes"] == 3 * s ** 3 * R * 8
    assert direct["pp_build_intermediate_bytes"] == 0
    assert direct["workspace_bytes"] < tree["workspace_bytes"]
    l1 = [o for o in direct["pp_build_ops"] if o["op"] == "level1"]
    assert len(l1) == 6 and all(o["flops"] == 2 * s ** 4 * R for o in l1)
    assert sorted(tuple(o["kept"]) for o in l1) == [(i, j) for i in range(4) for j in range(i + 1, 4)]
    assert sum(1 for o in l1 if o["strided"]) == 3      # (0,2), (1,2), (1,3)
    assert direct["pp_build_tree_ttv_flops"] == 0
    st, _ = describe((s,) * 4, R, 1, 2, 2)
    assert st == _lib.PPALS_E_UNSUPPORTED
    st, o3 = describe((s,) * 3, R, 0, 0, 2)
    assert st == 0 and o3["pp_build"] == "tree"


@pytest.mark.parametrize("dims,R,tdt", [((128, 128, 3, 7200), 15, 1), ((1024, 1344, 33, 9), 50, 1),
                                        ((40, 30, 20, 50, 10), 12, 0), ((9, 14, 6, 11, 7, 5), 8, 0)])
def test_build_model_prices_the_scheduled_nodes(lib, dims, R, tdt):
    """The cost model behind the automatic choice of combined levels (Section 3.2.3)
    prices exactly the nodes the schedule builds: for every level count l, each
    contraction of X at the slower of its MFMA time (0.6 of the tier's peak, 0.45 when
    strided) and one read of X plus one write of the node (0.6 of 8 TB/s), and each tree
    contraction by its parent (elements = flops / 2) read and its node (the parent over
    the contracted extent) written at 0.55 of 8 TB/s.  Unequal mode sizes tell the parents
    apart: a parent priced with the wrong third mode misses by orders of magnitude."""
    import json
    from math import prod

    def describe(levels):
        d = _desc(dims, R, tdt, tdt)
        d.pp_build_levels = levels
        h = ctypes.c_void_p()
        assert lib.ppals_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
        buf = ctypes.create_string_buffer(1 << 20)
        assert lib.ppals_plan_describe(h, buf, len(buf)) == 0
        lib.ppals_plan_destroy(h)
        return json.loads(buf.value.decode())

    N = len(dims)
    peak, xsz = (78.6e12, 8.0) if tdt == 0 else (157.3e12, 4.0)
    model = describe(-1)["pp_build_model_ms"]
    assert len(model) == N - 2
    for l in range(1, N - 1):
        plan = describe(l)
        want = 0.0
        for o in plan["pp_build_ops"]:
            if o["op"] == "level1":
                eff = 0.45 if (l >= 2 and o["strided"]) else 0.6
                want += max(o["flops"] / (eff * peak),
                            (prod(dims) * xsz + o["M"] * R * xsz) / (0.6 * 8e12))
            elif o["op"] == "ttv" and o["out_mode"] == -1:
                parent = o["flops"] / 2
                want += (parent + parent / o["X"]) * xsz / (0.55 * 8e12)
        assert model[l - 1] == pytest.approx(want * 1e3, rel=2e-3), (l, model, want * 1e3)
