"""GPU parity of the individual kernels against the float64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import tensorgen
from oracle import bf16 as obf16
from oracle import cp as ocp
from oracle import linalg as olinalg

from gpu_util import U32, U64, assert_within, dev, fp32_round, level1_reference, to_dev

pytestmark = pytest.mark.gpu

pp = pytest.importorskip("paper_1811_10573_amd")


def test_library_is_the_native_one():
    from paper_1811_10573_amd import _lib
    lib = _lib.load()
    assert lib._name.endswith("libppals.so")


def test_cast_bf16_bit_exact():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(100003).astype(np.float32)
    bits = x.view(np.uint32)
    bits[:1000] = (bits[:1000] & 0xFFFF0000) | 0x8000       # exact ties
    bits[1000:1010] = np.array([0x7F800000, 0xFF800000, 0x7FC00000, 0x00000001, 0x807FFFFF,
                                0x7F7FFFFF, 0x3F808000, 0x3F818000, 0x00008000, 0x80018000],
                               dtype=np.uint32)
    X = torch.from_numpy(x).to(dev())
    out = torch.empty(x.size, dtype=torch.int16, device=dev())
    pp.cast_bf16(X, out)
    got = out.cpu().numpy().view(np.uint16)
    want = obf16.round_bits(x)
    assert np.array_equal(got, want), np.flatnonzero(got != want)[:10]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 255, 1000003])
def test_tensor_norm2(dt, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    if dt == torch.float32:
        x = fp32_round(x)
    out = torch.zeros(1, dtype=torch.float64, device=dev())
    pp.tensor_norm2(torch.from_numpy(x).to(dev(), dtype=dt), out)
    want = float(np.dot(x, x))
    assert abs(out.item() - want) <= 2 * n * U64 * want + 1e-300


L1_CASES = [
    ((37, 29, 41), 5), ((64, 48, 80), 50), ((130, 33, 67), 17), ((19, 23, 9), 1),
    ((40, 36, 44), 64), ((24, 18, 20), 65), ((21, 13, 17), 128), ((1, 7, 5), 3),
    # FP32 with 1..4 columns in the last 16-column block (the 4x4x1 tail path), three
    # blocks: odd extents (scalar loads) and 16-byte-aligned extents (vector loads)
    ((29, 31, 27), 35), ((32, 40, 48), 34),
]


@pytest.mark.parametrize("tier", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims,R", L1_CASES)
def test_level1_single_mode(tier, dims, R):
    rng = np.random.default_rng(sum(dims) * R)
    X = rng.standard_normal(dims)
    if tier != "f64":
        X = fp32_round(X)
    A = [rng.standard_normal((s, R)) for s in dims]
    plan = pp.Plan(dims, R, "f64" if tier == "f64" else "f32", tier)
    Xd = to_dev(X, plan.torch_dtype)
    Xb = None
    if tier == "bf16":
        Xb = torch.empty(Xd.numel(), dtype=torch.int16, device=dev())
        pp.cast_bf16(Xd, Xb)
    Ad = [to_dev(a) for a in A]
    ws = plan.workspace(dev())
    u = U64 if tier == "f64" else U32
    for w in range(3):
        keep = [m for m in range(3) if m != w]
        out = torch.empty([dims[m] for m in keep] + [R], dtype=plan.torch_dtype, device=dev())
        pp.level1(plan, Xd, Xb, Ad, [w], out, ws)
        want, base = level1_reference(X, A, [w], tier)
        K = dims[w]
        assert_within(out.cpu().numpy(), want, (K + 1) * u * base, f"{tier} level1 w={w} {dims} R={R}")


@pytest.mark.parametrize("tier", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims,R,blocks", [
    ((12, 10, 14, 9), 7, [[0], [1], [2], [3], [0, 1], [2, 3]]),
    ((9, 8, 10, 11), 20, [[2, 3], [0, 1], [1, 2]]),
    ((6, 5, 4, 7, 3), 6, [[3, 4], [0, 1, 2], [0], [4]]),
])
def test_level1_blocks(tier, dims, R, blocks):
    rng = np.random.default_rng(R)
    X = rng.standard_normal(dims)
    if tier != "f64":
        X = fp32_round(X)
    A = [rng.standard_normal((s, R)) for s in dims]
    plan = pp.Plan(dims, R, "f64" if tier == "f64" else "f32", tier)
    Xd = to_dev(X, plan.torch_dtype)
    Xb = None
    if tier == "bf16":
        Xb = torch.empty(Xd.numel(), dtype=torch.int16, device=dev())
        pp.cast_bf16(Xd, Xb)
    Ad = [to_dev(a) for a in A]
    ws = plan.workspace(dev())
    u = U64 if tier == "f64" else U32
    for blk in blocks:
        keep = [m for m in range(len(dims)) if m not in blk]
        out = torch.empty([dims[m] for m in keep] + [R], dtype=plan.torch_dtype, device=dev())
        try:
            pp.level1(plan, Xd, Xb, Ad, blk, out, ws)
        except pp.PPALSError as e:
            if e.status == -2:   # operand larger than the plan's buffer
                continue
            raise
        want, base = level1_reference(X, A, blk, tier)
        K = int(np.prod([dims[m] for m in blk]))
        assert_within(out.cpu().numpy(), want, (K + 1) * u * base, f"{tier} level1 {blk} {dims}")


@pytest.mark.parametrize("tier", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims,R,blocks", [
    ((8, 700, 8), 50, [[1]]),                         # long contraction, few rows: split over k
    ((24, 40, 40, 24), 64, [[2, 3], [0, 1], [1, 2]]),  # combined two-mode contractions
    ((20, 30, 30, 20), 48, [[2, 3], [0, 1]]),
])
def test_level1_split_k(tier, dims, R, blocks):
    """Contractions long enough for the k range to be split over workgroups."""
    test_level1_blocks(tier, dims, R, blocks)


@pytest.mark.parametrize("tier", ["f64", "f32"])
@pytest.mark.parametrize("dims,R", [((33, 27, 45), 9), ((10, 12, 9, 11), 16), ((5, 6, 4, 5, 6), 5),
                                    ((64, 64, 64), 10), ((3, 2, 3, 2, 2, 3), 4)])
def test_mttkrp_all_modes(tier, dims, R):
    rng = np.random.default_rng(len(dims) * 100 + R)
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((s, R)) for s in dims]
    if tier == "f32":
        X = fp32_round(X)
        A = [fp32_round(a) for a in A]
    plan = pp.Plan(dims, R, tier)
    Xd = to_dev(X, plan.torch_dtype)
    Ad = [to_dev(a) for a in A]
    ws = plan.workspace(dev())
    u = U64 if tier == "f64" else U32
    total_k = int(np.prod(dims))
    for n in range(len(dims)):
        out = torch.empty(dims[n] * R, dtype=torch.float64, device=dev())
        pp.mttkrp(plan, Xd, None, Ad, n, out, ws)
        want = ocp.mttkrp(X, A, n)
        base = ocp.mttkrp(np.abs(X), [np.abs(a) for a in A], n)
        K = total_k // dims[n]
        assert_within(out.cpu().numpy().reshape(dims[n], R), want, (K + 2) * u * base,
                      f"{tier} mttkrp mode {n} {dims}")


@pytest.mark.parametrize("R", [1, 7, 16, 50, 64, 65, 100, 128])
@pytest.mark.parametrize("rows", [1, 5, 97])
@pytest.mark.parametrize("mdt", [torch.float64, torch.float32])
def test_gram_solve(R, rows, mdt):
    rng = np.random.default_rng(R * 1000 + rows)
    B = rng.standard_normal((R + 20, R))
    gamma = B.T @ B + 0.1 * np.eye(R)
    M = rng.standard_normal((rows, R))
    if mdt == torch.float32:
        M = fp32_round(M)
    A_old = rng.standard_normal((rows, R))
    want, st = olinalg.solve_normal(gamma, M)
    assert st == 0
    cond = np.linalg.cond(gamma)
    Ad = to_dev(A_old)
    g = torch.zeros(1, dtype=torch.float64, device=dev())
    s = torch.zeros(1, dtype=torch.int32, device=dev())
    ws = torch.empty(pp.gram_solve_workspace_bytes(R, rows), dtype=torch.uint8, device=dev())
    pp.gram_solve(R, rows, to_dev(gamma), to_dev(M, mdt), Ad, g, s, ws)
    got = Ad.cpu().numpy().reshape(rows, R)
    scale = np.abs(want).max() + 1e-300
    assert np.abs(got - want).max() <= 50 * R * U64 * cond * scale
    grad = np.linalg.norm((A_old - want) @ gamma)
    assert abs(g.item() - grad) <= 1e-9 * max(1.0, grad) * max(1.0, cond * 1e-6)
    assert s.item() == 0


def test_gram_solve_singular_uses_the_diagonal_shift():
    rng = np.random.default_rng(3)
    R, rows = 6, 9
    B = rng.standard_normal((30, R))
    B[:, 2] = 0.0
    gamma = B.T @ B
    M = rng.standard_normal((rows, R))
    M[:, 2] = 0.0
    want, st = olinalg.solve_normal(gamma, M)
    assert st == 1
    Ad = to_dev(np.zeros((rows, R)))
    g = torch.zeros(1, dtype=torch.float64, device=dev())
    s = torch.zeros(1, dtype=torch.int32, device=dev())
    ws = torch.empty(pp.gram_solve_workspace_bytes(R, rows), dtype=torch.uint8, device=dev())
    pp.gram_solve(R, rows, to_dev(gamma), to_dev(M), Ad, g, s, ws)
    # outcome 1 (shifted), no non-finite value, first failed pivot at the zero column
    assert s.item() & 3 == 1 and not s.item() & 16
    assert (s.item() >> 8) - 1 == olinalg.first_failed_pivot(gamma) == 2
    got = Ad.cpu().numpy().reshape(rows, R)
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got @ gamma, M, atol=1e-6 * np.abs(M).max())


@pytest.mark.parametrize("dims,R,dt", [((20, 17, 23), 5, "f64"), ((9, 8, 7, 6), 70, "f64"),
                                       ((30, 31, 29), 12, "f32"), ((64, 10, 300), 3, "f64")])
def test_exact_residual(dims, R, dt):
    p = tensorgen.make_problem(dims, R, seed=1, eta=0.05)
    X = p.X if dt == "f64" else fp32_round(p.X)
    A = [a * 0.9 for a in p.planted]
    plan = pp.Plan(dims, R, dt)
    out = torch.zeros(1, dtype=torch.float64, device=dev())
    pp.exact_residual2(plan, to_dev(X, plan.torch_dtype), [to_dev(a) for a in A], out,
                       plan.workspace(dev()))
    want = float(np.sum((X - ocp.cp_full(A)) ** 2))
    assert abs(out.item() - want) <= 1e-10 * want


def test_gram_solve_flags_non_finite_results():
    """A right-hand side with a NaN: the factorisation is clean (no pivot), and bit 4 of
    the status word reports the non-finite factor."""
    rng = np.random.default_rng(5)
    R, rows = 7, 11
    B = rng.standard_normal((30, R))
    gamma = B.T @ B
    M = rng.standard_normal((rows, R))
    M[4, 2] = np.nan
    Ad = to_dev(np.zeros((rows, R)))
    g = torch.zeros(1, dtype=torch.float64, device=dev())
    s = torch.zeros(1, dtype=torch.int32, device=dev())
    ws = torch.empty(pp.gram_solve_workspace_bytes(R, rows), dtype=torch.uint8, device=dev())
    pp.gram_solve(R, rows, to_dev(gamma), to_dev(M), Ad, g, s, ws)
    assert s.item() == 16
    got = Ad.cpu().numpy().reshape(rows, R)
    assert np.isnan(got[4]).any() and np.all(np.isfinite(np.delete(got, 4, axis=0)))


@pytest.mark.parametrize("dims,R", [((20, 18, 16), 5), ((80, 75, 72), 70)])
def test_sweep_record_reports_the_failed_pivot(dims, R):
    """Factors 1 and 2 start with column 3 zero, so every Gamma of the first ALS sweep has
    a zero row and column 3: the record names pivot 3 (the oracle's first failed pivot)
    with outcome 1 (diagonal shift) in every mode, on the fused tail (R = 5) and on the
    general-rank tail (R = 70), and flags no non-finite value."""
    prob = tensorgen.make_problem(dims, R, seed=3, eta=1e-2)
    init = [a.copy() for a in prob.init]
    init[1][:, 3] = 0.0
    init[2][:, 3] = 0.0
    plan = pp.Plan(dims, R, "f64")
    X = to_dev(prob.X)
    A = [to_dev(a) for a in init]
    S = to_dev(np.stack([a.T @ a for a in init]).reshape(-1))
    ws = plan.workspace(dev())
    rec = pp.new_record(dev())
    nrm = torch.zeros(1, dtype=torch.float64, device=dev())
    pp.tensor_norm2(X, nrm)
    pp.cp_als_sweep(plan, X, None, A, S, float(nrm.item()), ws, rec)
    got = pp.read_record(rec)
    Ao = [a.copy() for a in init]
    So = [a.T @ a for a in Ao]
    ref = ocp.als_sweep(prob.X, [a.copy() for a in init], [s.copy() for s in So])
    Aw = [a.copy() for a in init]
    Sw = [a.T @ a for a in Aw]
    for n in range(3):
        gamma = ocp.hadamard_except(Sw, n)
        want = olinalg.first_failed_pivot(gamma)
        ocp.als_update(Aw, Sw, n, ocp.mttkrp(prob.X, Aw, n))
        assert want == 3
        assert got["chol_pivot"][n] == want, (n, got["chol_pivot"])
        assert got["chol_status"][n] == ref.chol_status[n] == 1
        assert got["nonfinite"][n] == 0
