"""gram_solve_noalloc: the normal-equation solve with the library's fixed scratch array
instead of a caller workspace.  Checked against gram_solve (same kernels, so the same
bits) and against the float64 oracle, on consecutive calls of decreasing size (the
array keeps the previous call's contents), plus the host-side size limit."""
import numpy as np
import pytest
import torch

from oracle import linalg as olinalg

from gpu_util import U64, dev, fp32_round, to_dev

pytestmark = pytest.mark.gpu

pp = pytest.importorskip("paper_1811_10573_amd")


def _case(R, rows, seed, singular=False):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((R + 20, R))
    if singular:
        B[:, 1] = 0.0
    gamma = B.T @ B + (0.0 if singular else 0.1) * np.eye(R)
    M = rng.standard_normal((rows, R))
    if singular:
        M[:, 1] = 0.0
    A_old = rng.standard_normal((rows, R))
    return gamma, M, A_old


def _solve(fn, R, rows, gamma, M, A_old, mdt, ws=None):
    A = to_dev(A_old)
    g = torch.full((1,), -1.0, dtype=torch.float64, device=dev())
    s = torch.full((1,), -7, dtype=torch.int32, device=dev())
    args = (R, rows, to_dev(gamma), to_dev(M, mdt), A, g, s)
    if ws is None:
        fn(*args)
    else:
        fn(*args, ws)
    torch.cuda.synchronize()
    return A.cpu().numpy().reshape(rows, R), g.item(), s.item()


@pytest.mark.parametrize("mdt", [torch.float64, torch.float32])
def test_noalloc_matches_gram_solve_on_consecutive_calls(mdt):
    """Two calls in a row, the second smaller (fewer rows and a lower rank), then a
    singular Gamma that takes the diagonal shift: every output equals gram_solve's bit
    for bit and the oracle's within the conditioning bound."""
    for R, rows, seed, singular in [(128, 5000, 1, False), (50, 800, 2, False), (6, 9, 3, True)]:
        gamma, M, A_old = _case(R, rows, seed, singular)
        if mdt == torch.float32:
            M = fp32_round(M)
        got, g, st = _solve(pp.gram_solve_noalloc, R, rows, gamma, M, A_old, mdt)
        ws = torch.empty(pp.gram_solve_workspace_bytes(R, rows), dtype=torch.uint8, device=dev())
        ref, g_ref, st_ref = _solve(pp.gram_solve, R, rows, gamma, M, A_old, mdt, ws)
        assert np.array_equal(got, ref), (R, rows)
        assert g == g_ref and st == st_ref, (R, rows, g, g_ref, st, st_ref)
        want, st_or = olinalg.solve_normal(gamma, M)
        # status word: outcome in bits 0-1, first failed pivot plus one from bit 8
        assert st & 3 == st_or and (st >> 8) - 1 == olinalg.first_failed_pivot(gamma)
        if not singular:
            cond = np.linalg.cond(gamma)
            assert np.abs(got - want).max() <= 50 * R * U64 * cond * (np.abs(want).max() + 1e-300)
            grad = np.linalg.norm((A_old - want) @ gamma)
            assert abs(g - grad) <= 1e-9 * max(1.0, grad) * max(1.0, cond * 1e-6)
        else:
            assert np.all(np.isfinite(got))
            np.testing.assert_allclose(got @ gamma, M, atol=1e-6 * np.abs(M).max())


def test_noalloc_rejects_rows_above_the_limit():
    """More rows than the fixed scratch holds: refused on the host, nothing enqueued, and
    the output buffers keep their contents."""
    R, rows = 4, pp.GRAM_SOLVE_NOALLOC_MAX_ROWS + 1
    gamma = to_dev(np.eye(R))
    M = torch.zeros(rows * R, dtype=torch.float64, device=dev())
    A = torch.ones(rows * R, dtype=torch.float64, device=dev())
    g = torch.full((1,), -1.0, dtype=torch.float64, device=dev())
    s = torch.full((1,), -7, dtype=torch.int32, device=dev())
    with pytest.raises(pp.PPALSError, match="scratch limit"):
        pp.gram_solve_noalloc(R, rows, gamma, M, A, g, s)
    torch.cuda.synchronize()
    assert g.item() == -1.0 and s.item() == -7
    assert bool(torch.all(A == 1.0))
