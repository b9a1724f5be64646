"""Pins for the bf16 emulation and the seeded generators."""
import numpy as np

import tensorgen
from oracle import bf16, cp


def test_bf16_known_values_and_ties_to_even():
    one = np.float32(1.0)
    ulp = 2.0 ** -7                       # bf16 spacing at 1.0
    x = np.array([1.0, 1.0 + ulp / 2, 1.0 + 3 * ulp / 2, 1.0 + ulp / 2 + 2.0 ** -20,
                  -2.5, 65504.0, 3.0e38, 1e-40], dtype=np.float64)
    r = bf16.round_to_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even (mantissa LSB 0)
    assert r[2] == 1.0 + 2 * ulp          # tie -> even (rounds up)
    assert r[3] == 1.0 + ulp              # above the tie -> up
    assert r[4] == -2.5
    assert r[5] == 65536.0                # 65504 is closer to 65536 than to 65280
    assert np.isfinite(r[6])
    assert bf16.round_bits(np.array([1.0], dtype=np.float32))[0] == 0x3F80
    assert bf16.round_bits(np.array([np.nan], dtype=np.float32))[0] == 0x7FC0
    del one


def test_bf16_relative_error_bound():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(100000).astype(np.float32).astype(np.float64)
    r = bf16.round_to_bf16(x)
    rel = np.abs(r - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -8 + 1e-12     # half a bf16 ulp (8 significant bits)
    # rms relative rounding error of uniform mantissas is about 2^-9 / sqrt(3)
    assert 0.5 * 2 ** -9 / np.sqrt(3) < np.sqrt(np.mean(rel ** 2)) < 2.5 * 2 ** -9 / np.sqrt(3)


def test_noise_ratio_exact():
    p = tensorgen.make_problem((10, 12, 14), 3, seed=0, eta=1e-3)
    T = tensorgen.cp_reconstruct(p.planted)
    assert abs(np.linalg.norm(p.X - T) / np.linalg.norm(T) - 1e-3) < 1e-12


def test_collinearity_realised():
    rng = np.random.default_rng(1)
    for C in (0.2, 0.5, 0.9):
        A = tensorgen.planted_factors((4000,), 6, rng, collinearity=C)[0]
        cos = A.T @ A
        off = cos[~np.eye(6, dtype=bool)]
        assert np.all(np.abs(np.diag(cos) - 1) < 1e-12)
        assert abs(off.mean() - C) < 0.05


def test_seeds_are_reproducible_and_independent():
    a = tensorgen.make_problem((5, 6, 7), 2, seed=3)
    b = tensorgen.make_problem((5, 6, 7), 2, seed=3)
    c = tensorgen.make_problem((5, 6, 7), 2, seed=4)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.init[0], b.init[0])
    assert not np.array_equal(a.X, c.X)
    assert all(0 <= x.min() and x.max() < 1 for x in a.init)


def test_generator_reconstruction_matches_oracle_model():
    rng = np.random.default_rng(5)
    A = [rng.standard_normal((s, 3)) for s in (3, 4, 5, 2)]
    np.testing.assert_allclose(tensorgen.cp_reconstruct(A), cp.cp_full(A), rtol=1e-13, atol=1e-13)
