"""Helpers shared by the GPU tests: device transfer, error bounds, oracle variants.

Tolerances are derived from the arithmetic (Higham's bound for a sum of K
products accumulated in precision u: |err| <= gamma_K * sum |x_i b_i| with
gamma_K ~ K u).  Each test feeds both sides identical inputs; when a tier rounds
its inputs (FP32 factors, bf16 operands) the oracle applies the same rounding
to its float64 copies, so only accumulation order and precision differ.
"""
import numpy as np
import torch

from oracle import bf16 as obf16
from oracle import cp as ocp

U64 = 2.0 ** -53
U32 = 2.0 ** -24

DEV = "cuda:0"


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    return torch.device(DEV)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def fp32_round(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def assert_within(got, want, bound, what, slack=2.0):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    err = np.abs(got - want)
    lim = slack * np.asarray(bound) + 1e-300
    bad = err > lim
    if bad.any():
        i = np.argmax(err - lim)
        raise AssertionError(
            f"{what}: {bad.sum()} of {err.size} entries outside the bound; worst flat index {i}: "
            f"got {got.flat[i]!r} want {want.flat[i]!r} err {err.flat[i]:.3e} bound {lim.flat[i]:.3e}")


def level1_reference(X, A, contract, tier):
    """Oracle first-level contraction with the tier's input rounding.

    Returns (value, bound_base): value in float64, bound_base = the same contraction
    of |X| and |B| (used to scale the accumulation error bound)."""
    N = X.ndim
    keep = [m for m in range(N) if m not in contract]
    Af = [np.asarray(a, dtype=np.float64) for a in A]
    if tier == "f64":
        Xr, Ar = X, Af
    elif tier == "f32":
        Xr = fp32_round(X)
        Ar = [a.copy() for a in Af]
        if len(contract) == 1:
            Ar[contract[0]] = fp32_round(Af[contract[0]])
    else:  # bf16: X and the (Khatri-Rao) operand rounded float64 -> float32 -> bf16
        Xr = obf16.round_to_bf16(fp32_round(X))
        Ar = [a.copy() for a in Af]
        if len(contract) == 1:
            Ar[contract[0]] = obf16.round_to_bf16(Af[contract[0]])
    if len(contract) > 1 and tier != "f64":
        # the operand is the Khatri-Rao product, rounded once after an FP64 product
        mats = [Af[m] for m in contract]
        krp = ocp.khatri_rao(mats)
        krp = fp32_round(krp) if tier == "f32" else obf16.round_to_bf16(krp)
        shp = [X.shape[m] for m in contract]
        lo = contract[0]
        xm = Xr.reshape(int(np.prod(X.shape[:lo])), int(np.prod(shp)), -1)
        val = np.einsum("pkq,kr->pqr", xm, krp)
        base = np.einsum("pkq,kr->pqr", np.abs(xm), np.abs(krp))
        return val.reshape([X.shape[m] for m in keep] + [-1]), base.reshape([X.shape[m] for m in keep] + [-1])
    val = ocp.partial_mttkrp(Xr, Ar, keep)
    base = ocp.partial_mttkrp(np.abs(Xr), [np.abs(a) for a in Ar], keep)
    return val, base
