"""bfloat16 emulation for the BF16-input first-level contraction (test oracle).

The paper fixes no precision; the BF16 tier is a property of this library.
Reading: values are first held in float32, then rounded to bfloat16 with
round-to-nearest, ties-to-even, which is the rounding of the hardware convert.
"""
from __future__ import annotations

import numpy as np


def round_bits(x):
    """float32(x) rounded to bfloat16 (nearest-even), as uint16 bit patterns."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    keep = u >> 16
    rest = u & 0xFFFF
    # round half to even on the 16 discarded bits
    up = (rest > 0x8000) | ((rest == 0x8000) & ((keep & 1) == 1))
    out = (keep + up.astype(np.uint64)).astype(np.uint16)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = 0x7FC0
    return out


def from_bits(b):
    """uint16 bfloat16 patterns -> float64 values."""
    u = np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def round_to_bf16(x):
    """float64 values of bf16(float32(x))."""
    return from_bits(round_bits(x))
