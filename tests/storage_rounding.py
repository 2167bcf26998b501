"""Rounding of a population state to the library's storage formats (test
infrastructure; no lattice Boltzmann arithmetic).

The library stores the deviation h_i = f_i - w_i of every population from a
reference equilibrium w_i: FP32 keeps h, FP16 keeps h * 2^12, BF16 keeps h,
each rounded to nearest even. `round_state` applies exactly that rounding to
an FP64 state, so that an FP64 run whose state is rounded after every step
measures the error the storage format alone causes (the floor below which no
kernel with that storage can go, whatever precision it computes in).
"""
import numpy as np

SCALE = {"f32": 1.0, "f16": 4096.0, "bf16": 1.0}


def _to_f32_odd(x):
    """FP64 -> FP32 rounding to odd: a following round-to-nearest-even to a
    format with at least two fewer significand bits is then correctly rounded."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    inexact = f.astype(np.float64) != x
    bits = f.view(np.uint32).copy()
    even = (bits & 1) == 0
    fix = inexact & even & np.isfinite(x)
    away = np.abs(x) > np.abs(f.astype(np.float64))
    bits[fix & away] += 1
    bits[fix & ~away] -= 1
    return bits.view(np.float32)


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    b = _to_f32_odd(x).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_values(h, storage):
    """Deviations h (FP64) -> the nearest value the storage format holds, as FP64."""
    s = SCALE[storage]
    if storage == "f32":
        return np.asarray(h, dtype=np.float64).astype(np.float32).astype(np.float64)
    if storage == "f16":
        return (np.asarray(h, dtype=np.float64) * s).astype(np.float16).astype(np.float64) / s
    if storage == "bf16":
        return to_bf16(h)
    raise ValueError(storage)


def round_state(f, w, storage):
    """f -> w + round(f - w): the state as the library would store it."""
    return w + round_values(f - w, storage)
