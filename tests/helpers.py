"""Test-side helpers: rounding of float64 test data into the storage formats
(single correct rounding, as numpy does for float16/float32) and the
normwise relative error used by the parity tests."""
import numpy as np

# Parity tolerances per storage format: normwise inf-norm relative error of a
# single kernel's output against the oracle on the same (upcast) inputs.
# FP64: rounding-order differences only; FP32 ~ 8 u32; FP16 ~ 4 u16; BF16 ~ 4 u_bf16.
TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3, "bf16": 1.6e-2}


def _f64_to_f32_odd(x):
    f = x.astype(np.float32)
    back = f.astype(np.float64)
    inexact = (back != x) & ~np.isnan(x)
    bits = f.view(np.uint32).copy()
    away = inexact & (np.abs(back) > np.abs(x))
    bits[away] -= 1
    bits[inexact] |= 1
    return bits.view(np.float32)


def _f32_to_bf16_bits(f):
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def round_to(x, prec):
    """Round float64 values to the nearest `prec` value (ties to even), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    if prec == "f64":
        return x.copy()
    if prec == "f32":
        return x.astype(np.float32).astype(np.float64)
    if prec == "f16":
        return x.astype(np.float16).astype(np.float64)
    if prec == "bf16":
        bits = _f32_to_bf16_bits(_f64_to_f32_odd(x))
        return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    raise ValueError(prec)


def rel_err(y, ref, denom=None):
    d = np.abs(ref).max() if denom is None else denom
    return float(np.abs(np.asarray(y) - np.asarray(ref)).max() / (d if d > 0 else 1.0))
