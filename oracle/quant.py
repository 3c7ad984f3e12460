"""Storage rounding of control points (test infrastructure only).

The paper stores control points as the model's coefficients (Sec. III-A,
Sec. IV-A2) and gives no reduced-precision form.  The reading used: stored
value = RNE(FP64 -> FP32), then for 16-bit storage RNE(FP32 -> BF16) or
RNE(FP32 -> FP16), each round-to-nearest-even at the bit level.
"""
from __future__ import annotations

import numpy as np


def to_f32(x64: np.ndarray) -> np.ndarray:
    """FP64 -> FP32, IEEE round-to-nearest-even (numpy's conversion)."""
    return np.asarray(x64, dtype=np.float64).astype(np.float32)


def f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit pattern (uint16), round to nearest even.

    The BF16 value is the top 16 bits of the FP32 pattern after adding
    0x7FFF plus the lowest kept bit (ties go to the even pattern); NaNs keep
    their sign and become a quiet NaN.
    """
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep_lsb) >> np.uint64(16)) & np.uint64(0xFFFF)
    isnan = np.isnan(np.asarray(x32, dtype=np.float32))
    qnan = ((u >> np.uint64(16)) | np.uint64(0x0040)) & np.uint64(0xFFFF)
    return np.where(isnan, qnan, r).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def f32_to_f16_bits(x32: np.ndarray) -> np.ndarray:
    """FP32 -> IEEE binary16 bit pattern (uint16), round to nearest even,
    with gradual underflow and overflow to infinity."""
    x = np.asarray(x32, dtype=np.float32)
    u = x.view(np.uint32).astype(np.int64)
    sign = (u >> 31) & 1
    exp = (u >> 23) & 0xFF
    man = u & 0x7FFFFF
    out = np.zeros(u.shape, dtype=np.int64)
    isnan = (exp == 0xFF) & (man != 0)
    isinf = (exp == 0xFF) & (man == 0)
    e16 = exp - 127 + 15
    # normal range result (before rounding): 10-bit mantissa
    full = man | (1 << 23)                              # 24-bit significand
    # number of bits to drop: 13 for normals, more for subnormals
    shift = np.where(e16 >= 1, 13, 13 + 1 - e16)
    shift = np.clip(shift, 13, 40)
    sig = np.where(exp == 0, man, full)                 # fp32 subnormals ~ 0
    kept = sig >> shift
    rem = sig - (kept << shift)
    half = np.int64(1) << (shift - 1)
    round_up = (rem > half) | ((rem == half) & ((kept & 1) == 1))
    kept = kept + round_up.astype(np.int64)
    # assemble: for normals, kept includes the implicit bit at position 10
    normal = e16 >= 1
    mag_norm = ((e16 << 10) + (kept - (1 << 10)))      # carries into exponent naturally
    mag_sub = kept                                       # exponent field 0 (or 1 after carry)
    mag = np.where(normal, mag_norm, mag_sub)
    mag = np.where(mag >= 0x7C00, 0x7C00, mag)          # overflow -> inf
    out = (sign << 15) | mag
    out = np.where(isinf, (sign << 15) | 0x7C00, out)
    out = np.where(isnan, (sign << 15) | 0x7E00 | (man >> 13), out)
    return (out & 0xFFFF).astype(np.uint16)


def f16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return np.asarray(b, dtype=np.uint16).view(np.float16).astype(np.float32)


def stored_values(ctrl64: np.ndarray, dtype: str) -> np.ndarray:
    """The FP64 values the stored control points represent."""
    x32 = to_f32(ctrl64)
    if dtype == "f32":
        return x32.astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f32(f32_to_bf16_bits(x32)).astype(np.float64)
    if dtype == "f16":
        return f16_bits_to_f32(f32_to_f16_bits(x32)).astype(np.float64)
    if dtype == "f64":
        return np.asarray(ctrl64, dtype=np.float64)
    raise ValueError(dtype)


def stored_bits(ctrl64: np.ndarray, dtype: str) -> np.ndarray:
    """Bit patterns of the stored control points (uint32 for f32, uint16 else)."""
    x32 = to_f32(ctrl64)
    if dtype == "f32":
        return x32.view(np.uint32)
    if dtype == "bf16":
        return f32_to_bf16_bits(x32)
    if dtype == "f16":
        return f32_to_f16_bits(x32)
    raise ValueError(dtype)
