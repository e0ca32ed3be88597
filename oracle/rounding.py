"""Round-to-nearest-even into the reduced formats the HIP path stores.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * binary32: numpy's float64 -> float32 cast (IEEE RNE).
  * bfloat16: 1 sign, 8 exponent, 7 mantissa bits; a float32 is rounded
    to its upper 16 bits, ties to the even upper half. Values arrive as
    float32 first (the kernels round FP32 accumulators), so bf16(x) is
    RNE_bf16(RNE_f32(x)). bf16_down / bf16_up round toward -inf / +inf (the
    16-bit normalisation metadata).
  * OCP FP8 E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits, no
    infinities, largest finite 448, smallest subnormal 2^-9; rounding to
    nearest even with saturation at +-448 (the latent quantiser never
    produces magnitudes above 448 before rounding).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """uint16 bit patterns of RNE_bf16(RNE_f32(x)) (finite inputs)."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32)).view(np.uint32)
    lsb = (u >> np.uint32(16)) & np.uint32(1)
    r = (u + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_from_bits(b) -> np.ndarray:
    u = np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    with np.errstate(invalid="ignore"):
        return u.view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    return bf16_from_bits(bf16_bits(x))


def _bf16_ordered(b):
    """bfloat16 bits -> integers ordered like the values (sign-magnitude to two's
    complement order; -0 and +0 both map to 0)."""
    b = np.asarray(b, dtype=np.uint16).astype(np.int64)
    return np.where(b & 0x8000, -(b & 0x7FFF), b)


def _bf16_from_ordered(o):
    o = np.asarray(o, dtype=np.int64)
    return np.where(o < 0, (-o) | 0x8000, o).astype(np.uint16)


def bf16_down(x) -> np.ndarray:
    """Largest bfloat16 value <= x (finite x, float64 exact comparison)."""
    x = np.asarray(x, dtype=np.float64)
    o = _bf16_ordered(bf16_bits(x))
    c = bf16_from_bits(_bf16_from_ordered(o))
    o = np.where(c > x, o - 1, o)
    return bf16_from_bits(_bf16_from_ordered(o))


def bf16_up(x) -> np.ndarray:
    """Smallest bfloat16 value >= x (finite x, float64 exact comparison)."""
    x = np.asarray(x, dtype=np.float64)
    o = _bf16_ordered(bf16_bits(x))
    c = bf16_from_bits(_bf16_from_ordered(o))
    o = np.where(c < x, o + 1, o)
    return bf16_from_bits(_bf16_from_ordered(o))


def e4m3(x) -> np.ndarray:
    """Values of RNE_e4m3(x) with saturation (x float64, finite)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    _, ex = np.frexp(a)                 # a = f 2^ex, f in [0.5, 1)
    e = np.maximum(ex - 1, -6)          # binade exponent; subnormals share 2^-6
    quantum = np.ldexp(1.0, e - 3)      # 3 mantissa bits
    r = np.rint(a / quantum) * quantum  # np.rint rounds half to even
    r = np.minimum(r, E4M3_MAX)
    r = np.where(a == 0.0, 0.0, r)
    return np.copysign(r, x)


def e4m3_bits(x) -> np.ndarray:
    """uint8 codes of e4m3(x)."""
    v = e4m3(x)
    sign = (np.signbit(v)).astype(np.uint8) << 7
    a = np.abs(v)
    _, ex = np.frexp(a)
    e = ex - 1
    normal = (a >= 2.0 ** -6)
    exp_field = np.where(normal, e + 7, 0)
    mant = np.where(normal, a / np.ldexp(1.0, e) - 1.0, a / 2.0 ** -6) * 8.0
    code = (exp_field.astype(np.int64) << 3) | np.rint(mant).astype(np.int64)
    code = np.where(a == 0.0, 0, code)
    return (code.astype(np.uint8) | sign).astype(np.uint8)


def e4m3_decode(code) -> np.ndarray:
    c = np.asarray(code, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    ex = (c >> 3) & 0xF
    mt = c & 0x7
    val = np.where(ex == 0, mt * 2.0 ** -9, (1.0 + mt / 8.0) * np.ldexp(1.0, ex - 7))
    val = np.where((c & 0x7F) == 0x7F, np.nan, val)
    return s * val
