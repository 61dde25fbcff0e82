"""bfloat16 storage of a float32 factor (reduced-precision variant of the
factor L of Sec. 2.1).

bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits
of the IEEE-754 binary32 encoding.  Rounding to nearest, ties to even:
add 0x7FFF plus the lowest kept bit to the 32-bit pattern and drop the
low 16 bits.  NaNs stay NaN (quiet bit set).
"""
import numpy as np


def to_bf16_bits(x32):
    """uint16 bit patterns of bfloat16(x) for float32 x (round to nearest even)."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u.astype(np.uint64) + 0x7FFF + lsb) >> 16).astype(np.uint16)
    r = np.where(nan, ((u >> 16) | 0x40).astype(np.uint16), r)
    return r


def bf16_bits_to_f64(b):
    """float64 values of bfloat16 bit patterns."""
    u = (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16)
    return u.view(np.float32).astype(np.float64)


def round_to_bf16(x32):
    """bfloat16(x) as float64 values."""
    return bf16_bits_to_f64(to_bf16_bits(x32))
