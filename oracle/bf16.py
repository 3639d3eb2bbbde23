"""BF16 emulation for the oracle (test infrastructure only).

The precision variant feeds D and Y to the matrix cores as BF16 (round to
nearest, ties to even) and accumulates in FP32.  The oracle separates
quantisation from kernel error by running its FP64 arithmetic on inputs
rounded the same way: ``round_bf16`` is that rounding, written out on the bit
pattern of an IEEE binary32 value (1 sign, 8 exponent, 23 fraction bits; BF16
keeps the top 16 bits).
"""
import numpy as np


def round_bf16(x):
    """Round float32 values to the nearest BF16 value (ties to even), returned
    as float32.  NaN stays NaN; values that round past the largest finite BF16
    become infinity, as the IEEE rounding rule gives."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(nan, np.float32(np.nan), out).reshape(a.shape)
