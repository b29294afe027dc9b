"""bfloat16 round-to-nearest-even and the 3-term split-bf16 product.

Used only to unit-test the reduced-precision sketch products: the sketch runs
with bf16 operands (float32 inputs rounded to nearest even in the loader) and
float32 accumulation; the "bf16x3" form writes x = hi + lo with hi = bf16(x),
lo = bf16(x - hi) and keeps the three leading partial products
lo*hi + hi*lo + hi*hi (Henry, Tang & Heinecke, ARITH 2019).
"""
import numpy as np


def to_bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32 holding the bf16 value.  NaN stays NaN."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))
    r = ((b + bias) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = np.nan
    return out


def split3(x):
    """hi, lo bf16 parts (as float32) of float32 x: hi = bf16(x), lo = bf16(x - hi)."""
    x = np.asarray(x, dtype=np.float32)
    hi = to_bf16(x)
    lo = to_bf16((x - hi).astype(np.float32))
    return hi, lo


def matmul_bf16(A, B):
    """Exact (float64) product of the bf16-rounded operands."""
    return to_bf16(A).astype(np.float64) @ to_bf16(B).astype(np.float64)


def matmul_bf16x3(A, B):
    """Exact (float64) value of the three-term split-bf16 product."""
    ah, al = (t.astype(np.float64) for t in split3(A))
    bh, bl = (t.astype(np.float64) for t in split3(B))
    return al @ bh + ah @ bl + ah @ bh
