"""FP64 oracle: 16-bit checkpoint encodings with per-snapshot max-abs scaling.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper stores no checkpoints; the scheme is this implementation's (precision of stored
wavefield snapshots for the recomputation of the forward wavefield). Each field of a
snapshot gets one scale: FP16 stores x / s with s = max|x| / 2^14 (largest code 16384, well
inside FP16's 65504, values down to max|x| 2^-28 stay normal); BF16 stores x / s with
s = max|x| (BF16 has FP32's exponent range, the scale only normalizes). Both round to
nearest, ties to even. A field of zeros keeps scale 0 and decodes to zeros.
"""
from __future__ import annotations

import numpy as np

FP16_RANGE = 2.0 ** 14


def _bf16_round(x32):
    """float32 -> bfloat16 bits with round-to-nearest-even (finite inputs)."""
    u = np.ascontiguousarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def encode(x, codec):
    """Return (codes, scale) for one field."""
    x = np.asarray(x, np.float64)
    mx = float(np.max(np.abs(x))) if x.size else 0.0
    if codec == "fp16":
        scale = mx / FP16_RANGE
        q = (x / scale).astype(np.float16) if scale > 0 else np.zeros(x.shape, np.float16)
        return q, scale
    if codec == "bf16":
        scale = mx
        q = _bf16_round((x / scale).astype(np.float32)) if scale > 0 else np.zeros(x.shape, np.uint16)
        return q, scale
    raise ValueError(codec)


def decode(q, scale, codec):
    if codec == "fp16":
        return q.astype(np.float64) * scale
    if codec == "bf16":
        return _bf16_value(q) * scale
    raise ValueError(codec)


def roundtrip(x, codec):
    """decode(encode(x)); the identity (a copy) for codec None."""
    if codec is None:
        return np.array(x, np.float64, copy=True)
    q, s = encode(x, codec)
    return decode(q, s, codec)
