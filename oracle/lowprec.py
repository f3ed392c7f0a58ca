"""Emulation of reduced-precision storage, for kernel-level parity of the
mixed-precision sketch.

* FP64 -> FP32: round to nearest, ties to even (IEEE 754 default; numpy's
  astype(float32) does exactly this).
* FP32 -> BF16: keep the upper 16 bits of the FP32 encoding after rounding
  the lower 16 bits to nearest, ties to even.  BF16 has the FP32 exponent
  range and 8 significant bits.
* FP64 -> BF16 is defined as FP64 -> FP32 -> BF16 (two roundings).

Test infrastructure (see the package docstring).
"""

import numpy as np


def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_bits(x32):
    """uint16 BF16 encodings of finite FP32 values, round to nearest even."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_to_f64(bits):
    u = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def round_bf16(x):
    """FP64 values rounded to BF16 (via FP32), returned as FP64."""
    return bf16_to_f64(bf16_bits(to_f32(x)))


def round_f32(x):
    return to_f32(x).astype(np.float64)


def sketch_bf16(A32, d, Omega):
    """The mixed-precision sketch Y = A D A^T Omega with BF16 operands:
    A_b = bf16(A32), O_b = bf16(Omega), W = d * (A_b^T O_b) rounded to BF16,
    Y = A_b W_b.  The products are exact sums in FP64 here (the device sums
    in FP32), so the two differ by the accumulation error only."""
    Ab = round_bf16(A32)
    Ob = round_bf16(Omega)
    W = d[:, None] * (Ab.T @ Ob)
    Wb = round_bf16(W)
    return Ab @ Wb
