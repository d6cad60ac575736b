"""Reduced-precision emulation of the M2L step.  Oracle: test infrastructure.

Used only to predict, before and beside the GPU kernels, the error that a
reduced-precision coupling step adds to Alg. 4, and so to fix the tolerance
of the mixed-precision GPU path from the arithmetic rather than from the GPU
output.  Modes (operands = coupling matrix and moments of one M2L product):

* ``fp64``      plain FP64 (the oracle itself);
* ``fp32``      operands rounded to FP32, each product summed in FP32, the
                sum over offsets accumulated in FP32;
* ``fp32acc64`` as ``fp32`` but the sum over offsets accumulated in FP64;
* ``bf16x3``    operands split into BF16 hi + lo parts, products
                ``hi*hi + hi*lo + lo*hi`` summed in FP32, sum over offsets in
                FP64;
* ``bf16x6``    operands split into BF16 hi + mid + lo parts (24 significant
                bits), the six products of order <= 2 (hh, hm, mh, hl, mm,
                lh) summed in FP32, sum over offsets in FP64.

Pinned by: BF16 rounding equal to torch's float32 -> bfloat16 conversion
(round to nearest even) and on hand-made ties; the error bounds of the two-
and three-part splits; products on operands built from exact BF16 parts,
where the three-product split equals the exact product minus the lo*lo
terms bit for bit; and the error band of each mode on random operands.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), as FP32."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split_bf16(x: np.ndarray):
    x = np.asarray(x, dtype=np.float32)
    hi = round_bf16(x)
    lo = round_bf16(x - hi)
    return hi, lo


def split3_bf16(x: np.ndarray):
    """x (FP64) = hi + mid + lo + O(2^-25 |x|), each part a BF16 value."""
    x = np.asarray(x, dtype=np.float64)
    hi = round_bf16(x.astype(np.float32)).astype(np.float64)
    mid = round_bf16((x - hi).astype(np.float32)).astype(np.float64)
    lo = round_bf16((x - hi - mid).astype(np.float32)).astype(np.float64)
    return hi.astype(np.float32), mid.astype(np.float32), lo.astype(np.float32)


def product(A: np.ndarray, M: np.ndarray, mode: str) -> np.ndarray:
    """``M @ A.T`` (rows of moments times coupling) in the given precision."""
    if mode == "fp64":
        return M @ A.T
    if mode in ("fp32", "fp32acc64"):
        return (M.astype(np.complex64) @ A.T.astype(np.complex64))
    if mode == "bf16x3":
        Ar_h, Ar_l = split_bf16(A.real)
        Ai_h, Ai_l = split_bf16(A.imag)
        Mr_h, Mr_l = split_bf16(M.real)
        Mi_h, Mi_l = split_bf16(M.imag)

        def mm(xh, xl, yh, yl):
            return (xh @ yh.T) + (xh @ yl.T) + (xl @ yh.T)

        re = mm(Mr_h, Mr_l, Ar_h, Ar_l) - mm(Mi_h, Mi_l, Ai_h, Ai_l)
        im = mm(Mr_h, Mr_l, Ai_h, Ai_l) + mm(Mi_h, Mi_l, Ar_h, Ar_l)
        return (re + 1j * im).astype(np.complex64)
    if mode == "bf16x6":
        Ar, Ai = split3_bf16(A.real), split3_bf16(A.imag)
        Mr, Mi = split3_bf16(M.real), split3_bf16(M.imag)

        def mm6(x, y):
            h, m, l = x
            H, Mm, Lo = y
            return ((h @ H.T) + (h @ Mm.T) + (m @ H.T) + (h @ Lo.T) + (m @ Mm.T) +
                    (l @ H.T))

        re = mm6(Mr, Ar) - mm6(Mi, Ai)
        im = mm6(Mr, Ai) + mm6(Mi, Ar)
        return (re + 1j * im).astype(np.complex64)
    raise ValueError(mode)


def accumulate_dtype(mode: str):
    return np.complex64 if mode == "fp32" else np.complex128
