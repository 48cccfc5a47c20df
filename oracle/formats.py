"""Exact decoders for the low-precision storage formats of A.

The method itself is precision-agnostic; the library can hold A in BF16 or in
FP8 with one FP32 scale per row.  The stored values are the ground truth: the
oracle works on their exact FP64 values.

* BF16: the upper 16 bits of an IEEE binary32 value.
* FP8 E4M3 (OCP 8-bit floating point specification, "E4M3FN"): 1 sign bit,
  4 exponent bits with bias 7, 3 mantissa bits, no infinities, NaN when all
  exponent and mantissa bits are set; largest finite magnitude 448;
  subnormals 2^-6 * m/8.
"""

import numpy as np


def bf16_bits_to_f64(bits):
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def e4m3_value(byte):
    """Value of one OCP E4M3 byte, written out from the format's definition."""
    byte = int(byte) & 0xFF
    sign = -1.0 if byte & 0x80 else 1.0
    exp = (byte >> 3) & 0xF
    man = byte & 0x7
    if exp == 0xF and man == 0x7:
        return float("nan")
    if exp == 0:
        return sign * (2.0 ** -6) * (man / 8.0)
    return sign * (2.0 ** (exp - 7)) * (1.0 + man / 8.0)


_E4M3_TABLE = np.array([e4m3_value(b) for b in range(256)], dtype=np.float64)


def e4m3_bits_to_f64(bits):
    return _E4M3_TABLE[np.asarray(bits, dtype=np.uint8)]


def fp8_rows_to_f64(bits, row_scale):
    """diag(row_scale) * decode(bits): the matrix an FP8 A with row scales stores."""
    vals = e4m3_bits_to_f64(bits)
    return vals * np.asarray(row_scale, dtype=np.float32).astype(np.float64)[:, None]
