"""Emulation of the reduced-precision correlator inputs, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's cost model assumes 2 bytes per visibility or DFT bin (Sec. 5.2,
Table survey_params); the 8- and 16-bit input formats emulated here are this
project's precision options, not the paper's.  Formats:

* OCP FP8 E4M3 ("e4m3fn"): sign, 4 exponent bits (bias 7), 3 mantissa bits,
  no infinities, S.1111.111 is NaN, so the largest finite value is 448;
  subnormals are m * 2^-9.  Conversion rounds to nearest, ties to even, and
  saturates to +-448.
* IEEE binary16 with round-to-nearest-even, saturated to +-65504.
"""

import numpy as np

E4M3_MAX = 448.0
F16_MAX = 65504.0


def e4m3_decode_table():
    """Value of each of the 256 E4M3 codes (NaN for the two NaN codes)."""
    vals = np.empty(256, dtype=np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * m * 2.0 ** -9
        else:
            vals[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


def e4m3_quantize(x):
    """Round real x to the nearest E4M3 value (ties to even), saturating."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    _, ex = np.frexp(np.where(a > 0, a, 1.0))  # a = mant * 2**ex, mant in [0.5, 1)
    e = ex - 1                                   # floor(log2 a)
    q = np.where(a < 2.0 ** -6, 2.0 ** -9, np.ldexp(1.0, e - 3))
    r = np.rint(a / q) * q                       # np.rint rounds half to even
    r = np.minimum(r, E4M3_MAX)
    return np.copysign(r, x)


def fp16_quantize(x):
    """Round real x to binary16 (ties to even), saturating to +-65504."""
    x = np.asarray(x, dtype=np.float64)
    return np.clip(x, -F16_MAX, F16_MAX).astype(np.float16).astype(np.float64)


def quantize(z, kind):
    """Quantise real and imaginary parts of complex z separately."""
    f = {"e4m3": e4m3_quantize, "f16": fp16_quantize}[kind]
    z = np.asarray(z)
    return f(z.real) + 1j * f(z.imag)
