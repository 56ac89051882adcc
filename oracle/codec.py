"""Storage codecs of the precision form, written out from their public definitions.

TEST INFRASTRUCTURE ONLY (see oracle/oracle.py).  The paper states no numeric
precision; the reduced-precision residual storage is this project's addition,
so this module follows the format definitions rather than the paper:

* OCP 8-bit floating point, E4M3 "fn" variant: 1 sign, 4 exponent (bias 7),
  3 mantissa bits; no infinities; S.1111.111 is NaN; largest finite 448;
  subnormals m * 2^-9.  Encoding rounds to nearest, ties to even, and
  saturates at +-448.
* bfloat16: the top 16 bits of an IEEE binary32, rounded to nearest even.
* IEEE binary16, rounded to nearest even (numpy's float16 cast).

Per-tile scaling: each frame is cut into 64x64 tiles aligned at (0,0) (edge
tiles may be partial).  A tile with largest magnitude amax gets the power of
two s = 2^(ceil(log2 amax) - E) (E = 8 for E4M3, 15 for binary16/bfloat16), or
s = 1 for an all-zero tile; codes store R/s and decode to q*s exactly in FP32.
"""
from __future__ import annotations

import numpy as np

TILE = 64
E_BITS = {"fp8_e4m3": 8, "f16": 15, "bf16": 15}


def e4m3_decode_table() -> np.ndarray:
    """Value of every one of the 256 E4M3fn codes (NaN for the two NaN codes)."""
    out = np.zeros(256, np.float64)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e = (c >> 3) & 0xF
        m = c & 0x7
        if e == 0xF and m == 0x7:
            out[c] = np.nan
        elif e == 0:
            out[c] = s * m * 2.0 ** -9
        else:
            out[c] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return out


_E4M3 = e4m3_decode_table()
_POS_CODES = np.array([c for c in range(0x7F)], dtype=np.int64)  # 0x00..0x7E finite, >= 0
_POS_VALS = _E4M3[_POS_CODES]


def e4m3_encode(x) -> np.ndarray:
    """Round-to-nearest-even, saturating encode of finite values to E4M3fn codes.

    The non-negative finite codes 0x00..0x7E decode to increasing values, so
    the two codes bracketing |x| are found by bisection; the nearer wins, and
    an exact tie goes to the code with an even mantissa (lowest bit 0)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    hi = np.searchsorted(_POS_VALS, a, side="left")          # _POS_VALS[hi-1] < a <= _POS_VALS[hi]
    hi = np.minimum(hi, _POS_VALS.size - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - _POS_VALS[lo]
    dhi = _POS_VALS[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((_POS_CODES[hi] & 1) == 0))
    code = np.where(pick_hi, _POS_CODES[hi], _POS_CODES[lo])
    code = np.where(a == _POS_VALS[hi], _POS_CODES[hi], code)
    sign = (np.signbit(x) & (code != 0)).astype(np.int64) << 7
    return (code | sign).astype(np.uint8)


def e4m3_decode(c) -> np.ndarray:
    return _E4M3[np.asarray(c, dtype=np.int64)]


def bf16_encode(x) -> np.ndarray:
    """binary32 -> bfloat16 bits, round to nearest even (finite inputs)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    return ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_decode(c) -> np.ndarray:
    return (np.asarray(c, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def f16_encode(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def f16_decode(c) -> np.ndarray:
    return np.asarray(c, dtype=np.uint16).view(np.float16).astype(np.float64)


ENCODE = {"fp8_e4m3": e4m3_encode, "f16": f16_encode, "bf16": bf16_encode}
DECODE = {"fp8_e4m3": e4m3_decode, "f16": f16_decode, "bf16": bf16_decode}


def pow2_scale(amax: float, E: int) -> float:
    """2^(ceil(log2 amax) - E), or 1 for amax == 0."""
    if amax == 0.0:
        return 1.0
    m, e = np.frexp(amax)  # amax = m * 2^e, m in [0.5, 1)
    c = e - 1 if m == 0.5 else e
    return float(np.ldexp(1.0, int(c) - E))


def pow2_scales(amax: np.ndarray, E: int) -> np.ndarray:
    """pow2_scale applied elementwise."""
    m, e = np.frexp(amax.astype(np.float64))
    c = np.where(m == 0.5, e - 1, e)
    return np.where(amax == 0.0, 1.0, np.ldexp(1.0, c - E)).astype(np.float32)


def quantize(R, dtype: str):
    """Quantize a [T][H][W] float32 stack.  Returns (codes, scales) with
    scales [T][ceil(H/64)][ceil(W/64)] float32.  Frame by frame: the frame is
    zero-padded to whole tiles (padding does not change a tile's amax), each
    tile's scale comes from its amax, and every value is encoded as R/s."""
    R = np.asarray(R, dtype=np.float32)
    T, H, W = R.shape
    ty, tx = -(-H // TILE), -(-W // TILE)
    E = E_BITS[dtype]
    scales = np.zeros((T, ty, tx), np.float32)
    codes = np.zeros(R.shape, np.uint8 if dtype == "fp8_e4m3" else np.uint16)
    pad = np.zeros((ty * TILE, tx * TILE), np.float32)
    for k in range(T):
        pad[:H, :W] = R[k]
        amax = np.abs(pad).reshape(ty, TILE, tx, TILE).max(axis=(1, 3))
        s = pow2_scales(amax, E)
        scales[k] = s
        sfull = np.repeat(np.repeat(s, TILE, axis=0), TILE, axis=1)[:H, :W]
        codes[k] = ENCODE[dtype](R[k] / sfull)
    return codes, scales


def dequantize(codes, scales, dtype: str) -> np.ndarray:
    """q * s for every element, in float32 (exact for power-of-two s)."""
    T, H, W = codes.shape
    vals = DECODE[dtype](codes).astype(np.float32)
    s = np.repeat(np.repeat(scales, TILE, axis=1), TILE, axis=2)[:, :H, :W]
    return (vals * s).astype(np.float32)
