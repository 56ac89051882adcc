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


def _e4m3_encode_flat(x: np.ndarray) -> np.ndarray:
    a = np.minimum(np.abs(x), 448.0)
    # exhaustive nearest search over the 127 non-negative finite codes
    d = np.abs(a[:, None] - _POS_VALS[None, :])
    best = d.min(axis=-1, keepdims=True)
    cand = d == best
    # ties: prefer the code with an even mantissa (lowest bit 0)
    even = (_POS_CODES & 1) == 0
    pick_even = cand & even[None, :]
    has_even = pick_even.any(axis=-1, keepdims=True)
    cand = np.where(has_even, pick_even, cand)
    code = _POS_CODES[np.argmax(cand, axis=-1)]
    sign = (np.signbit(x) & (code != 0)).astype(np.int64) << 7
    return (code | sign).astype(np.uint8)


def e4m3_encode(x) -> np.ndarray:
    """Round-to-nearest-even, saturating encode of finite values to E4M3fn codes."""
    x = np.asarray(x, dtype=np.float64)
    flat = x.reshape(-1)
    out = np.empty(flat.shape, np.uint8)
    step = 1 << 15
    for s in range(0, flat.size, step):
        out[s:s + step] = _e4m3_encode_flat(flat[s:s + step])
    return out.reshape(x.shape)


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


def quantize(R, dtype: str):
    """Quantize a [T][H][W] float32 stack.  Returns (codes, scales) with
    scales [T][ceil(H/64)][ceil(W/64)] float32."""
    R = np.asarray(R, dtype=np.float32)
    T, H, W = R.shape
    ty, tx = -(-H // TILE), -(-W // TILE)
    E = E_BITS[dtype]
    scales = np.zeros((T, ty, tx), np.float32)
    codes = np.zeros(R.shape, np.uint8 if dtype == "fp8_e4m3" else np.uint16)
    for k in range(T):
        for a in range(ty):
            for b in range(tx):
                blk = R[k, a * TILE:(a + 1) * TILE, b * TILE:(b + 1) * TILE]
                s = pow2_scale(float(np.max(np.abs(blk))), E)
                scales[k, a, b] = s
                codes[k, a * TILE:(a + 1) * TILE, b * TILE:(b + 1) * TILE] = \
                    ENCODE[dtype](blk / np.float32(s))
    return codes, scales


def dequantize(codes, scales, dtype: str) -> np.ndarray:
    """q * s for every element, in float32 (exact for power-of-two s)."""
    T, H, W = codes.shape
    vals = DECODE[dtype](codes).astype(np.float32)
    s = np.repeat(np.repeat(scales, TILE, axis=1), TILE, axis=2)[:, :H, :W]
    return (vals * s).astype(np.float32)
