"""Pins of the oracle's storage codecs against torch's own conversions and the
OCP E4M3 definition."""
import numpy as np
import pytest
import torch

from oracle import codec


def test_e4m3_decode_table_matches_torch():
    codes = torch.arange(256, dtype=torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = codec.e4m3_decode_table()
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(got))
    assert np.array_equal(ref[~nan], got[~nan])
    assert got[0x7E] == 448.0 and got[0x01] == 2.0 ** -9 and got[0x08] == 2.0 ** -6


def test_e4m3_encode_matches_torch_rne():
    g = np.random.default_rng(0)
    tbl = codec.e4m3_decode_table()
    fin = tbl[np.isfinite(tbl)]
    mids = (np.sort(np.unique(fin))[1:] + np.sort(np.unique(fin))[:-1]) / 2  # exact ties
    x = np.concatenate([g.standard_normal(20000) * 40, g.uniform(-448, 448, 5000),
                        g.standard_normal(5000) * 1e-2, mids, -mids, [0.0, -0.0, 448.0, -448.0]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = codec.e4m3_encode(x)
    # torch keeps the sign of -0.0 and of values that round to zero; the
    # codec folds them to +0 (same decoded value 0)
    zero = (ref & 0x7F) == 0
    assert np.array_equal(got[~zero], ref[~zero])
    assert np.all((got[zero] & 0x7F) == 0)


def test_e4m3_saturates():
    assert codec.e4m3_encode(np.array([1e6, -1e6, 470.0], np.float32)).tolist() == [0x7E, 0xFE, 0x7E]


def test_bf16_and_f16_match_torch():
    g = np.random.default_rng(1)
    x = np.concatenate([g.standard_normal(50000) * 100, g.standard_normal(1000) * 1e-3,
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8)])]).astype(np.float32)
    bf = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(codec.bf16_encode(x), bf)
    hf = torch.from_numpy(x).to(torch.float16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(codec.f16_encode(x), hf)
    np.testing.assert_array_equal(codec.bf16_decode(bf),
                                  torch.from_numpy(bf.view(np.int16)).view(torch.bfloat16).double().numpy())


@pytest.mark.parametrize("amax,E,expect", [
    (1.0, 8, 2.0 ** -8), (1.5, 8, 2.0 ** -7), (0.75, 15, 2.0 ** -15), (256.0, 8, 1.0),
    (257.0, 8, 2.0), (0.0, 8, 1.0), (3.0, 15, 2.0 ** -13)])
def test_pow2_scale(amax, E, expect):
    assert codec.pow2_scale(amax, E) == expect


@pytest.mark.parametrize("dtype", ["bf16", "f16", "fp8_e4m3"])
def test_tile_quantization_round_trip(dtype):
    g = np.random.default_rng(4)
    R = (g.standard_normal((3, 70, 130)) * np.exp(g.standard_normal((3, 70, 130)))).astype(np.float32)
    R[1, :64, :64] = 0.0
    codes, scales = codec.quantize(R, dtype)
    assert scales.shape == (3, 2, 3)
    assert scales[1, 0, 0] == 1.0
    deq = codec.dequantize(codes, scales, dtype)
    rel = {"bf16": 2 ** -8, "f16": 2 ** -11, "fp8_e4m3": 2 ** -4}[dtype]
    # error bounded by half an ulp relative, or half the subnormal step x s
    s_full = np.repeat(np.repeat(scales, 64, 1), 64, 2)[:, :70, :130]
    sub = {"bf16": 2.0 ** -134, "f16": 2.0 ** -25, "fp8_e4m3": 2.0 ** -10}[dtype]
    assert np.all(np.abs(deq - R) <= np.maximum(np.abs(R) * rel, s_full * sub))
    # value-idempotent: re-quantizing the dequantized stack reproduces it
    # (codes may differ where a tile's amax rounded down into the binade below)
    c2, s2 = codec.quantize(deq, dtype)
    assert np.array_equal(codec.dequantize(c2, s2, dtype), deq)
