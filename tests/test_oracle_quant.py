"""Pins of the oracle's storage quantizers against the format definitions and torch's
CPU conversions (an independent library routine).  BF16 is round-to-nearest-even from
FP32; FP8 is OCP E4M3FN with a per-Gaussian power-of-two FP32 scale."""
import numpy as np
import pytest
import torch


def test_e4m3_decode_all_codes(orc):
    t = orc.e4m3_table()
    lib = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).double().numpy()
    nan = np.isnan(lib)
    assert list(np.nonzero(nan)[0]) == [0x7F, 0xFF]
    assert np.all(np.isnan(t[nan]))
    np.testing.assert_array_equal(t[~nan], lib[~nan])
    # spec landmarks
    assert t[0x01] == 2.0 ** -9 and t[0x08] == 2.0 ** -6 and t[0x38] == 1.0 and t[0x7E] == 448.0
    assert t[0xFE] == -448.0 and np.signbit(t[0x80])
    assert np.all(np.diff(t[:0x7F]) > 0)


def _torch_e4m3(x):
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()


def test_e4m3_rounding_matches_library_in_range(orc):
    rng = np.random.default_rng(0)
    t = orc.e4m3_table()
    mids = (t[0:0x7E] + t[1:0x7F]) / 2        # exact ties between neighbours
    x = np.concatenate([rng.uniform(-460, 460, 20000), rng.uniform(-1e-2, 1e-2, 20000),
                        mids, -mids, t[:0x7F], [2.0 ** -10, 1e-4, 0.0]]).astype(np.float32)
    x = x[np.abs(x) < 464]
    # single-element rows with |x| in [224, 448) get scale 1: the encoding is direct
    xs = x[(np.abs(x) >= 224) & (np.abs(x) < 448)]
    c1, s1 = orc.fp8_quantize(xs.reshape(-1, 1))
    assert np.all(s1 == 1.0)
    np.testing.assert_array_equal(c1[:, 0], _torch_e4m3(xs))
    # the full set: pad each value into a row whose amax is 448 - so s = 2
    # (powers of two keep x/s exact); check against the library on x/2
    rows = np.stack([x, np.full_like(x, 448.0)], 1)
    c2, s2 = orc.fp8_quantize(rows)
    assert np.all(s2 == 2.0)
    np.testing.assert_array_equal(c2[:, 0], _torch_e4m3(x / 2))


def test_e4m3_saturates(orc):
    c, s = orc.fp8_quantize(np.array([[1000.0, 448.0]], np.float32))
    assert s[0] == 4.0
    c, s = orc.fp8_quantize(np.array([[447.9, 300.0]], np.float32))
    assert s[0] == 1.0 and c[0, 0] == 0x7E


def test_fp8_scale_rule(orc):
    rng = np.random.default_rng(1)
    x = (rng.standard_normal((500, 64)) * np.exp(rng.uniform(-30, 30, (500, 1)))).astype(np.float32)
    x[0] = 0
    codes, s = orc.fp8_quantize(x)
    amax = np.abs(x).max(1).astype(np.float64)
    assert s[0] == 1.0
    m, e = np.frexp(s[1:])
    assert np.all(m == 0.5)                      # powers of two
    r = amax[1:] / s[1:]
    assert np.all((r >= 224) & (r < 448))
    deq = orc.fp8_dequant(codes, s)
    rel = np.abs(deq - x) / np.maximum(amax[:, None], 1e-300)
    assert rel[1:].max() <= 2.0 ** -4     # half an ulp of amax's binade, relative to amax


def test_bf16_matches_library(orc):
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(50000) * np.exp(rng.uniform(-80, 80, 50000)),
                        rng.standard_normal(1000) * 1e-39]).astype(np.float32)
    # exact ties: low 16 bits = 0x8000, with even and odd kept parts
    u = rng.integers(0, 2 ** 31, 4000, dtype=np.uint64).astype(np.uint32)
    ties = ((u & 0xFFFF0000) | 0x8000).view(np.float32)
    x = np.concatenate([x, ties[np.isfinite(ties)]])
    ours = orc.bf16_bits(x)
    lib = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, lib)
    np.testing.assert_array_equal(orc.bf16_to_f64(ours),
                                  torch.from_numpy(x).to(torch.bfloat16).double().numpy())
