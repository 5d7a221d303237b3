"""Pins of the oracle's precision reduction (FP64 -> FP32 -> BF16/FP16, each
step round-to-nearest-even) against independent library conversions and
hand-checked boundary values of the IEEE formats."""
import numpy as np
import torch


def _edge_f32():
    vals = [0.0, -0.0, 1.0, -1.0, 65504.0, 65505.0, 65519.0, 65520.0, 65536.0, 1e30, -1e30,
            np.inf, -np.inf, 2.0**-24, 2.0**-25, 2.0**-25 * 1.5, 2.0**-26, 2.0**-14, 2.0**-15,
            2.0**-14 * (1 - 2.0**-11), 3.0 * 2.0**-25, 1.0 + 2.0**-11, 1.0 + 3 * 2.0**-11,
            3.4028234e38, 1e-40, -1e-45, 2.0**-133]
    rng = np.random.default_rng(0)
    rand = np.concatenate([rng.standard_normal(20000),
                           rng.standard_normal(20000) * 10.0 ** rng.uniform(-10, 6, 20000)])
    return np.array(vals + list(rand), dtype=np.float32)


def test_f64_to_f32_matches_numpy(orc):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(50000) * 10.0 ** rng.uniform(-40, 40, 50000),
                        [0.0, -0.0, 1e-320, 3.4028235677973366e38, 1e39, np.inf]])
    with np.errstate(over="ignore"):
        np.testing.assert_array_equal(orc.round_f64_to_f32(x).view(np.uint32), x.astype(np.float32).view(np.uint32))


def test_f32_to_f16_matches_numpy(orc):
    x = _edge_f32()
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(orc.round_f32_to_f16_bits(x), ref)
    # hand-checked: 65520 is the tie to infinity, 2^-25 ties to +0, 1.5*2^-25
    # rounds up to the smallest subnormal
    got = orc.round_f32_to_f16_bits(np.array([65519.0, 65520.0, 2.0**-25, 1.5 * 2.0**-25], np.float32))
    np.testing.assert_array_equal(got, [0x7BFF, 0x7C00, 0x0000, 0x0001])


def test_f32_to_bf16_matches_torch(orc):
    x = _edge_f32()
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(orc.round_f32_to_bf16_bits(x), ref)
    # ties: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> even (1.0)
    got = orc.round_f32_to_bf16_bits(np.array([1 + 2.0**-8, 1 + 3 * 2.0**-8], np.float32))
    np.testing.assert_array_equal(got, [0x3F80, 0x3F82])


def test_two_step_rounding(orc):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-8, 4, 10000)
    f = x.astype(np.float32)
    np.testing.assert_array_equal(orc.round_f64_to_f16_bits(x), f.astype(np.float16).view(np.uint16))
    bf = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(orc.round_f64_to_bf16_bits(x), bf)
