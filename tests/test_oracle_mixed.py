"""Pins for the storage roundings of the mixed-precision form: FP64 -> FP32
and FP64 -> FP32 -> BF16, both round to nearest with ties to even. They are
checked against torch's CPU conversions (an independent implementation of
the IEEE rounding) and against hand-worked ties, carries and overflows."""
import numpy as np
import pytest

from oracle.mixed import round_bf16, round_f32


def _values(seed, n=20000):
    rng = np.random.default_rng(seed)
    mags = 10.0 ** rng.uniform(-40, 38, n)
    vals = mags * rng.choice([-1.0, 1.0], n)
    # values that sit exactly on or next to FP32 and BF16 rounding boundaries
    f = rng.standard_normal(n).astype(np.float32)
    bits = f.view(np.uint32)
    ties_bf16 = ((bits & 0xFFFF0000) | 0x8000).view(np.float32).astype(np.float64)
    near_bf16 = ((bits & 0xFFFF0000) | 0x7FFF).view(np.float32).astype(np.float64)
    d = rng.standard_normal(n)
    ties_f32 = d.astype(np.float32).astype(np.float64) * (1.0 + 2.0 ** -24)
    return np.concatenate([vals, ties_bf16, near_bf16, ties_f32, d, [0.0, -0.0]])


@pytest.mark.parametrize("seed", [0, 1])
def test_round_f32_matches_torch(seed):
    import torch
    x = _values(seed)
    want = torch.from_numpy(x).to(torch.float32).to(torch.float64).numpy()
    assert np.array_equal(round_f32(x), want)


@pytest.mark.parametrize("seed", [0, 1])
def test_round_bf16_matches_torch(seed):
    import torch
    x = _values(seed)
    want = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = round_bf16(x)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all()


def test_round_bf16_hand_cases():
    # BF16 keeps 8 significant bits: the spacing just above 1 is 2^-7
    cases = [
        (1.0 + 2.0 ** -8, 1.0),                        # tie, even neighbour below
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),        # tie, even neighbour above
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),   # just past the tie
        (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),  # sign symmetric
        (2.0 - 2.0 ** -9, 2.0),                        # carry into the exponent
        (3.3895313892515355e38, 3.3895313892515355e38),  # largest finite BF16
        (3.4028234663852886e38, np.inf),               # largest FP32 rounds past it
        (2.0 ** -133, 2.0 ** -133),                    # subnormal, exact
        (0.1, 0.10009765625),
    ]
    for x, want in cases:
        assert round_bf16(np.array([x]))[0] == want, x


def test_round_f32_hand_cases():
    cases = [
        (1.0 + 2.0 ** -24, 1.0),                       # tie, even below
        (1.0 + 3 * 2.0 ** -24, 1.0 + 2.0 ** -22),      # tie, even above
        (1.0 + 2.0 ** -24 + 2.0 ** -40, 1.0 + 2.0 ** -23),
        (0.1, 0.100000001490116119384765625),
        (3.4028235677973366e38, np.inf),               # half an ulp past FP32's largest
    ]
    for x, want in cases:
        assert round_f32(np.array([x]))[0] == want, x
