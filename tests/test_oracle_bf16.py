"""Pins of the oracle's BF16 rounding (the storage form of c and a).

oracle.bf16_round is written from the format's definition (8 significant bits,
FP32's exponent range, round to nearest with ties to even).  It is checked here
against two things that do not share its arithmetic: PyTorch's own float32 ->
bfloat16 conversion, and hand-worked bit patterns for ties, the largest finite
value, subnormals, infinities and NaN.
"""
import numpy as np
import pytest


def _bits(x):
    return np.asarray(x, dtype=np.float32).view(np.uint32)


def _f(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32)


def test_matches_torch_over_the_exponent_range(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    # random bit patterns: every exponent, subnormals included; NaN excluded here
    u = rng.integers(0, 2 ** 32, size=400_000, dtype=np.uint64).astype(np.uint32)
    x = _f(u)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(_bits(orc.bf16_round(x)), _bits(ref))


def test_ties_round_to_even_by_hand(orc):
    # the low 16 bits 0x8000 are exactly half a BF16 quantum
    cases = {
        0x3F808000: 0x3F800000,  # 1 + 2^-8: tie, kept bit even -> down to 1.0
        0x3F818000: 0x3F820000,  # 1 + 3 * 2^-8: tie, kept bit odd -> up
        0xBF808000: 0xBF800000,  # negative tie, even -> toward zero
        0xBF818000: 0xBF820000,  # negative tie, odd -> away from zero
        0x3F807FFF: 0x3F800000,  # just below the tie -> down
        0x3F808001: 0x3F810000,  # just above the tie -> up
        0x3F7FFFFF: 0x3F800000,  # largest float below 1 -> carries into the exponent
        0x00000000: 0x00000000,  # +0
        0x80000000: 0x80000000,  # -0 keeps its sign
        0x00008000: 0x00000000,  # subnormal tie at the bottom: even -> 0
        0x00018000: 0x00020000,  # subnormal tie, odd -> up
        0x007FFFFF: 0x00800000,  # largest subnormal rounds up to the smallest normal
        0x7F7F7FFF: 0x7F7F0000,  # below the tie under the largest BF16 -> largest finite BF16
        0x7F7F8000: 0x7F800000,  # tie at the top, kept bit odd -> overflows to +inf
        0x7F7FFFFF: 0x7F800000,  # FLT_MAX -> +inf
        0xFF7FFFFF: 0xFF800000,  # -FLT_MAX -> -inf
        0x7F800000: 0x7F800000,  # +inf
        0xFF800000: 0xFF800000,  # -inf
    }
    x = _f(list(cases))
    got = _bits(orc.bf16_round(x))
    for (src, want), g in zip(cases.items(), got):
        assert g == want, f"{src:#010x}: got {g:#010x}, want {want:#010x}"


def test_nan_stays_nan(orc):
    x = _f([0x7FC00000, 0x7FFFFFFF, 0xFFC00001, 0x7F800001])
    assert np.all(np.isnan(orc.bf16_round(x)))


def test_idempotent_and_monotone(orc):
    rng = np.random.default_rng(1)
    x = np.sort(rng.normal(size=100_000).astype(np.float32) * 100)
    r = orc.bf16_round(x)
    assert np.array_equal(_bits(orc.bf16_round(r)), _bits(r))
    assert np.all(np.diff(r.astype(np.float64)) >= 0)
    # within half a quantum: |x - r| <= 2^-8 |x| for normal values (8 significant bits)
    assert np.all(np.abs(x.astype(np.float64) - r) <= 2.0 ** -8 * np.abs(x.astype(np.float64)))
