"""Pins of the oracle's random-number layer (not GPU)."""
import numpy as np
import pytest

from oracle import oracle as O

# Known-answer vectors published with Philox4x32-10 (Salmon et al., SC'11,
# distributed with the Random123 library): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert tuple(O.philox4x32_10(ctr, key)) == expect


def test_u53_construction():
    # 27 high bits of the first word, 26 of the second, scaled by 2^-53.
    assert O.u53(0, 0) == 0.0
    assert O.u53(0xFFFFFFFF, 0xFFFFFFFF) == (2.0 ** 53 - 1) / 2.0 ** 53
    assert O.u53(1 << 5, 0) == 2.0 ** 26 / 2.0 ** 53
    assert O.u53(0, 1 << 6) == 1.0 / 2.0 ** 53
    assert O.u53(0x1F, 0x3F) == 0.0  # dropped low bits
    assert 1.0 - O.u53(0xFFFFFFFF, 0xFFFFFFFF) == 2.0 ** -53  # 1-u exact, never 0


def test_philox_uniform_moments():
    # Counter-mode outputs over consecutive counters: the four words are
    # uniform and uncorrelated (mean, variance, lag/word correlations).
    n = 20000
    words = np.array([O.philox4x32_10((k, 7, 0, 3), (1, 0x10)) for k in range(n)], dtype=np.float64)
    u = words / 2.0 ** 32
    se = np.sqrt(1.0 / 12.0 / n)
    for j in range(4):
        assert abs(u[:, j].mean() - 0.5) < 5 * se
        assert abs(u[:, j].var() - 1.0 / 12.0) < 5 * np.sqrt(1.0 / 180.0 / n)
    z = u - 0.5
    for j in range(4):
        for k in range(j + 1, 4):
            assert abs((z[:, j] * z[:, k]).mean()) < 5 / 12.0 / np.sqrt(n)
        assert abs((z[1:, j] * z[:-1, j]).mean()) < 5 / 12.0 / np.sqrt(n)
    # bit balance of every output bit
    bits = ((words[:, :, None].astype(np.uint64) >> np.arange(32, dtype=np.uint64)) & 1).mean(0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(n))
