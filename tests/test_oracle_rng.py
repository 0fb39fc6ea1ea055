"""Oracle pins: the counter-based generator and the uniform map."""
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox_known_answers(ctr, key, want):
    assert O.philox(ctr, key) == want


def test_philox_counter_sensitivity():
    base = O.philox([5, 6, 7, 8], [1234, 0])
    for lane in range(4):
        c = [5, 6, 7, 8]
        c[lane] ^= 1
        other = O.philox(c, [1234, 0])
        # every output word changes when any counter bit changes (avalanche)
        assert all(a != b for a, b in zip(base, other))


def test_uniform_map_exact():
    assert O.uniform(0) == 2.0 ** -24
    assert O.uniform(0xFFFFFFFF) == 1.0
    assert O.uniform(0x000000FF) == 2.0 ** -24       # low 8 bits dropped
    assert O.uniform(0x00000100) == 2.0 * 2.0 ** -24
    # every value is a multiple of 2^-24 in (0, 1]: exact in float32 too
    for w in [1, 12345, 0x80000000, 0xDEADBEEF]:
        u = O.uniform(w)
        assert 0 < u <= 1 and np.float32(u) == u and (u * 2 ** 24).is_integer()


def test_uniform_chi2():
    # 2^16 draws from consecutive counters; 64-bin chi^2 (p > 1e-4)
    from scipy import stats
    vals = []
    for c in range(1 << 14):
        vals.extend(O.uniform(w) for w in O.philox([c, 0, 0, 0], [99, 0]))
    h, _ = np.histogram(vals, bins=64, range=(0, 1))
    chi2 = ((h - len(vals) / 64) ** 2 / (len(vals) / 64)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4
