"""Pins for the oracle's Philox4x64-10: numpy's independent implementation."""
import numpy as np

from oracle import philox


def _numpy_block(counter, key):
    # numpy's Philox advances its counter by one before producing a block
    c = list(counter)
    c[0] = (c[0] - 1) & philox.MASK64
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


def test_matches_numpy_philox():
    rng = np.random.default_rng(0)
    cases = [((1, 0, 0, 0), (0, 0)), ((0xFFFFFFFFFFFFFFFF, 5, 6, 7), (9, 11))]
    for _ in range(20):
        cases.append((tuple(int(v) for v in rng.integers(0, 2**63, 4)),
                      tuple(int(v) for v in rng.integers(0, 2**63, 2))))
    for ctr, key in cases:
        if ctr[0] == 0:
            continue
        assert philox.philox4x64_10(ctr, key) == _numpy_block(ctr, key)


def test_purposes_are_distinct_streams():
    a = philox.philox4x64_10((3, 4, 0, 0), (7, philox.GKTS))
    b = philox.philox4x64_10((3, 4, 0, 0), (7, philox.PRTB))
    assert a != b
    assert len({philox.INIT, philox.GKTS, philox.PRTB, philox.AMSP}) == 4


def test_uniform_and_index_maps():
    assert philox.uniform53(0) == 0.0
    assert philox.uniform53(2**64 - 1) == 1.0 - 2.0**-53
    assert philox.index_below(2**64 - 1, 7) == 6
    assert philox.index_below(0, 7) == 0
    # uniformity of the stream (chi-square on 16 bins)
    words = [philox.philox4x64_10((i, 0, 0, 0), (1, 2))[0] for i in range(4000)]
    counts = np.bincount([philox.index_below(w, 16) for w in words], minlength=16)
    chi2 = ((counts - 250.0) ** 2 / 250.0).sum()
    assert chi2 < 45  # 15 dof, p ~ 1e-4
