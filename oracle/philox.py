"""Philox4x64-10 counter-based generator, from its published definition.

Test infrastructure (see ``oracle/__init__``).

Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, Section 3.2): a 4-word counter x and a 2-word key k; each of
10 rounds multiplies x0 and x2 by the constants M0 and M1 into 128-bit
products, and forms the new words from the high/low halves XOR-ed with the
other two words and the round key; the key is bumped by the Weyl constants
W0, W1 between rounds.  Pinned against ``numpy.random.Philox`` (an independent
library implementation of the same generator) in ``tests/test_oracle_philox``.

Random streams used by the method (one purpose tag per use, so that no two
uses ever draw the same counter):

=============  ==============  ===========================================
purpose        key             counter
=============  ==============  ===========================================
init noise     (seed, INIT)    (cell = y*nx + x, member, 0, 0), word 0
GKTL select    (key,  GKTS)    (slot m, period, 0, 0), word 0
perturbation   (key,  PRTB)    (slot m, period, n // 4, 0), word n % 4
AMS parent     (key,  AMSP)    (kill index j, iteration, 0, 0), word 0
=============  ==============  ===========================================

A 64-bit word w becomes a uniform double in [0, 1) as (w >> 11) * 2**-53, and
an index in [0, n) as floor(w * n / 2**64).
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B

# purpose tags: ASCII of the four-letter names, stored in key word 1
INIT = 0x494E4954  # "INIT"
GKTS = 0x474B5453  # "GKTS"
PRTB = 0x50525442  # "PRTB"
AMSP = 0x414D5350  # "AMSP"


def philox4x64_10(counter, key):
    """Return the four 64-bit output words for ``counter`` (4 ints) and ``key`` (2 ints)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for _ in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + W0) & MASK64
        k1 = (k1 + W1) & MASK64
    return (x0, x1, x2, x3)


def uniform53(word: int) -> float:
    """Map a 64-bit word to a double in [0, 1) with 53 random bits (exact)."""
    return (int(word) >> 11) * (2.0 ** -53)


def index_below(word: int, n: int) -> int:
    """Map a 64-bit word to an integer in [0, n) by the high half of word * n."""
    return (int(word) * int(n)) >> 64


def draw_word(key: int, purpose: int, c0: int, c1: int, c2: int = 0, word: int = 0) -> int:
    """One word of the stream ``purpose`` at counter (c0, c1, c2, 0)."""
    return philox4x64_10((c0, c1, c2, 0), (key, purpose))[word]
