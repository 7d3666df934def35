"""Second, independent Philox4x32-10 in plain Python integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Written from the generator's published definition (Salmon, Moraes, Dror,
Shaw, SC'11): a 4-word counter passes through ten rounds of an S-box made of
two 32x32->64 multiplications; the two 32-bit key words advance by Weyl
constants between rounds.  The state is held as a Python list and the
products as arbitrary-precision integers, so that it shares neither structure
nor integer types with the C oracle.
"""
from __future__ import annotations

MASK32 = (1 << 32) - 1
MULTIPLIERS = (0xD2511F53, 0xCD9E8D57)
WEYL = (0x9E3779B9, 0xBB67AE85)


def _round(x, k):
    prod0 = MULTIPLIERS[0] * x[0]
    prod1 = MULTIPLIERS[1] * x[2]
    hi0, lo0 = divmod(prod0, 1 << 32)
    hi1, lo1 = divmod(prod1, 1 << 32)
    return [hi1 ^ x[1] ^ k[0], lo1, hi0 ^ x[3] ^ k[1], lo0]


def philox4x32_10(counter, key):
    x = [int(c) & MASK32 for c in counter]
    k = [int(key[0]) & MASK32, int(key[1]) & MASK32]
    for r in range(10):
        x = _round(x, k)
        k = [(k[0] + WEYL[0]) & MASK32, (k[1] + WEYL[1]) & MASK32]
    return x


def u01(word: int) -> float:
    """(2k+1) / 2^24 with k the top 23 bits -- exact rational, as a float."""
    return (2 * (word >> 9) + 1) / float(1 << 24)
