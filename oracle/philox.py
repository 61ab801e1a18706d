"""Philox4x64-10 counter-based random number generator (oracle side).

Written from the published definition: J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11, Sec. 4 (Philox), with the 4x64 multipliers and Weyl key increments
given there.  Plain Python integers, one block at a time: obviously correct,
slow.  Pinned against ``numpy.random.Philox`` (tests/test_oracle_philox.py).

How the method uses it (readings of Sec. 2.4 steps 2 and 5, where the paper
only says "generate a random number Y ~ U(0,1)"):

* key = (seed, 0); counter = (global beam id, index, stream tag, 0).
* tag HOP: block (gid, k) serves hop k (k >= 1): word 0 -> U picks the
  destination, word 1 -> Y gives the next waiting-time threshold.
  Block (gid, 0) word 1 is the first threshold Y_0.
* tag NORMAL: block (gid, j) gives four standard normals for phase-space
  coordinates 4j..4j+3 by Box-Muller (Box & Muller 1958).
* tag UNIF: block (gid, c) word 0 is a uniform for coordinate c.
* a 64-bit word w maps to Y = ((w >> 12) + 1/2) * 2^-52, strictly inside
  (0, 1), so that 1 - Y is exact.
"""

MASK64 = (1 << 64) - 1

# Salmon et al. 2011, Philox4x64 round multipliers and key schedule constants.
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1

TAG_HOP = 0x48      # 'H'
TAG_NORMAL = 0x4E   # 'N'
TAG_UNIF = 0x55     # 'U'


def _mulhilo(a, b):
    p = a * b
    return p >> 64, p & MASK64


def philox4x64_10(counter, key):
    """Ten Philox rounds on a 4x64-bit counter under a 2x64-bit key."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0, c1, c2, c3)


def block(seed, gid, index, tag):
    """The block the method reads for (beam gid, draw index, stream tag)."""
    return philox4x64_10((gid, index, tag, 0), (seed, 0))


def u01(word):
    """Map a 64-bit word to a double strictly inside (0, 1)."""
    k = (int(word) & MASK64) >> 12
    return float(2 * k + 1) * 2.0 ** -53
