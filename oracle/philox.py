"""Philox4x32-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11.  Four 32-bit counter words and two
key words; ten rounds of two 32x32->64 multiplies, with a Weyl-sequence bump
of the key between rounds.

The paper draws its random numbers from a Mersenne twister (section 3.1.1).
A counter-based generator gives the same uniform distribution and lets two
independent implementations draw *identical* streams, so a Metropolis chain
can be replayed proposal for proposal.

Pinned by the published known-answer vectors in tests/golden/philox_kat.txt.

Stream layout used by the sampler (both implementations follow it):
  key     = (seed & 0xffffffff, seed >> 32)
  counter = (n & 0xffffffff, n >> 32, walker_global_id, tag)
with n the walker's proposal index and tag 0 for Metropolis proposals.
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85


def philox4x32_10(ctr: tuple[int, int, int, int], key: tuple[int, int]) -> tuple[int, int, int, int]:
    c0, c1, c2, c3 = (int(c) & MASK32 for c in ctr)
    k0, k1 = (int(k) & MASK32 for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK32,
                          (p0 >> 32) ^ c3 ^ k1, p0 & MASK32)
    return c0, c1, c2, c3


def proposal_draw(seed: int, walker_gid: int, n: int, tag: int = 0) -> tuple[int, int, int, int]:
    key = (seed & MASK32, (seed >> 32) & MASK32)
    ctr = (n & MASK32, (n >> 32) & MASK32, walker_gid & MASK32, tag & MASK32)
    return philox4x32_10(ctr, key)


def scaled_index(r: int, n: int) -> int:
    """Map a 32-bit word to {0..n-1} by multiply-shift (no floating point)."""
    return (r * n) >> 32


def uniform53(r2: int, r3: int) -> float:
    """53-bit uniform in [0, 1) from two 32-bit words; exact in binary64."""
    return ((r2 >> 5) * 67108864 + (r3 >> 6)) * (1.0 / 9007199254740992.0)
