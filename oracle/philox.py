"""Philox4x32-10 counter-based generator in pure Python integers.

Test infrastructure only.  Written from the published definition (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
a round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
  (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.

The walk replaces the paper's CPU-made random pool (Sec. 3.1.3) with one
Philox block per photon step: counter = (step, instance, id_lo, id_hi),
key = (seed_lo, seed_hi).  Each 32-bit word r becomes the uniform
u = (2 floor(r / 2^9) + 1) / 2^24, which lies in (0, 1) and is exact in FP32.
"""
from __future__ import annotations

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def _round(c, k):
    p0 = M0 * c[0]
    p1 = M1 * c[2]
    return ((p1 >> 32) ^ c[1] ^ k[0], p1 & MASK, (p0 >> 32) ^ c[3] ^ k[1], p0 & MASK)


def philox4x32_10(counter, key):
    """Ten Philox4x32 rounds of a 4-word counter under a 2-word key."""
    c = tuple(int(v) & MASK for v in counter)
    k = [int(key[0]) & MASK, int(key[1]) & MASK]
    for r in range(10):
        if r:
            k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
        c = _round(c, k)
    return c


def step_block(seed: int, photon_id: int, step: int, instance: int = 0):
    """The four 32-bit words a photon draws at one step of its walk."""
    ctr = (step & MASK, instance & MASK, photon_id & MASK, (photon_id >> 32) & MASK)
    key = (seed & MASK, (seed >> 32) & MASK)
    return philox4x32_10(ctr, key)


def to_uniform(r: int) -> float:
    """u = (2 floor(r / 2^9) + 1) / 2^24 in (0, 1)."""
    return (2 * (int(r) >> 9) + 1) / 16777216.0
