"""Philox4x32-10 counter-based generator (oracle side).

Test infrastructure only: nothing in the product path imports this module.

Definition: Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3" (SC'11), section 4.2.  One round maps counter (c0, c1, c2, c3) and
key (k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with M0 = 0xD2511F53 and M1 = 0xCD9E8D57; between rounds the key is bumped
by the Weyl constants (0x9E3779B9, 0xBB67AE85).  Ten rounds.

Pinned by the known-answer vectors published with the reference
implementation (Random123), see tests/test_oracle_philox.py.

Uniform conversion used by the sampler and by the accept step: the 53-bit
integer (w0 >> 5) * 2**26 + (w1 >> 6) scaled by 2**-53, a double in [0, 1).

Stream layout (counter words), shared by both sides of the parity tests:

* site draw of the sampler:   (site = r*L + c, sample, instance, 0)
* Metropolis accept draw:     (proposal, 0, instance, 1)

The key is (seed & 0xffffffff, seed >> 32).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

STREAM_SITE = 0
STREAM_ACCEPT = 1


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Vectorised Philox4x32; all arguments broadcast, uint32 semantics."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK32 for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3, k0, k1 = (x.copy() for x in (c0, c1, c2, c3, k0, k1))
    for rnd in range(rounds):
        if rnd > 0:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = M0 * c0          # < 2**64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def key_of(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def to_unit_double(w0, w1):
    """53 random bits from two words -> double in [0, 1)."""
    hi = np.asarray(w0, dtype=np.uint64) >> np.uint64(5)
    lo = np.asarray(w1, dtype=np.uint64) >> np.uint64(6)
    return (hi * np.uint64(1 << 26) + lo).astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, c0, c1, c2, stream: int):
    """Uniform double for counter (c0, c1, c2, stream) under key(seed)."""
    k0, k1 = key_of(seed)
    w0, w1, _, _ = philox4x32(c0, c1, c2, stream, k0, k1)
    return to_unit_double(w0, w1)
