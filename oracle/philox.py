"""Counter-based Gaussian draws for the peeling probes (oracle; TEST
INFRASTRUCTURE ONLY).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 128-bit counter c = (c0, c1, c2, c3)
and a 64-bit key k = (k0, k1); ten rounds of

    (hi0, lo0) = mulhilo32(0xD2511F53, c0)
    (hi1, lo1) = mulhilo32(0xCD9E8D57, c2)
    c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)

with the key bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
rounds.  The four output words make two 53-bit uniforms in (0, 1),

    u1 = (((x0 << 32 | x1) >> 11) + 1/2) / 2^53,   u2 likewise from (x2, x3),

and one standard normal by the Box-Muller transform
sqrt(-2 log u1) cos(2 pi u2).

Counter layout of one probe entry (peeling level l, probe column j, DOF d in
tree order, operator stream s): c = (d, j, l, s), k = (seed mod 2^32, seed >> 32).
Rademacher entries of the Hutchinson estimator use c = (d, j, 0, 1) and the
lowest bit of the first output word: +1 when it is 0, -1 when it is 1.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 arrays; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32).astype(np.uint64)
    c1 = np.asarray(c1, dtype=np.uint32).astype(np.uint64)
    c2 = np.asarray(c2, dtype=np.uint32).astype(np.uint64)
    c3 = np.asarray(c3, dtype=np.uint32).astype(np.uint64)
    k0 = np.uint64(np.uint32(k0))
    k1 = np.uint64(np.uint32(k1))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for r in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
        if r < 9:
            k0 = (k0 + np.uint64(_W0)) & _MASK
            k1 = (k1 + np.uint64(_W1)) & _MASK
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def _uniform53(hi, lo):
    u = ((hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)) >> np.uint64(11)
    return (u.astype(np.float64) + 0.5) * (2.0 ** -53)


def normal(d, j, level, stream, seed):
    """Standard normal for counter (d, j, level, stream) under key seed."""
    seed = int(seed)
    x0, x1, x2, x3 = philox4x32_10(d, j, level, stream, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u1 = _uniform53(x0, x1)
    u2 = _uniform53(x2, x3)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def rademacher(d, j, seed):
    """+1 / -1 for counter (d, j, 0, 1) under key seed (lowest bit of word 0)."""
    seed = int(seed)
    x0, _, _, _ = philox4x32_10(d, j, 0, 1, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return np.where((x0 & np.uint32(1)) == 0, 1.0, -1.0)
