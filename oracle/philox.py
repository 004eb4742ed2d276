"""Philox4x32-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11 (the Philox-4x32 bijection with 10 rounds).

The random numbers the method draws (the random initial H of the experimental
setup, the Gaussian sketch Omega of Algorithm RRF, and the leverage-score
draws of the sampling matrix S) are taken from this generator.  The HIP
library implements the same published bijection independently; both sides
agree on the *stream layout* below, which is this project's convention:

  key     = (seed mod 2^32, seed div 2^32)
  counter = (block mod 2^32, block div 2^32, sub, tag)
  a block's four 32-bit words w0..w3 form two 64-bit values
      v0 = w0 | w1 << 32,   v1 = w2 | w3 << 32
  value e of a stream is v[e mod 2] of block e div 2.

Conversions: uniform u = (v >> 11) * 2^-53 in [0, 1) (exact in FP64);
Gaussian value e uses both words of block e:  u1, u2 from v0, v1 and
z = sqrt(-2 ln(1 - u1)) * cos(2 pi u2)  (Box-Muller; libm on each side, so the
Gaussians agree to a few ulps, not bitwise);  a draw in [0, W) is the high
64 bits of v * W (exact integer arithmetic).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)

TAG_H0 = 1
TAG_OMEGA = 2
TAG_SAMPLE = 3


def philox4x32_10(ctr, key):
    """Apply the Philox-4x32 bijection with 10 rounds.

    ctr: uint32 array of shape (N, 4); key: two uint32.  Returns (N, 4) uint32.
    One round maps (c0, c1, c2, c3) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is bumped by the Weyl constants between rounds.
    """
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy()
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def _blocks(seed, first_block, nblocks, sub, tag):
    b = np.arange(first_block, first_block + nblocks, dtype=np.uint64)
    ctr = np.empty((nblocks, 4), dtype=np.uint64)
    ctr[:, 0] = b & _MASK
    ctr[:, 1] = b >> np.uint64(32)
    ctr[:, 2] = np.uint64(sub)
    ctr[:, 3] = np.uint64(tag)
    seed = int(seed)
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).astype(np.uint64)
    v0 = w[:, 0] | (w[:, 1] << np.uint64(32))
    v1 = w[:, 2] | (w[:, 3] << np.uint64(32))
    return v0, v1


def u64_stream(seed, count, sub, tag):
    """Values 0..count-1 of the 64-bit stream (seed, sub, tag)."""
    nb = (count + 1) // 2
    v0, v1 = _blocks(seed, 0, nb, sub, tag)
    out = np.empty(2 * nb, dtype=np.uint64)
    out[0::2] = v0
    out[1::2] = v1
    return out[:count]


def uniform(seed, count, sub, tag):
    """Uniform FP64 numbers in [0, 1): (v >> 11) * 2^-53."""
    v = u64_stream(seed, count, sub, tag)
    return (v >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian(seed, count, sub, tag):
    """Standard normal FP64 numbers by Box-Muller, one per block."""
    v0, v1 = _blocks(seed, 0, count, sub, tag)
    u1 = (v0 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    u2 = (v1 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)


def draws(seed, count, sub, tag, bound):
    """Integers in [0, bound): high 64 bits of v * bound (exact)."""
    v = u64_stream(seed, count, sub, tag)
    bound = int(bound)
    return np.array([(int(x) * bound) >> 64 for x in v], dtype=np.uint64)
