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
a draw in [0, W) is the high 64 bits of v * W (exact integer arithmetic);
Gaussian value e uses both words of block e (Box-Muller):
z = sqrt(-2 ln(1 - u1)) * cos(2 pi u2), u1, u2 from v0, v1, with the logarithm
and cosine below (`log_unit`, `cos_turn`) instead of a math library, so that
every value is fixed bit for bit by this definition: each step is one
correctly rounded FP64 operation (+, -, *, /, sqrt) in the order written, and
numpy performs exactly those (it fuses no multiply-add).
"""
import math
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


# ln 2 = LN2_HI + LN2_LO: LN2_HI keeps 32 fraction bits, so e * LN2_HI is
# exact for the exponents that occur (Cody and Waite's split of the constant);
# both are derived here from a 60-digit ln 2.
def _ln2_split():
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    hi = Decimal(int(ln2 * (1 << 32))) / Decimal(1 << 32)
    return float(hi), float(ln2 - hi)


LN2_HI, LN2_LO = _ln2_split()
SQRT_HALF = math.sqrt(0.5)
HALF_PI = math.pi / 2.0      # the double nearest pi/2 (math.pi is the double nearest pi)


def log_unit(a):
    """ln x for x = (2^53 - a) 2^-53 in (0, 1], a: uint64 array of 53-bit integers.

    x = m 2^e with m in [sqrt(1/2), sqrt(2)); with s = (m - 1)/(m + 1),
    ln m = 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ...), summed by Horner up to
    the s^22/23 term (|s| <= 0.1716, so the rest is below 2^-62 relative);
    ln x = e LN2_HI + (e LN2_LO + ln m).
    """
    x = ((np.uint64(1) << np.uint64(53)) - np.asarray(a, dtype=np.uint64)).astype(np.float64) * 2.0 ** -53
    m, e = np.frexp(x)                       # m in [1/2, 1), exact
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = np.full_like(s, 1.0 / 23.0)
    for j in range(10, -1, -1):
        p = 1.0 / float(2 * j + 1) + z * p
    lnm = (s + s) * p
    return e * LN2_HI + (e * LN2_LO + lnm)


def cos_turn(b):
    """cos(2 pi b 2^-53) for b: uint64 array of 53-bit integers.

    The angle is q quarter turns plus theta = f pi/2 with q the nearest
    integer to b / 2^51 and f = (b - q 2^51) 2^-51 in [-1/2, 1/2] (both exact);
    sin and cos of theta by their Taylor series up to theta^17/17! and
    theta^18/18! (the rest is below 2^-62 relative for |theta| <= pi/4), each
    coefficient the double nearest +-1/n!; q mod 4 = 0..3 selects cos, -sin,
    -cos, sin.
    """
    b = np.asarray(b, dtype=np.uint64)
    q = (b + (np.uint64(1) << np.uint64(50))) >> np.uint64(51)
    f = (b.astype(np.int64) - (q << np.uint64(51)).astype(np.int64)).astype(np.float64) * 2.0 ** -51
    theta = f * HALF_PI
    t = theta * theta
    S = np.full_like(t, 1.0 / float(math.factorial(17)))
    for j in range(7, 0, -1):
        S = (-1.0) ** j / float(math.factorial(2 * j + 1)) + t * S
    C = np.full_like(t, -1.0 / float(math.factorial(18)))
    for j in range(8, 0, -1):
        C = (-1.0) ** j / float(math.factorial(2 * j)) + t * C
    sn = theta + (theta * t) * S
    cs = 1.0 + t * C
    qm = (q & np.uint64(3)).astype(np.int64)
    return np.choose(qm, [cs, -sn, -cs, sn])


def gaussian(seed, count, sub, tag):
    """Standard normal FP64 numbers by Box-Muller, one per block:
    sqrt(-2 ln(1 - u1)) * cos(2 pi u2) with the log and cosine above."""
    v0, v1 = _blocks(seed, 0, count, sub, tag)
    r2 = -2.0 * log_unit(v0 >> np.uint64(11))
    return np.sqrt(r2) * cos_turn(v1 >> np.uint64(11))


def draws(seed, count, sub, tag, bound):
    """Integers in [0, bound): high 64 bits of v * bound (exact)."""
    v = u64_stream(seed, count, sub, tag)
    bound = int(bound)
    return np.array([(int(x) * bound) >> 64 for x in v], dtype=np.uint64)
