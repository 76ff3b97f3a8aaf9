"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from its published definition.

The paper does not say how its random numbers are drawn; the sweep uses this
counter-based generator so that every decision's uniform is a pure function
of its position: key = (seed, walker_id), counter = (sweep, dir*M + slice,
site, purpose).  Pinned bit-for-bit against numpy.random.Philox in the tests.
"""
MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

# purpose tags (fourth counter word)
PURPOSE_INIT = 1   # initial field configuration
PURPOSE_MH = 2     # Metropolis uniform of one proposal
PURPOSE_HB = 3     # heat-bath uniform of one site in a force-bias block


def philox4x64_10(ctr, key):
    """Ten Philox rounds on a 4x64-bit counter with a 2x64-bit key."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def uniform(key, c0, c1, c2, purpose):
    """u in [0, 1): the top 53 bits of output word 0, times 2^-53."""
    w0 = philox4x64_10((c0, c1, c2, purpose), key)[0]
    return (w0 >> 11) * (1.0 / 9007199254740992.0)
