"""Philox4x32-10 counter-based generator and the TJM draw layout.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper draws a uniform epsilon for each jump process (Sec. "Stochastic jump
process") and, when a jump occurs, samples one jump operator from the
distribution Pi (Sec. "Stochastic jump process", Eq. for Pi_m).  It does not
say which generator.  Both implementations use Philox4x32-10 from
J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11 (2011): ten rounds of the S-box

    (c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2),
                         hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))

with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) before every round but the first.

Draw layout (a reading; the paper is silent): key = (seed & 0xffffffff,
seed >> 32); counter = (trajectory id, step k, branch, 0) with branch 0 for
the jump process of the sampling MPS at step k (k = 0 is F_0) and branch 1
for the sampling layer F_n applied at step k.  From the four output words,
eps = ((x0 >> 5) * 2^26 + (x1 >> 6)) * 2^-53 and r likewise from (x2, x3),
both in [0, 1).
"""

MASK32 = 0xFFFFFFFF
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85

BRANCH_MAIN = 0
BRANCH_SAMPLE = 1


def _round(c, k):
    p0 = M0 * c[0]
    p1 = M1 * c[2]
    hi0, lo0 = p0 >> 32, p0 & MASK32
    hi1, lo1 = p1 >> 32, p1 & MASK32
    return [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]


def philox4x32_10(counter, key):
    """Ten Philox rounds on a 4x32-bit counter with a 2x32-bit key."""
    c = [int(x) & MASK32 for x in counter]
    k = [int(x) & MASK32 for x in key]
    for i in range(10):
        if i:
            k = [(k[0] + W0) & MASK32, (k[1] + W1) & MASK32]
        c = _round(c, k)
    return c


def _u53(a, b):
    return ((a >> 5) * 67108864 + (b >> 6)) * (1.0 / 9007199254740992.0)


def draws(seed, traj, step, branch):
    """(eps, r): the two uniforms in [0,1) used by one jump process."""
    seed = int(seed)
    x = philox4x32_10([traj, step, branch, 0], [seed & MASK32, (seed >> 32) & MASK32])
    return _u53(x[0], x[1]), _u53(x[2], x[3])
