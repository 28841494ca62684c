"""Oracle code construction -- TEST INFRASTRUCTURE ONLY (never product code).

The paper states only that the k reliable positions carry information and
the n-k unreliable ones are frozen to 0 (Section II); it gives no
construction method.  The construction used throughout is the Bhattacharyya
recursion in natural order for G = F^{(x)m}:

    z_{2i} = 2 z_i - z_i^2,   z_{2i+1} = z_i^2,   z_0 = exp(-R * Eb/N0)

with R = K/N and the design Eb/N0 as a linear ratio; the N-K positions with
the largest z are frozen, ties freezing the lower index first.

It is written out here in decimal arithmetic with 80 significant digits and
an unbounded exponent range.  Alongside z the recursion carries w = 1 - z,
using only the exact identities 2z - z^2 = z(1 + w), 1 - (2z - z^2) = w^2
and 1 - z^2 = w(1 + z), so that neither quantity loses relative precision
when the other approaches 1 (at N = 16384, w reaches about 1e-6600).
Positions are ranked by logit = ln z - ln w, a monotone function of z.
"""

from decimal import Decimal, localcontext

PREC = 80


def bhattacharyya(m, z0):
    """(z, w) lists of length 2^m from the recursion, as Decimals.
    ``z0`` may be a Decimal, a Fraction-free string or a float."""
    with localcontext() as ctx:
        ctx.prec = PREC
        ctx.Emin = -999999999
        ctx.Emax = 999999999
        z = [Decimal(z0) if not isinstance(z0, Decimal) else z0]
        w = [Decimal(1) - z[0]]
        one = Decimal(1)
        for _ in range(m):
            nz, nw = [], []
            for zi, wi in zip(z, w):
                nz.append(zi * (one + wi))   # index 2i:   2z - z^2
                nw.append(wi * wi)
                nz.append(zi * zi)           # index 2i+1: z^2
                nw.append(wi * (one + zi))
            z, w = nz, nw
        return z, w


def design_z0(N, K, design_ebn0_db):
    """z0 = exp(-R * 10^(design/10)) with R = K/N, in decimal."""
    with localcontext() as ctx:
        ctx.prec = PREC
        ebn0 = Decimal(10) ** (Decimal(repr(float(design_ebn0_db))) / 10)
        return (-(Decimal(K) / Decimal(N)) * ebn0).exp()


def logits(m, z0):
    """ln z - ln w for every position."""
    z, w = bhattacharyya(m, z0)
    with localcontext() as ctx:
        ctx.prec = PREC
        ctx.Emin = -999999999
        ctx.Emax = 999999999
        return [zi.ln() - wi.ln() for zi, wi in zip(z, w)]


def construct(N, K, design_ebn0_db=0.0):
    """Frozen mask (list of N ints, 1 = frozen) and the logit gap at the
    frozen/information boundary (None when K is 0 or N)."""
    m = N.bit_length() - 1
    assert N == 1 << m and 0 <= K <= N
    lg = logits(m, design_z0(N, K, design_ebn0_db))
    order = sorted(range(N), key=lambda i: (-lg[i], i))
    frozen = [0] * N
    for i in order[:N - K]:
        frozen[i] = 1
    gap = None
    if 0 < K < N:
        gap = float(lg[order[N - K - 1]] - lg[order[N - K]])
    return frozen, gap
