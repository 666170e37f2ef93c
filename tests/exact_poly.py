"""Exact power-series expansion of a degree-optimal scheme (test helper).

Every stored double is an integer multiple of 2^-S (S = 1100 covers the whole double
range), so each polynomial is kept as integer coefficients over a power of two and
products use Kronecker substitution (one big-integer product per polynomial
product).  The result is exact: the same rationals as Fraction arithmetic, much
faster for the degree-256 and degree-512 schemes."""

from fractions import Fraction


def _dyadic(v):
    """(numerator, exponent) with v = numerator / 2^exponent, exponent >= 0."""
    f = Fraction(v)
    e = f.denominator.bit_length() - 1
    assert f.denominator == 1 << e
    return f.numerator, e


class _Poly:
    def __init__(self, c, e):
        self.c = c      # integer coefficients
        self.e = e      # value = c / 2^e

    def at(self, e):
        return [x << (e - self.e) for x in self.c]


def _add(a, b):
    e = max(a.e, b.e)
    x, y = a.at(e), b.at(e)
    n = max(len(x), len(y))
    x += [0] * (n - len(x))
    y += [0] * (n - len(y))
    return _Poly([u + v for u, v in zip(x, y)], e)


def _scale(v, p):
    num, e = _dyadic(v)
    return _Poly([num * x for x in p.c], p.e + e)


def _mul(a, b):
    w = (max(abs(x).bit_length() for x in a.c) + max(abs(x).bit_length() for x in b.c)
         + min(len(a.c), len(b.c)).bit_length() + 2)
    pa = 0
    for c in reversed(a.c):
        pa = (pa << w) + c
    pb = 0
    for c in reversed(b.c):
        pb = (pb << w) + c
    prod = pa * pb
    out, mask, half = [], (1 << w) - 1, 1 << (w - 1)
    for _ in range(len(a.c) + len(b.c) - 1):
        v = prod & mask
        if v >= half:
            v -= 1 << w
        out.append(v)
        prod = (prod - v) >> w
    assert prod == 0
    return _Poly(out, a.e + b.e)


def expand_rows(k, h, g, y):
    """Monomial coefficients b_0..b_{2^k} (Fractions) of S = sum_q y_q P_q with
    P_1 = 1, P_2 = x, P_3 = x^2 and P_{j+2} = (sum_i h[j][i-2] P_i)(sum_i g[j][i-2] P_i),
    i = 2..j+1, j = 2..k (h[j], g[j] indexable by j)."""
    P = [None, _Poly([1], 0), _Poly([0, 1], 0), _Poly([0, 0, 1], 0)]
    for j in range(2, k + 1):
        left = _Poly([0], 0)
        right = _Poly([0], 0)
        for i in range(2, j + 2):
            left = _add(left, _scale(h[j][i - 2], P[i]))
            right = _add(right, _scale(g[j][i - 2], P[i]))
        P.append(_mul(left, right))
    z = _Poly([0], 0)
    for q in range(1, k + 3):
        z = _add(z, _scale(y[q - 1], P[q]))
    return [Fraction(c, 1 << z.e) for c in z.c]
