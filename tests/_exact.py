"""Exact rational checker for tiny images (pins the FP64 oracle).

Written independently of the oracle, in the paper's own 1-based indexing:
D_{s,t} is enumerated literally as the (i', j') with 1 <= i' <= m,
1 <= j' <= n, 1 <= i'+s <= m, 1 <= j'+t <= n (sec. 2, overlap set), and f is
the mean of (a_{i+s,j+t} - b_{i,j})^2 over it as a ``Fraction``.
Pure Python loops: use only on images of a few pixels a side.
"""
from fractions import Fraction


def overlap_set(m, n, s, t):
    return [(i, j) for i in range(1, m + 1) for j in range(1, n + 1)
            if 1 <= i + s <= m and 1 <= j + t <= n]


def f_exact(a, b, s, t):
    """a, b: lists of lists (0-based storage) of ints; returns Fraction or None if D is empty."""
    m, n = len(a), len(a[0])
    D = overlap_set(m, n, s, t)
    if not D:
        return None
    tot = Fraction(0)
    for (i, j) in D:
        d = Fraction(a[i + s - 1][j + t - 1]) - Fraction(b[i - 1][j - 1])
        tot += d * d
    return tot / len(D)
