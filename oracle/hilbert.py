"""Exact integer tables for the moment-matching step (Sec. II-B).

* ``hilbert(N)``           the (N+1) x (N+1) Hilbert matrix, eq. (HM), as
                           Fractions: A[m][n] = 1/(m+n-1), 1 <= m, n <= N+1.
* ``hilbert_inverse(N)``   its inverse from the closed form of the Theorem,
                           eq. (inv), as Python integers.
* ``shifted_legendre(N)``  ell[k][r], the coefficient of t^r in the shifted
                           Legendre polynomial P_k(2t-1), which is
                           (-1)^(k+r) C(k,r) C(k+r,r).

The tables are pinned in tests: A * A^-1 = I exactly in rational arithmetic,
ell against numpy's Legendre-series conversion, and the factorisation
A^-1 = sum_k (2k+1) ell_k ell_k^T, which follows from the Gram matrix of the
monomials on [0,1] being A and the shifted Legendre polynomials being
orthogonal on [0,1] with squared norm 1/(2k+1).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb


def hilbert(N: int):
    """Eq. (HM): A[m-1][n-1] = 1/(m+n-1) for 1 <= m, n <= N+1."""
    return [[Fraction(1, m + n - 1) for n in range(1, N + 2)] for m in range(1, N + 2)]


def hilbert_inverse(N: int):
    """Eq. (inv): (A^-1)_{mn} = (-1)^(m+n) (m+n-1) C(N+m, N+1-n) C(N+n, N+1-m)
    C(m+n-2, m-1)^2 for 1 <= m, n <= N+1, returned 0-based as integers."""
    out = []
    for m in range(1, N + 2):
        row = []
        for n in range(1, N + 2):
            v = ((-1) ** (m + n) * (m + n - 1) * comb(N + m, N + 1 - n)
                 * comb(N + n, N + 1 - m) * comb(m + n - 2, m - 1) ** 2)
            row.append(v)
        out.append(row)
    return out


def shifted_legendre(N: int):
    """ell[k][r] = (-1)^(k+r) C(k,r) C(k+r,r): P_k(2t-1) = sum_r ell[k][r] t^r."""
    return [[((-1) ** (k + r)) * comb(k, r) * comb(k + r, r) if r <= k else 0
             for r in range(N + 1)] for k in range(N + 1)]
