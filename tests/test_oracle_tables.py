"""Pins for the exact tables of the moment-matching step (Sec. II-B)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.hilbert import hilbert, hilbert_inverse, shifted_legendre

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_matrix(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("N", range(0, 12))
def test_inverse_times_hilbert_is_identity(N):
    A = hilbert(N)
    B = hilbert_inverse(N)
    n = N + 1
    for i in range(n):
        for j in range(n):
            s = sum(A[i][k] * B[k][j] for k in range(n))
            assert s == (1 if i == j else 0)


def test_inverse_n2_matches_textbook_value():
    assert hilbert_inverse(2) == _load_matrix("hilbert_inverse_n2.txt")
    A = hilbert(2)
    B = _load_matrix("hilbert_inverse_n2.txt")
    for i in range(3):
        for j in range(3):
            assert sum(A[i][k] * B[k][j] for k in range(3)) == (i == j)


@pytest.mark.parametrize("N", range(0, 12))
def test_shifted_legendre_matches_numpy(N):
    ell = shifted_legendre(N)
    for k in range(N + 1):
        P = np.polynomial.Legendre.basis(k, domain=[0, 1]).convert(kind=np.polynomial.Polynomial)
        coef = np.zeros(N + 1)
        coef[: len(P.coef)] = P.coef
        assert np.allclose(coef, ell[k], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("N", range(0, 12))
def test_inverse_factorises_through_legendre(N):
    # Gram matrix of 1, t, ..., t^N on [0,1] is the Hilbert matrix; the
    # shifted Legendre polynomials are orthogonal there with norm^2 1/(2k+1).
    ell = shifted_legendre(N)
    B = hilbert_inverse(N)
    for m in range(N + 1):
        for n in range(N + 1):
            assert sum((2 * k + 1) * ell[k][m] * ell[k][n] for k in range(N + 1)) == B[m][n]


def test_inverse_entries_fit_fp64_exactly():
    # Every entry up to N = 8 is an integer below 2^53, so the FP64 copy used
    # by the GPU library and the oracle is exact.
    for N in range(9):
        for row in hilbert_inverse(N):
            for v in row:
                assert abs(v) < 2 ** 53
                assert float(v) == v
