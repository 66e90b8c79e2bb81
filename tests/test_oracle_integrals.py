"""Pins for the range integrals of eq. (integrals) (Sec. II-C)."""
import mpmath as mp
import numpy as np
import pytest

from oracle.hilbert import shifted_legendre
from oracle.integrals import I_mpmath, I_paper, I_quadrature, J_quadrature


@pytest.mark.parametrize("lam,t0", [(0.7, 0.3), (3.0, 0.5), (25.0, 0.9), (400.0, 0.1)])
def test_paper_formulas_match_definition(lam, t0):
    # eqs. (I_0), (I_1), (F_forward) against 50-digit quadrature of the definition
    K = 6
    ref = [float(v) for v in I_mpmath(lam, t0, K)]
    got = I_paper(np.array([lam]), np.array([t0]), K)[0]
    assert np.allclose(got, ref, rtol=1e-9, atol=0)


def test_forward_recursion_identity_high_precision():
    # 2 lam I_k = 2 lam t0 I_{k-1} + (k-1) I_{k-2} - exp(-lam (1-t0)^2)
    with mp.workdps(50):
        for lam, t0 in [(0.01, 0.4), (2.0, -0.7), (50.0, 1.6)]:
            I = I_mpmath(lam, t0, 7, dps=50)
            for k in range(2, 8):
                lhs = 2 * mp.mpf(lam) * I[k]
                rhs = (2 * mp.mpf(lam) * mp.mpf(t0) * I[k - 1] + (k - 1) * I[k - 2]
                       - mp.e ** (-mp.mpf(lam) * (1 - mp.mpf(t0)) ** 2))
                assert abs(lhs - rhs) < mp.mpf(10) ** -40 * (1 + abs(lhs))


GRID = [(lam, t0) for lam in (0.0, 1e-6, 0.03, 0.9, 7.0, 60.0, 900.0, 2e4)
        for t0 in (-6.0, -0.8, 0.0, 0.25, 0.5, 0.99, 1.0, 1.7, 9.0)]


@pytest.mark.parametrize("lam,t0", GRID)
def test_quadrature_matches_mpmath(lam, t0):
    K = 9
    I, ls = I_quadrature(np.array([lam]), np.array([t0]), K)
    with mp.workdps(50):
        ref = I_mpmath(lam, t0, K, dps=50) if lam > 0 else [mp.mpf(1) / (k + 1) for k in range(K + 1)]
        scale = mp.e ** (mp.mpf(lam) * (mp.mpf(t0) - min(max(t0, 0.0), 1.0)) ** 2)
        ref = [float(v * scale) for v in ref]
    # every I_k relative to the scaled I_0 (the size that matters in T1/T2)
    # (rounding of an exponent of size up to 80 bounds the relative accuracy
    # at about 80 ulp)
    assert np.all(np.abs(I[0] - ref) <= 1e-13 * ref[0] + 1e-300)


def test_legendre_integrals_are_ell_combinations():
    N = 8
    lam = np.array([0.2, 5.0, 120.0])
    t0 = np.array([0.4, -0.3, 1.2])
    I, ls = I_quadrature(lam, t0, N + 1)
    J, Jt, ls2 = J_quadrature(lam, t0, N)
    ell = np.array(shifted_legendre(N), dtype=float)
    assert np.allclose(ls, ls2)
    assert np.allclose(J, I[:, :-1] @ ell.T, rtol=1e-9, atol=1e-12 * I[:, :1])
    assert np.allclose(Jt, I[:, 1:] @ ell.T, rtol=1e-9, atol=1e-12 * I[:, :1])
