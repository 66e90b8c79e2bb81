"""The range stage's erfcx (Weideman's rational expansion on the real axis,
coefficients in csrc/erfcx_weideman.h) against SciPy's erfcx and 40-digit
values. Host logic only: the stored coefficients are read from the header
and the expansion is evaluated in FP64 in the kernel's order."""
import os
import re

import numpy as np
import pytest

from paper_1811_02308_amd import gen_erfcx

HDR = os.path.join(os.path.dirname(gen_erfcx.__file__), "csrc", "erfcx_weideman.h")


def header_coefficients():
    text = open(HDR).read()
    L = float.fromhex(re.search(r"kErfcxL = ([0-9a-fx.p+-]+);", text).group(1))
    body = text[text.index("kErfcxA[kErfcxTerms] = {"):]
    a = [float.fromhex(m) for m in re.findall(r"^\s+(-?0x[0-9a-f.]+p[+-]\d+),", body, re.M)]
    return L, a


def test_header_matches_generator():
    L, a = header_coefficients()
    L2, a2 = gen_erfcx.coefficients()
    assert len(a) == gen_erfcx.TERMS == len(a2)
    assert L == L2
    assert np.max(np.abs(np.array(a) - np.array(a2))) <= 1e-15


def test_against_scipy():
    special = pytest.importorskip("scipy.special")
    L, a = header_coefficients()
    x = np.concatenate([np.linspace(0, 1, 5001), np.linspace(1, 8, 5001), np.geomspace(8, 1e12, 400)])
    got = gen_erfcx.evaluate(x, L, a)
    ref = special.erfcx(x)
    assert np.max(np.abs(got - ref) / ref) < 3e-15


def test_against_40_digits():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    L, a = header_coefficients()
    x = np.array([0.0, 1e-8, 0.017, 0.074, 0.5, 1.0, 2.0, 3.3, 5.045, 7.5, 12.0, 30.0, 100.0])
    ref = np.array([float(mp.exp(mp.mpf(v) ** 2) * mp.erfc(mp.mpf(v))) for v in x])
    got = gen_erfcx.evaluate(x, L, a)
    assert np.max(np.abs(got - ref) / ref) < 1.3e-15
    # the limit 1 / (sqrt(pi) x)
    big = gen_erfcx.evaluate(np.array([1e150]), L, a)[0]
    assert abs(big * 1e150 * np.sqrt(np.pi) - 1.0) < 1e-15
