"""Pins of the oracle's lower regularized incomplete gamma function (the
chi^2 probability): closed forms at dof 1 and 2, and scipy.special.gammainc."""
import math

import numpy as np
from scipy.special import gammainc

import oracle as O


def test_dof1_dof2_closed_forms():
    for chi2 in (1e-6, 0.3, 1.0, 4.0, 17.0, 60.0):
        assert abs(O.gammainc_lower(0.5, chi2 / 2) - math.erf(math.sqrt(chi2 / 2))) < 1e-14
        assert abs(O.gammainc_lower(1.0, chi2 / 2) - (-math.expm1(-chi2 / 2))) < 1e-14


def test_against_scipy():
    rng = np.random.default_rng(0)
    for _ in range(300):
        a = rng.uniform(0.5, 40)
        x = rng.uniform(0, 3 * a)
        assert abs(O.gammainc_lower(a, x) - gammainc(a, x)) < 1e-13


def test_edges():
    assert O.gammainc_lower(2.0, 0.0) == 0.0
    assert O.gammainc_lower(2.0, float("inf")) == 1.0
