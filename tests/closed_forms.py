"""Closed-form integrals of the Genz families over [0,1]^d (test pins).

Each follows from integrating the family one coordinate at a time:
  Gaussian      prod sqrt(pi)/(2 a_i) [erf(a_i (1-u_i)) + erf(a_i u_i)]
  oscillatory   cos(2 pi u_1 + sum a / 2) prod 2 sin(a_i/2) / a_i
  product peak  prod a_i [atan(a_i (1-u_i)) + atan(a_i u_i)]
  corner peak   1/(d! prod a) sum_{S subset [d]} (-1)^|S| / (1 + sum_{i in S} a_i)
  C0            prod (2 - exp(-a_i u_i) - exp(-a_i (1-u_i))) / a_i
The corner-peak alternating sum loses digits as d grows, so it is evaluated
with 50-digit mpmath arithmetic.
"""
import itertools
import math

import mpmath
import numpy as np
from scipy.special import erf

GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, C0 = range(5)


def exact(family, a, u):
    a = np.asarray(a, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    d = len(a)
    if family == GAUSSIAN:
        return float(np.prod(np.sqrt(np.pi) / (2 * a) * (erf(a * (1 - u)) + erf(a * u))))
    if family == OSCILLATORY:
        return float(math.cos(2 * math.pi * u[0] + a.sum() / 2)
                     * np.prod(2 * np.sin(a / 2) / a))
    if family == PRODUCT_PEAK:
        return float(np.prod(a * (np.arctan(a * (1 - u)) + np.arctan(a * u))))
    if family == CORNER_PEAK:
        with mpmath.workdps(50):
            am = [mpmath.mpf(float(v)) for v in a]
            s = mpmath.mpf(0)
            for S in itertools.product((0, 1), repeat=d):
                sub = mpmath.mpf(1) + sum(am[i] for i in range(d) if S[i])
                s += (-1) ** sum(S) / sub
            den = mpmath.factorial(d)
            for v in am:
                den *= v
            return float(s / den)
    if family == C0:
        return float(np.prod((2 - np.exp(-a * u) - np.exp(-a * (1 - u))) / a))
    raise ValueError(family)
