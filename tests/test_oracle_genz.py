"""Pins of the oracle's Genz integrands: tensor-product Gauss-Legendre
quadrature at d=2 of the oracle's own values must reproduce the closed-form
integral of each family (a dropped term, wrong sign or swapped parameter in
the oracle's formula fails this)."""
import numpy as np
import pytest

import oracle as O
from closed_forms import exact
import workloads as W


def _gl_2d(fam, a, u, prec, n=96):
    # split each axis at u_i (C0 has a kink there) and use n GL nodes per piece
    x, w = np.polynomial.legendre.leggauss(n)
    nodes, weights = [], []
    for j in range(2):
        cuts = [0.0, 1.0] if fam != O.C0 else [0.0, u[j], 1.0]
        xs, ws = [], []
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            xs.append(lo + (hi - lo) * (x + 1) / 2)
            ws.append((hi - lo) / 2 * w)
        nodes.append(np.concatenate(xs))
        weights.append(np.concatenate(ws))
    X0, X1 = np.meshgrid(nodes[0], nodes[1], indexing="ij")
    W2 = np.outer(weights[0], weights[1])
    pts = np.stack([X0.ravel(), X1.ravel()], axis=1)
    f = O.genz_eval(fam, a, u, pts, precision=prec)
    return float((W2.ravel() * f).sum())


@pytest.mark.parametrize("fam", range(5))
def test_gauss_legendre_matches_closed_form_fp64(fam):
    for seed in (1, 2):
        a, u = W.genz_params(fam, 2, seed)
        assert abs(_gl_2d(fam, a, u, O.FP64) / exact(fam, a, u) - 1) < 1e-10


@pytest.mark.parametrize("fam", range(5))
def test_gauss_legendre_matches_closed_form_fp32(fam):
    a, u = W.genz_params(fam, 2, 3)
    assert abs(_gl_2d(fam, a, u, O.FP32_EVAL) / exact(fam, a, u) - 1) < 2e-6


def test_special_values():
    # values fixed by the definitions: at x = u the Gaussian, product peak and
    # C0 reach their maxima 1, prod a_i^2 and 1; the corner peak is 1 at 0
    a = np.array([0.5, 1.5, 2.0])
    u = np.array([0.2, 0.4, 0.9])
    assert O.genz_eval(O.GAUSSIAN, a, u, u)[0] == 1.0
    assert O.genz_eval(O.C0, a, u, u)[0] == 1.0
    assert abs(O.genz_eval(O.PRODUCT_PEAK, a, u, u)[0] / np.prod(a**2) - 1) < 1e-15
    assert O.genz_eval(O.CORNER_PEAK, a, u, np.zeros(3))[0] == 1.0
    # oscillatory at x = 0 is cos(2 pi u_1)
    assert abs(O.genz_eval(O.OSCILLATORY, a, u, np.zeros(3))[0]
               - np.cos(2 * np.pi * u[0])) < 1e-15
