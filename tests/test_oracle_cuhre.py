"""Pins of the oracle's Cuhre: exactness of the Genz-Malik degree-7 rule on
every monomial of degree <= 7 (degree 5 for the embedded rule), failure at
degree 8, the fourth-difference split axis, closed-form integrals, and the
interface semantics (nvec, -999 abort, maxeval, mineval)."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from closed_forms import exact
import workloads as W


def _monomial(powers):
    p = np.array(powers)
    return O.python_integrand(lambda x: np.prod(x ** p, axis=1))


def _exact_monomial(powers, c, h):
    # integral over prod [c_i - h_i, c_i + h_i] of prod x_i^p_i
    v = 1.0
    for p, ci, hi in zip(powers, c, h):
        a, b = ci - hi, ci + hi
        v *= (b ** (p + 1) - a ** (p + 1)) / (p + 1)
    return v


def _powers(d, deg):
    for tot in range(deg + 1):
        for comb in itertools.combinations_with_replacement(range(d), tot):
            p = [0] * d
            for i in comb:
                p[i] += 1
            yield p


@pytest.mark.parametrize("d", [2, 3, 4, 6])
def test_degree7_exact_degree5_embedded(d):
    # on the symmetric cube [-1,1]^d and on an off-centre box
    for c, h in ((np.zeros(d), np.ones(d)), (np.linspace(0.3, 0.6, d), np.linspace(0.1, 0.25, d))):
        seen = set()
        for p in _powers(d, 7):
            key = tuple(p)
            if key in seen:
                continue
            seen.add(key)
            r = O.gm_rule(_monomial(p), c, h)
            ex = _exact_monomial(p, c, h)
            scale = max(1.0, abs(ex)) * np.prod(2 * h)
            assert abs(r["I7"] - ex) < 1e-13 * scale, (p, r["I7"], ex)
            if sum(p) <= 5:
                assert abs(r["I5"] - ex) < 1e-13 * scale, (p, r["I5"], ex)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_not_exact_at_degree8(d):
    c, h = np.zeros(d), np.ones(d)
    bad = 0
    for p in ([8] + [0] * (d - 1), [4, 4] + [0] * (d - 2), [6, 2] + [0] * (d - 2)):
        r = O.gm_rule(_monomial(p), c, h)
        if abs(r["I7"] - _exact_monomial(p, c, h)) > 1e-8:
            bad += 1
    assert bad >= 1
    # and the degree-5 rule is not exact at degree 6
    p = [6] + [0] * (d - 1)
    r = O.gm_rule(_monomial(p), c, h)
    assert abs(r["I5"] - _exact_monomial(p, c, h)) > 1e-8


def test_fourth_difference_split_axis():
    d = 5
    c, h = np.full(d, 0.5), np.full(d, 0.5)
    # cubics have zero fourth difference on every axis
    r = O.gm_rule(O.python_integrand(lambda x: x[:, 0] ** 3 + 2 * x[:, 2] ** 2 * x[:, 1]), c, h)
    assert np.max(r["dfour"]) < 1e-13
    for k in range(d):
        r = O.gm_rule(O.python_integrand(lambda x, k=k: x[:, k] ** 4), c, h)
        assert r["axis"] == k and r["dfour"][k] > 1e-3
    # a tie resolves to the lowest axis
    r = O.gm_rule(O.python_integrand(lambda x: x[:, 1] ** 4 + x[:, 3] ** 4), c, h)
    assert r["axis"] == 1


def test_constant_has_zero_error():
    for d in (2, 7, 12):
        r = O.gm_rule(O.python_integrand(lambda x: np.full(len(x), 3.0)),
                      np.full(d, 0.5), np.full(d, 0.5))
        assert abs(r["I7"] - 3.0) < 1e-13 and r["err"] <= 1e-14 * 3 * 4 ** d / 2 ** d


def test_npoints():
    for d in range(2, 17):
        assert O.gm_npoints(d) == 2 ** d + 2 * d * d + 2 * d + 1
    assert O.gm_npoints(6) == 149


@pytest.mark.parametrize("fam", range(5))
def test_closed_forms_reach_requested_accuracy(fam):
    for d, seed in ((2, 1), (4, 2)):
        a, u = W.genz_params(fam, d, seed)
        r = O.cuhre(O.genz(fam, a, u), d, epsrel=1e-6, maxeval=5 * 10**7,
                    max_regions_per_batch=2000)
        assert r["fail"] == 0
        ex = exact(fam, a, u)
        assert abs(r["integral"] - ex) <= max(r["error"], 1e-6 * abs(ex)), (fam, d)


def test_corner_peak_d6_config():
    a, u = W.genz_params(3, 6, 1)
    r = O.cuhre(O.genz(3, a, u), 6, epsrel=1e-6, maxeval=10**9, max_regions_per_batch=10**4)
    assert r["fail"] == 0 and abs(r["integral"] / exact(3, a, u) - 1) < 1e-6


def test_region_count_exact_sequence():
    # with B = 4 the batches split 1, 2, 2, 2, ... regions: leaves 1, 2, 4, 6, 8
    a, u = W.genz_params(0, 2, 1)
    p = O.gm_npoints(2)
    for nb in range(0, 5):
        budget = p * (1 + 2 * sum(min(2, 1 if b == 0 else 2) for b in range(nb)))
        r = O.cuhre(O.genz(0, a, u), 2, epsrel=1e-30, maxeval=budget, max_regions_per_batch=4)
        assert r["n_batches"] == nb and r["neval"] == budget
        assert r["nregions"] == 1 + sum(min(2, 1 if b == 0 else 2) for b in range(nb))


def test_nvec_does_not_change_results():
    a, u = W.genz_params(2, 3, 1)
    base = None
    for nvec in (1, 7, 1000):
        r = O.cuhre(O.genz(2, a, u), 3, epsrel=1e-5, nvec=nvec, max_regions_per_batch=100)
        key = (r["integral"], r["error"], r["nregions"], r["neval"])
        base = base or key
        assert key == base


def test_abort_and_maxeval():
    calls = []

    def f(x):
        calls.append(1)
        return -999 if len(calls) == 5 else np.ones(len(x))

    r = O.cuhre(O.python_integrand(f), 2, epsrel=1e-30, nvec=4)
    assert r["fail"] == -99
    a, u = W.genz_params(0, 4, 1)
    r = O.cuhre(O.genz(0, a, u), 4, epsrel=1e-12, maxeval=10**5)
    assert r["fail"] == 1 and r["neval"] <= 10**5


def test_mineval_forces_more_work():
    a, u = W.genz_params(0, 2, 1)
    r = O.cuhre(O.genz(0, a, u), 2, epsrel=1e-3)
    r2 = O.cuhre(O.genz(0, a, u), 2, epsrel=1e-3, mineval=r["neval"] * 4)
    assert r2["neval"] >= r["neval"] * 4 and r2["fail"] == 0
