"""GPU parity of the Cuhre path (Genz-Malik rule on region batches, top-K
selection, bisection, totals) against the CPU oracle.

The rule values are sums of about 2^d terms with weights of mixed sign, so
their agreement is bounded by the rounding of sum |w f|, which for the error
estimate |I7 - I5| is not small against the estimate itself.  Tolerances:
I7 within 1e-12 of |I7| plus 1e-15 of the region volume times sum |w|; the
error estimate within 1e-11 of itself plus 1e-13 of |I7|.  Full runs make the
same subdivisions (same neval and region count), so their totals agree
within 1e-12 (integral) and 1e-10 (error).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from closed_forms import exact

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import paper_1408_6373_amd as cc
    return cc


@pytest.fixture(scope="module")
def ctx(cc):
    c = cc.Context()
    yield c
    c.close()


def _regions(rng, d, n):
    lo = rng.random((n, d)) * 0.6
    w = rng.random((n, d)) * 0.4 + 1e-3
    return lo + w / 2, w / 2


@pytest.mark.parametrize("fam", range(5))
@pytest.mark.parametrize("d", [2, 3, 6, 9])
def test_rule_matches_oracle(cc, ctx, fam, d):
    rng = np.random.default_rng(100 * d + fam)
    a, u = W.genz_params(fam, d, 3)
    c, h = _regions(rng, d, 40)
    g = cc.cuhre_rule(ctx, fam, a, u, c, h)
    ig = O.genz(fam, a, u)
    for r in range(len(c)):
        o = O.gm_rule(ig, c[r], h[r])
        vol = np.prod(h[r]) * 2.0**d
        assert abs(g["I7"][r] - o["I7"]) <= 1e-12 * abs(o["I7"]) + 1e-15 * vol * 20
        assert abs(g["I5"][r] - o["I5"]) <= 1e-12 * abs(o["I5"]) + 1e-15 * vol * 60
        assert abs(g["err"][r] - o["err"]) <= 1e-11 * o["err"] + 1e-13 * abs(o["I7"]) + 1e-15 * vol * 60
        D = np.sort(o["dfour"])[::-1]
        if d == 1 or D[0] - D[1] > 1e-9 * D[0]:
            assert g["axis"][r] == o["axis"]


@pytest.mark.parametrize("fam,d", [(f, d) for d in (2, 5, 8) for f in range(5)] +
                         [(3, 3), (1, 4), (3, 6), (2, 7)])
def test_rule_lane_per_region_matches_oracle(cc, ctx, fam, d):
    # from 16384 regions on and up to d = 8 the rule runs one lane per region;
    # sampled regions against the oracle, to the same bars
    rng = np.random.default_rng(1000 + 10 * d + fam)
    a, u = W.genz_params(fam, d, 4)
    n = 16384 + 123
    c, h = _regions(rng, d, n)
    g = cc.cuhre_rule(ctx, fam, a, u, c, h)
    ig = O.genz(fam, a, u)
    for r in list(range(0, n, 997)) + [n - 1]:
        o = O.gm_rule(ig, c[r], h[r])
        vol = np.prod(h[r]) * 2.0**d
        assert abs(g["I7"][r] - o["I7"]) <= 1e-12 * abs(o["I7"]) + 1e-15 * vol * 20
        assert abs(g["I5"][r] - o["I5"]) <= 1e-12 * abs(o["I5"]) + 1e-15 * vol * 60
        assert abs(g["err"][r] - o["err"]) <= 1e-11 * o["err"] + 1e-13 * abs(o["I7"]) + 1e-15 * vol * 60
        D = np.sort(o["dfour"])[::-1]
        if D[0] - D[1] > 1e-9 * D[0]:
            assert g["axis"][r] == o["axis"]


def test_rule_d16(cc, ctx):
    rng = np.random.default_rng(16)
    a, u = W.genz_params(0, 16, 1)
    c, h = _regions(rng, 16, 3)
    g = cc.cuhre_rule(ctx, 0, a, u, c, h)
    for r in range(3):
        o = O.gm_rule(O.genz(0, a, u), c[r], h[r], nvec=70000)
        assert abs(g["I7"][r] - o["I7"]) <= 1e-12 * abs(o["I7"]) + 1e-17
        assert g["axis"][r] == o["axis"]


def _both(cc, ctx, fam, d, pseed=1, **kw):
    a, u = W.genz_params(fam, d, pseed)
    g = cc.cuhre(fam, a, u, ctx=ctx, **kw)
    o = O.cuhre(O.genz(fam, a, u), d, **kw)
    return g, o, (a, u)


def _assert_same_run(g, o):
    assert g["fail"] == o["fail"]
    assert g["neval"] == o["neval"] and g["nregions"] == o["nregions"]
    assert abs(g["integral"] - o["integral"]) <= 1e-12 * abs(o["integral"])
    assert abs(g["error"] - o["error"]) <= 1e-10 * o["error"] + 1e-14 * abs(o["integral"])


@pytest.mark.parametrize("fam", range(5))
@pytest.mark.parametrize("d", [2, 4])
def test_runs_match_oracle(cc, ctx, fam, d):
    g, o, (a, u) = _both(cc, ctx, fam, d, epsrel=1e-7, max_regions_per_batch=600,
                         maxeval=5 * 10**7)
    _assert_same_run(g, o)
    assert abs(g["integral"] - exact(fam, a, u)) <= max(g["error"], 1e-7 * abs(exact(fam, a, u)))


def test_corner_peak_d6_full_config(cc, ctx):
    # corner peak, d = 6, sum a = 5, batches of 10^5 regions, epsrel 1e-6
    g, o, (a, u) = _both(cc, ctx, 3, 6, epsrel=1e-6, max_regions_per_batch=10**5,
                         maxeval=10**9)
    _assert_same_run(g, o)
    assert g["fail"] == 0
    assert abs(g["integral"] / exact(3, a, u) - 1) < 1e-6


def test_maxeval_mineval_and_small_batches(cc, ctx):
    p = O.gm_npoints(3)
    for kw in (dict(epsrel=1e-30, maxeval=p * 15, max_regions_per_batch=4),
               dict(epsrel=1e-3, mineval=p * 200, max_regions_per_batch=2),
               dict(epsrel=1e-12, maxeval=10**5, max_regions_per_batch=10**5)):
        g, o, _ = _both(cc, ctx, 2, 3, pseed=5, **kw)
        _assert_same_run(g, o)
        assert g["neval"] <= kw.get("maxeval", 10**7)


def test_high_dimension_budget_limited(cc, ctx):
    g, o, _ = _both(cc, ctx, 0, 12, pseed=2, epsrel=1e-9, maxeval=3 * 10**6,
                    max_regions_per_batch=64)
    _assert_same_run(g, o)
    assert g["fail"] == 1


def test_constant_integrand_converges_at_root(cc, ctx):
    g = cc.cuhre(0, np.zeros(5), np.full(5, 0.5), ctx=ctx, epsrel=1e-12)
    assert g["fail"] == 0 and g["nregions"] == 1 and abs(g["integral"] - 1.0) < 1e-14
    assert g["error"] < 1e-13
