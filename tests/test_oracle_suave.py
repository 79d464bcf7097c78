"""Pins of the Suave oracle (subregion-adaptive Vegas; the Suave prototype of
Sect. 3.2.2, with the reading of its steps stated in oracle/suave.cpp).

Each pin ties the oracle to something outside its own code: the pinned
Vegas oracle (a root-only run is one Vegas iteration), exact invariants
(partition of the cube, the restriction estimator splitting the parent's
sum, exact scaling), a brute-force numpy run of one step with scipy's
incomplete gamma, the closed forms of the Genz families, and the selection
and cut rules observed run against run.
"""
import numpy as np
import pytest
from scipy.special import gammainc

import oracle as O
import workloads as W
from closed_forms import exact


def _root_only(fam, d, seed=3, nnew=3000, N=32):
    a, u = W.genz_params(fam, d, seed)
    s = O.suave(O.genz(fam, a, u), d, nnew=nnew, maxeval=3 * nnew - 1, nbins=N, seed=seed)
    v = O.vegas(O.genz(fam, a, u), d, nstart=nnew, maxeval=nnew, nbins=N, seed=seed)
    return s, v


@pytest.mark.parametrize("fam", range(5))
def test_root_only_run_is_one_vegas_iteration(fam):
    s, v = _root_only(fam, 4)
    assert s["nregions"] == 1 and s["neval"] == 3000 and s["fail"] == 1
    # the same combination of the one estimate
    assert s["integral"] == v["integral"] and s["error"] == v["error"]
    assert abs(s["integral"] - v["iter_I"][0]) <= 1e-15 * abs(v["iter_I"][0])
    assert s["prob"] == 0.0 and s["dof"] == 0
    assert np.array_equal(s["grid"][0].reshape(-1), v["grid"].reshape(-1))  # the refined root grid


@pytest.mark.parametrize("nsplit", [1, 3])
def test_regions_partition_the_cube(nsplit):
    d = 3
    a, u = W.genz_params(W.PRODUCT_PEAK, d, 5)
    r = O.suave(O.genz(W.PRODUCT_PEAK, a, u), d, nnew=1000, maxeval=60000, nbins=16,
                nsplit=nsplit)
    lo, hi = r["lo"], r["hi"]
    assert r["nregions"] == 1 + len(r["cut"]) > 10
    assert np.prod(hi - lo, axis=1).sum() == 1.0
    # dyadic bounds
    for b in (lo, hi):
        assert np.all(np.mod(b * 2.0 ** 30, 1.0) == 0.0)
    x = np.random.default_rng(0).random((20000, d))
    inside = ((x[:, None, :] >= lo[None]) & (x[:, None, :] < hi[None])).all(axis=2)
    assert np.all(inside.sum(axis=1) == 1)


def test_inherited_estimates_split_the_parent_sample():
    d, n = 4, 3000
    a, u = W.genz_params(W.GAUSSIAN, d, 6)
    s, _ = _root_only(W.GAUSSIAN, d, seed=6, nnew=n)
    r = O.suave(O.genz(W.GAUSSIAN, a, u), d, nnew=n, maxeval=3 * n, nbins=32, seed=6)
    assert r["nregions"] == 2 and r["neval"] == 3 * n
    c = r["cut"][0]
    assert r["hi"][0][c] == 0.5 and r["lo"][1][c] == 0.5
    assert np.all(r["inh_var"] > 0)
    # the two restriction estimators share out the parent's sum
    assert abs(r["inh_I"].sum() - s["integral"]) <= 1e-14 * s["integral"]
    # and each region's result lies between its two estimates' range
    assert r["dof"] == 2


@pytest.mark.parametrize("p", [1.0, 2.0, 25.0])
def test_cuts_follow_the_only_varying_axis(p):
    d = 4
    a = np.array([0.0, 0.0, 8.0, 0.0])
    u = np.array([0.5, 0.5, 0.3, 0.5])
    g = O.genz(W.GAUSSIAN, a, u)
    # frozen (uniform) grids: only the cuts along x_2 lower the fluctuation
    r = O.suave(g, d, nnew=2000, maxeval=40000, nbins=32, flatness=p, flags=O.FREEZE_GRID)
    assert len(r["cut"]) > 5 and np.all(r["cut"] == 2)
    others = [0, 1, 3]
    assert np.all(r["lo"][:, others] == 0.0) and np.all(r["hi"][:, others] == 1.0)
    # adapted grids flatten v along x_2, so later cuts may go elsewhere; the
    # first ones still follow x_2
    r = O.suave(g, d, nnew=2000, maxeval=40000, nbins=32, flatness=p)
    assert np.all(r["cut"][:2] == 2)


def test_one_step_by_brute_force():
    # frozen uniform grids, d = 2, one split, everything from the definitions
    d, N, n, seed, p = 2, 4, 64, 12, 2.0
    a, u = W.genz_params(W.C0, d, 12)
    r = O.suave(O.genz(W.C0, a, u), d, nnew=n, maxeval=3 * n, nbins=N, seed=seed,
                flatness=p, flags=O.FREEZE_GRID)
    uni = np.tile(np.arange(N + 1) / N, (d, 1))

    def sample(lo, hi, serial):
        pts = O.vegas_points(d, N, uni, seed, 0, serial, 0, n)
        x = pts["x"] * (hi - lo) + lo
        v = pts["w"] * np.prod(hi - lo) * O.genz_eval(W.C0, a, u, x)
        I = v.sum() / n
        return v, pts["x"] >= 0.5, I, max(0.0, (v * v).sum() / n - I * I) / (n - 1)

    v, side, I0, V0 = sample(np.zeros(d), np.ones(d), 0)
    scores = []
    for j in range(d):
        sc = 0.0
        for h in (False, True):
            vh = v[side[:, j] == h]
            if len(vh):
                sc += len(vh) / n * np.mean(np.abs(vh - vh.mean()) ** p) ** (1 / p)
        scores.append(sc)
    c = int(np.argmin(scores))
    assert r["cut"][0] == c
    I_tot, var_tot, chi2, dof = 0.0, 0.0, 0.0, 0
    for h in (0, 1):
        lo, hi = np.zeros(d), np.ones(d)
        (hi if h == 0 else lo)[c] = 0.5
        vh = np.where(side[:, c] == bool(h), v, 0.0)
        Ii = vh.sum() / n
        Vi = ((vh * vh).sum() / n - Ii * Ii) / (n - 1)
        _, _, In, Vn = sample(lo, hi, 1 + h)
        w = 1 / Vi + 1 / Vn
        Ir = (Ii / Vi + In / Vn) / w
        I_tot += Ir
        var_tot += 1 / w
        chi2 += (Ii - Ir) ** 2 / Vi + (In - Ir) ** 2 / Vn
        dof += 1
        assert np.array_equal(r["lo"][h], lo) and np.array_equal(r["hi"][h], hi)
        assert abs(r["I"][h] - Ir) <= 1e-13 * abs(Ir)
    assert np.all(r["grid"] == uni[None])
    assert abs(r["integral"] - I_tot) <= 1e-13 * abs(I_tot)
    assert abs(r["error"] - np.sqrt(var_tot)) <= 1e-12 * np.sqrt(var_tot)
    assert abs(r["prob"] - gammainc(dof / 2, chi2 / 2)) <= 1e-12


def test_constant_integrand_is_exact():
    d = 5
    r = O.suave(O.genz(W.GAUSSIAN, np.zeros(d), np.full(d, 0.5)), d, nnew=4000, epsrel=1e-3,
                maxeval=10**6)
    assert r["integral"] == 1.0 and r["error"] == 0.0
    assert r["fail"] == 0 and r["neval"] == 4000 and r["nregions"] == 1


def test_doubling_the_integrand_doubles_everything():
    d = 3
    a, u = W.genz_params(W.CORNER_PEAK, d, 7)

    def f(x):
        return (1.0 + x @ a) ** (-(d + 1))

    kw = dict(nnew=1500, maxeval=40000, nbins=16, nvec=512)
    r1 = O.suave(O.python_integrand(f), d, **kw)
    r2 = O.suave(O.python_integrand(lambda x: 2.0 * f(x)), d, **kw)
    assert r2["integral"] == 2 * r1["integral"] and r2["error"] == 2 * r1["error"]
    assert r2["prob"] == r1["prob"] and np.array_equal(r2["cut"], r1["cut"])
    assert np.array_equal(r2["I"], 2 * r1["I"]) and np.array_equal(r2["var"], 4 * r1["var"])


def test_budget_and_regions_split_per_step():
    d, n = 3, 500
    a, u = W.genz_params(W.OSCILLATORY, d, 8)
    r = O.suave(O.genz(W.OSCILLATORY, a, u), d, nnew=n, maxeval=11 * n, nbins=16, nsplit=4)
    # steps split 1, 2, 2 regions: neval 1, 3, 7, 11 (times nnew)
    assert r["neval"] == 11 * n and r["nregions"] == 6 and len(r["cut"]) == 5
    assert r["fail"] == 1
    r = O.suave(O.genz(W.OSCILLATORY, a, u), d, nnew=n, maxeval=n - 1)
    assert r["neval"] == 0 and r["nregions"] == 0 and r["fail"] == 1 and r["integral"] == 0


def test_each_step_splits_the_region_of_largest_variance():
    d, n = 3, 1000
    a, u = W.genz_params(W.PRODUCT_PEAK, d, 9)
    g = O.genz(W.PRODUCT_PEAK, a, u)
    prev = O.suave(g, d, nnew=n, maxeval=n, nbins=16)
    for s in range(1, 12):
        cur = O.suave(g, d, nnew=n, maxeval=(1 + 2 * s) * n, nbins=16)
        assert cur["nregions"] == prev["nregions"] + 1
        k = int(np.argmax(prev["var"]))
        # the lower child took position k, the upper one came last
        changed = [i for i in range(prev["nregions"])
                   if not (np.array_equal(cur["lo"][i], prev["lo"][i])
                           and np.array_equal(cur["hi"][i], prev["hi"][i]))]
        assert changed == [k]
        vol = np.prod(prev["hi"][k] - prev["lo"][k])
        assert np.prod(cur["hi"][k] - cur["lo"][k]) == vol / 2
        assert np.prod(cur["hi"][-1] - cur["lo"][-1]) == vol / 2
        prev = cur


@pytest.mark.parametrize("fam", range(5))
def test_converges_to_the_closed_form(fam):
    d = 4
    a, u = W.genz_params(fam, d, 13)
    ex = exact(fam, a, u)
    r = O.suave(O.genz(fam, a, u), d, nnew=2000, maxeval=2 * 10**6, epsrel=2e-3)
    assert r["fail"] == 0
    assert abs(r["integral"] - ex) <= 4 * r["error"]
    assert r["error"] <= 2e-3 * abs(r["integral"])


def test_error_estimate_is_honest_over_seeds():
    d = 3
    a, u = W.genz_params(W.PRODUCT_PEAK, d, 14)
    ex = exact(W.PRODUCT_PEAK, a, u)
    z = []
    for seed in range(40):
        r = O.suave(O.genz(W.PRODUCT_PEAK, a, u), d, nnew=1000, maxeval=30000, nbins=16,
                    seed=seed + 1)
        z.append((r["integral"] - ex) / r["error"])
    z = np.array(z)
    assert abs(z.mean()) < 0.5 and 0.6 < np.sqrt((z * z).mean()) < 1.5


def test_large_flatness_stays_finite():
    d = 4
    a, u = W.genz_params(W.GAUSSIAN, d, 15)
    r = O.suave(O.genz(W.GAUSSIAN, a, u), d, nnew=1000, maxeval=20000, flatness=700.0)
    assert np.isfinite(r["integral"]) and np.isfinite(r["error"]) and r["nregions"] > 5


def test_bad_arguments():
    g = O.genz(0, np.ones(3), np.full(3, 0.5))
    for kw in (dict(nnew=1), dict(flatness=0.0), dict(nsplit=0), dict(nbins=1),
               dict(flags=O.FP32_EVAL)):
        with pytest.raises(ValueError):
            O.suave(g, 3, **kw)
    with pytest.raises(ValueError):
        O.suave(g, 17)
