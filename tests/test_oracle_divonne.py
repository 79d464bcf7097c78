"""Pins of the Divonne partitioning-phase oracle (Sect. 2.2: regions of
about equal Spread(r) = 1/2 Vol(r) (sup f - inf f), extrema by numerical
search; the search and the cut are the readings stated in
oracle/divonne.cpp).

Outside anchors: closed-form extrema of monotone and separable unimodal
integrands (reached exactly at corners), the search sample's extrema
recomputed from the Philox known-answer generator and the integrand,
exact partition invariants, exact scaling, the evaluation count, and the
selection and cut rules observed run against run.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def test_corner_peak_extrema_are_the_corners():
    # (1 + a.x)^-(d+1) decreases in every coordinate: max at lo, min at hi
    d = 4
    a, u = W.genz_params(W.CORNER_PEAK, d, 2)
    r = O.divonne_partition(O.genz(W.CORNER_PEAK, a, u), d, nsearch=64, niter=64,
                            maxregions=24, nsplit=3)
    assert r["nregions"] == 24
    assert np.array_equal(r["xmax"], r["lo"]) and np.array_equal(r["xmin"], r["hi"])
    fl = (1.0 + r["lo"] @ a) ** -(d + 1)
    fh = (1.0 + r["hi"] @ a) ** -(d + 1)
    assert np.allclose(r["fmax"], fl, rtol=1e-14, atol=0)
    assert np.allclose(r["fmin"], fh, rtol=1e-14, atol=0)
    vol = np.prod(r["hi"] - r["lo"], axis=1)
    assert np.allclose(r["spread"], 0.5 * vol * (fl - fh), rtol=1e-13, atol=0)


def test_gaussian_extrema():
    # exp(-sum a^2 (x - u)^2): max at u, min at the corner farthest from u
    d = 3
    a = np.array([4.0, 5.0, 6.0])
    u = np.array([0.3, 0.55, 0.8])
    r = O.divonne_partition(O.genz(W.GAUSSIAN, a, u), d, nsearch=128, niter=80, maxregions=1)
    # at the peak f = 1 - a^2 delta^2: FP64 separates positions only to about
    # sqrt(eps)/a, so the value is held tight and the position to 1e-7
    assert np.max(np.abs(r["xmax"][0] - u)) < 1e-7 and r["fmax"][0] >= 1 - 1e-15
    far = np.where(u < 0.5, 1.0, 0.0)
    assert np.array_equal(r["xmin"][0], far)
    assert abs(r["fmin"][0] - np.exp(-np.sum(a * a * (far - u) ** 2))) <= 1e-15


def test_search_sample_extrema_without_local_search():
    # niter = 0: the extrema of the nsearch Philox points, recomputed here
    d, n, seed = 5, 40, 77
    a, u = W.genz_params(W.C0, d, 3)
    r = O.divonne_partition(O.genz(W.C0, a, u), d, seed=seed, stream_id=3, nsearch=n, niter=0,
                            maxregions=1)
    pts = np.zeros((n, d))
    for i in range(n):
        words = O.philox([i, 0, 3, 0], [seed, 0]) + O.philox([i, 1, 3, 0], [seed, 0])
        pts[i] = np.array(words[:d], dtype=np.float64) * 2.0 ** -32 + 2.0 ** -33
    f = O.genz_eval(W.C0, a, u, pts)
    assert r["fmax"][0] == f.max() and r["fmin"][0] == f.min()
    assert np.array_equal(r["xmax"][0], pts[np.argmax(f)])
    assert np.array_equal(r["xmin"][0], pts[np.argmin(f)])
    assert r["neval"] == n


def test_local_search_improves_and_evaluations_add_up():
    d = 4
    a, u = W.genz_params(W.PRODUCT_PEAK, d, 4)
    g = O.genz(W.PRODUCT_PEAK, a, u)
    r0 = O.divonne_partition(g, d, nsearch=50, niter=0, maxregions=1)
    r = O.divonne_partition(g, d, nsearch=50, niter=20, maxregions=1)
    assert r["fmax"][0] >= r0["fmax"][0] and r["fmin"][0] <= r0["fmin"][0]
    assert r["neval"] == 50 + 4 * d * 20
    rs = O.divonne_partition(g, d, nsearch=50, niter=20, maxregions=9, nsplit=2)
    # the root's search, two per split, and d probes per split
    ns = len(rs["cut"])
    assert rs["neval"] == (1 + 2 * ns) * (50 + 4 * d * 20) + d * ns


@pytest.mark.parametrize("nsplit", [1, 4])
def test_regions_partition_the_cube(nsplit):
    d = 3
    a, u = W.genz_params(W.OSCILLATORY, d, 5)
    r = O.divonne_partition(O.genz(W.OSCILLATORY, a, u), d, nsearch=64, niter=8,
                            maxregions=40, nsplit=nsplit)
    lo, hi = r["lo"], r["hi"]
    assert r["nregions"] == 40 == 1 + len(r["cut"])
    assert np.prod(hi - lo, axis=1).sum() == 1.0
    for b in (lo, hi):
        assert np.all(np.mod(b * 2.0 ** 30, 1.0) == 0.0)
    x = np.random.default_rng(1).random((20000, d))
    inside = ((x[:, None, :] >= lo[None]) & (x[:, None, :] < hi[None])).all(axis=2)
    assert np.all(inside.sum(axis=1) == 1)
    # the extrema's points lie in their regions, and the spread is its definition
    for k in ("xmin", "xmax"):
        assert np.all(r[k] >= lo) and np.all(r[k] <= hi)
    vol = np.prod(hi - lo, axis=1)
    assert np.array_equal(r["spread"], 0.5 * vol * (r["fmax"] - r["fmin"]))
    assert np.all(r["fmax"] >= r["fmin"])


def test_cut_follows_the_only_varying_axis():
    d = 4
    a = np.array([0.0, 0.0, 8.0, 0.0])
    u = np.array([0.5, 0.5, 0.3, 0.5])
    r = O.divonne_partition(O.genz(W.GAUSSIAN, a, u), d, nsearch=64, niter=16, maxregions=20,
                            nsplit=2)
    assert np.all(r["cut"] == 2)
    assert np.all(r["lo"][:, [0, 1, 3]] == 0) and np.all(r["hi"][:, [0, 1, 3]] == 1)


def test_each_step_splits_the_largest_spread():
    d = 3
    a, u = W.genz_params(W.PRODUCT_PEAK, d, 6)
    g = O.genz(W.PRODUCT_PEAK, a, u)
    prev = O.divonne_partition(g, d, nsearch=64, niter=8, maxregions=1)
    for m in range(2, 14):
        cur = O.divonne_partition(g, d, nsearch=64, niter=8, maxregions=m)
        k = int(np.argmax(prev["spread"]))
        changed = [i for i in range(prev["nregions"])
                   if not np.array_equal(cur["hi"][i], prev["hi"][i])
                   or not np.array_equal(cur["lo"][i], prev["lo"][i])]
        assert changed == [k]
        # the cut halves the parent along the recorded dimension
        c = cur["cut"][-1]
        assert cur["hi"][k][c] == cur["lo"][-1][c] == 0.5 * (prev["lo"][k][c] + prev["hi"][k][c])
        prev = cur


def test_stop_rules():
    d = 3
    a, u = W.genz_params(W.C0, d, 7)
    g = O.genz(W.C0, a, u)
    r = O.divonne_partition(g, d, nsearch=64, niter=8, maxregions=500, spread_tol=10.0)
    assert r["nregions"] == 1 and r["fail"] == 0
    tol = 2e-3
    r = O.divonne_partition(g, d, nsearch=64, niter=8, maxregions=500, nsplit=8, spread_tol=tol)
    assert r["fail"] == 0 and r["spread"].max() <= tol < 1 and r["nregions"] > 10
    r = O.divonne_partition(g, d, nsearch=64, niter=8, maxregions=12, nsplit=8, spread_tol=tol)
    assert r["fail"] == 1 and r["nregions"] == 12
    c = O.divonne_partition(O.genz(W.GAUSSIAN, np.zeros(d), np.full(d, 0.5)), d, nsearch=16,
                            niter=4, maxregions=50)
    assert c["nregions"] == 1 and c["fail"] == 0 and c["total_spread"] == 0.0


def test_doubling_the_integrand_doubles_the_spreads():
    d = 3
    a, u = W.genz_params(W.PRODUCT_PEAK, d, 8)
    a2 = a ** -2.0

    def f(x):
        return 1.0 / np.prod(a2 + (x - u) ** 2, axis=1)

    kw = dict(nsearch=32, niter=10, maxregions=15, nsplit=2)
    r1 = O.divonne_partition(O.python_integrand(f), d, **kw)
    r2 = O.divonne_partition(O.python_integrand(lambda x: 2.0 * f(x)), d, **kw)
    assert np.array_equal(r1["cut"], r2["cut"]) and np.array_equal(r1["lo"], r2["lo"])
    assert np.array_equal(r2["spread"], 2 * r1["spread"])
    assert np.array_equal(r2["fmax"], 2 * r1["fmax"]) and np.array_equal(r2["fmin"], 2 * r1["fmin"])


def test_bad_arguments():
    g = O.genz(0, np.ones(3), np.full(3, 0.5))
    for kw in (dict(nsearch=0), dict(niter=-1), dict(maxregions=0), dict(nsplit=0),
               dict(spread_tol=-1.0)):
        with pytest.raises(ValueError):
            O.divonne_partition(g, 3, **kw)
    with pytest.raises(ValueError):
        O.divonne_partition(g, 17)


@pytest.mark.parametrize("d", [1, 2])
def test_one_search_iteration_in_the_children_by_brute_force(d):
    # both children of the first split (search serials 1 and 2), niter = 1:
    # each sample's best point, then one compass move of w_j/4 (clipped)
    n, seed = 16, 5
    a, u = W.genz_params(W.GAUSSIAN, d, 9)
    r = O.divonne_partition(O.genz(W.GAUSSIAN, a, u), d, seed=seed, nsearch=n, niter=1,
                            maxregions=2)
    moved = 0
    for pos, serial in ((0, 1), (1, 2)):
        lo, hi = r["lo"][pos], r["hi"][pos]
        w = hi - lo
        assert np.prod(w) == 0.5
        pts = np.zeros((n, d))
        for i in range(n):
            y = np.array(O.philox([i, serial << 8, 0, 0], [seed, 0])[:d], dtype=np.float64)
            pts[i] = (y * 2.0 ** -32 + 2.0 ** -33) * w + lo
        f = O.genz_eval(W.GAUSSIAN, a, u, pts)
        for sign, key in ((1, "max"), (-1, "min")):
            i0 = int(np.argmax(sign * f))
            x, fx = pts[i0].copy(), f[i0]
            cand = []
            for j in range(d):
                for s_ in (1, -1):
                    z = x.copy()
                    z[j] = min(max(x[j] + s_ * w[j] / 4, lo[j]), hi[j])
                    cand.append(z)
            fc = O.genz_eval(W.GAUSSIAN, a, u, np.array(cand))
            b = int(np.argmax(sign * fc))
            if sign * fc[b] > sign * fx:
                x, fx = cand[b], fc[b]
                moved += 1
            assert np.array_equal(r["x" + key][pos], x) and r["f" + key][pos] == fx
    assert moved > 0
