"""GPU parity of Divonne's partitioning phase (ccuba_divonne_partition)
against the oracle.

Bar: the same regions (bounds bit-exact, the same cut of every split), neval,
fail and region count; fmax, fmin and spreads within 1e-12 relative, the total
spread within 1e-12.  The extrema's points agree exactly where they are
corners (monotone integrands) and otherwise to 1e-6: at a smooth extremum f
is flat to FP64 rounding over ~sqrt(eps) of x, so the device's and the
oracle's integrand roundings may stop the compass search at different points
of equal value there.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

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


def _both(cc, ctx, fam, d, seed=1, a=None, u=None, **kw):
    if a is None:
        a, u = W.genz_params(fam, d, seed)
    g = cc.divonne_partition(fam, a, u, ctx=ctx, trace=True, seed=seed, **kw)
    o = O.divonne_partition(O.genz(fam, a, u), d, seed=seed, **kw)
    return g, o


def _compare(g, o, xtol=1e-6):
    print("regions", g["nregions"], o["nregions"], "neval", g["neval"], o["neval"], flush=True)
    assert g["nregions"] == o["nregions"] and g["neval"] == o["neval"] and g["fail"] == o["fail"]
    assert np.array_equal(g["cut"], o["cut"])
    assert np.array_equal(g["lo"], o["lo"]) and np.array_equal(g["hi"], o["hi"])
    for k in ("fmax", "fmin", "spread"):
        assert np.allclose(g[k], o[k], rtol=1e-12, atol=1e-300), k
    assert abs(g["total_spread"] - o["total_spread"]) <= 1e-12 * abs(o["total_spread"])
    for k in ("xmax", "xmin"):
        assert np.allclose(g[k], o[k], rtol=0, atol=xtol), k


@pytest.mark.parametrize("fam", range(5))
@pytest.mark.parametrize("d", [3, 6])
def test_matches_oracle(cc, ctx, fam, d):
    g, o = _both(cc, ctx, fam, d, seed=fam + 10 * d, nsearch=300, niter=24, maxregions=48,
                 nsplit=1)
    _compare(g, o)


@pytest.mark.parametrize("nsplit", [4, 64])
def test_batched_splits_match_oracle(cc, ctx, nsplit):
    g, o = _both(cc, ctx, W.PRODUCT_PEAK, 5, seed=3, nsearch=500, niter=32, maxregions=400,
                 nsplit=nsplit)
    assert g["nregions"] == 400
    _compare(g, o)


def test_corner_peak_extrema_are_exact_corners(cc, ctx):
    g, o = _both(cc, ctx, W.CORNER_PEAK, 4, seed=2, nsearch=64, niter=64, maxregions=40,
                 nsplit=5)
    _compare(g, o, xtol=0.0)
    assert np.array_equal(g["xmax"], g["lo"]) and np.array_equal(g["xmin"], g["hi"])


@pytest.mark.parametrize("d,nsearch,niter", [(1, 1, 0), (1, 7, 3), (2, 129, 1), (16, 200, 8),
                                             (13, 1000, 40)])
def test_extreme_shapes(cc, ctx, d, nsearch, niter):
    g, o = _both(cc, ctx, W.C0, d, seed=d, nsearch=nsearch, niter=niter, maxregions=30,
                 nsplit=3)
    _compare(g, o)


def test_stop_rules_and_constant(cc, ctx):
    a, u = W.genz_params(W.C0, 3, 7)
    g, o = _both(cc, ctx, W.C0, 3, seed=7, a=a, u=u, nsearch=64, niter=8, maxregions=500,
                 nsplit=8, spread_tol=2e-3)
    assert g["fail"] == 0 and g["spread"].max() <= 2e-3
    _compare(g, o)
    r = cc.divonne_partition(W.C0, a, u, ctx=ctx, maxregions=500, spread_tol=10.0)
    assert r["nregions"] == 1 and r["fail"] == 0
    r = cc.divonne_partition(W.GAUSSIAN, np.zeros(3), np.full(3, 0.5), ctx=ctx, nsearch=16,
                             niter=4, maxregions=50)
    assert r["nregions"] == 1 and r["fail"] == 0 and r["total_spread"] == 0.0


def test_bench_shape_first_steps_match_oracle(cc, ctx):
    # Gaussian d = 8, 1024 search points and 64 compass iterations per region,
    # 256 splits per step
    g, o = _both(cc, ctx, W.GAUSSIAN, 8, seed=5, nsearch=1024, niter=64, maxregions=128,
                 nsplit=256)
    assert g["nregions"] == 128
    _compare(g, o)


def test_bad_arguments(cc, ctx):
    a, u = W.genz_params(W.GAUSSIAN, 3, 4)
    for kw in (dict(nsearch=0), dict(niter=-1), dict(niter=4097), dict(maxregions=0),
               dict(nsplit=0), dict(nsplit=1025), dict(spread_tol=-1.0)):
        with pytest.raises(cc.CcubaError) as e:
            cc.divonne_partition(W.GAUSSIAN, a, u, ctx=ctx, **kw)
        assert e.value.rc == cc.EINVAL


def test_full_bench_shape_properties(cc, ctx):
    # the benchmark's partition (d = 8 Gaussian to 16384 regions), checked
    # through what holds at any size; every extremum is recomputed from its
    # point by the oracle's integrand
    d = 8
    a, u = W.genz_params(W.GAUSSIAN, d, 1)
    kw = dict(nsearch=1024, niter=64, maxregions=16384, nsplit=1024)
    r = cc.divonne_partition(W.GAUSSIAN, a, u, ctx=ctx, trace=True, **kw)
    R = r["nregions"]
    assert R == 16384 and r["fail"] == 1 and len(r["cut"]) == R - 1
    assert r["neval"] == (2 * R - 1) * (1024 + 4 * d * 64) + d * (R - 1)
    lo, hi = r["lo"], r["hi"]
    vol = np.prod(hi - lo, axis=1)
    assert vol.sum() == 1.0 and np.all(vol > 0)
    x = np.random.default_rng(2).random((4000, d))
    inside = ((x[:, None, :] >= lo[None]) & (x[:, None, :] < hi[None])).all(axis=2)
    assert np.all(inside.sum(axis=1) == 1)
    for k in ("xmin", "xmax"):
        assert np.all(r[k] >= lo) and np.all(r[k] <= hi)
    assert np.array_equal(r["spread"], 0.5 * vol * (r["fmax"] - r["fmin"]))
    # f = exp(-s) with s up to ~100 at the minima: a few ulps of s, summed in
    # another order by the oracle's integrand, are ~1e-14 relative in f
    pick = np.random.default_rng(3).choice(R, 256, replace=False)
    assert np.allclose(O.genz_eval(W.GAUSSIAN, a, u, r["xmax"][pick]), r["fmax"][pick],
                       rtol=1e-12, atol=0)
    assert np.allclose(O.genz_eval(W.GAUSSIAN, a, u, r["xmin"][pick]), r["fmin"][pick],
                       rtol=1e-12, atol=0)
    assert abs(r["total_spread"] - r["spread"].sum()) <= 1e-12 * r["total_spread"]


def test_stream_id_and_large_seed_match_oracle(cc, ctx):
    a, u = W.genz_params(W.C0, 4, 32)
    kw = dict(nsearch=200, niter=12, maxregions=30, nsplit=3, stream_id=9)
    g = cc.divonne_partition(W.C0, a, u, ctx=ctx, trace=True, seed=(5 << 33) + 1, **kw)
    o = O.divonne_partition(O.genz(W.C0, a, u), 4, seed=(5 << 33) + 1, **kw)
    _compare(g, o)
