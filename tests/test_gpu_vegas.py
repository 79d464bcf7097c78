"""GPU parity of the Vegas DoSample path against the CPU oracle.

Bars: Philox words and bins bit-exact; FP64 points, weights and (for equal
inputs) refined grids bit-exact or within a few ulps; FP64 integral, error,
chi^2 probability and iteration history within 1e-12 relative; the
FP32-evaluate path's integral within 1e-6 relative of the oracle's FP32
emulation and of its FP64 result, its error estimate within 1e-5 (the
FP32 path's definition fixes it only to a few 1e-6: test_oracle_conditioning).
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


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _random_grid(rng, d, N):
    g = np.zeros((d, N + 1))
    for j in range(d):
        w = rng.random(N) ** 3 + 1e-3
        g[j, 1:] = np.cumsum(w) / w.sum()
        g[j, -1] = 1.0
    return g


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("d,N", [(1, 2), (4, 50), (7, 128), (8, 128), (16, 256)])
def test_points_bit_exact(cc, ctx, d, N, prec):
    rng = np.random.default_rng(d * 1000 + N)
    for grid in (np.tile(np.arange(N + 1) / N, (d, 1)), _random_grid(rng, d, N)):
        seed, sid, it, i0, n = 0xDEADBEEF12345678, 77, 5, (1 << 32) - 3000, 3000
        g = cc.vegas_points(ctx, d, N, grid, seed, sid, it, i0, n, flags=prec)
        o = O.vegas_points(d, N, grid, seed, sid, it, i0, n, precision=prec)
        nb = (d + 3) // 4
        assert np.array_equal(g["words"][:, :4 * nb], o["words"])
        assert np.array_equal(g["bin"], o["bin"])
        assert np.array_equal(g["x"], o["x"])
        assert np.array_equal(g["w"], o["w"])


def test_refine_matches_oracle(cc, ctx):
    rng = np.random.default_rng(5)
    for d, N in ((1, 2), (3, 50), (8, 128), (16, 256)):
        grid = _random_grid(rng, d, N)
        H = rng.random((d, N)) ** 6
        H[0, : N // 3] = 0.0  # empty stretches
        if d > 1:
            H[1] = 0.0        # an all-zero dimension keeps its grid
        G = cc.vegas_refine(ctx, H, grid)
        for j in range(d):
            ref = O.refine_dim(H[j], grid[j])
            assert np.max(np.abs(G[j] - ref)) <= 1e-14, (d, N, j)
            assert G[j][0] == 0.0 and G[j][-1] == 1.0


def _both(cc, ctx, fam, d, **kw):
    a, u = W.genz_params(fam, d, kw.pop("pseed", 1))
    prec = kw.get("flags", 0) & 3
    g = cc.vegas(fam, a, u, ctx=ctx, trace=True, **kw)
    kw2 = dict(kw)
    o = O.vegas(O.genz(fam, a, u, precision=prec), d, **kw2)
    return g, o


def _assert_vegas_close(g, o, tol, tol_err=None):
    tol_err = tol_err or tol
    assert g["neval"] == o["neval"] and g["fail"] == o["fail"]
    assert len(g["iter_I"]) == len(o["iter_I"])
    assert _rel(g["integral"], o["integral"]) < tol
    assert _rel(g["error"], o["error"]) < tol_err
    assert abs(g["prob"] - o["prob"]) < max(tol_err, 1e-12)
    assert np.allclose(g["iter_I"], o["iter_I"], rtol=tol, atol=0)
    assert np.allclose(g["iter_var"], o["iter_var"], rtol=tol_err, atol=0)


def test_small_config_fp64(cc, ctx):
    # Gaussian d=4, a=5, 50 bins, 10 iterations x 10^4 points, FP64 throughout
    for seed in (1, 2, 3):
        g, o = _both(cc, ctx, 0, 4, pseed=seed, seed=seed, nbins=50, nstart=10**4,
                     maxeval=10 * 10**4)
        _assert_vegas_close(g, o, 1e-12)
        assert np.max(np.abs(g["grid"] - o["grid"])) < 1e-12


@pytest.mark.parametrize("fam", range(5))
@pytest.mark.parametrize("d", [3, 6])
def test_families_fp64(cc, ctx, fam, d):
    g, o = _both(cc, ctx, fam, d, pseed=d, seed=11, nbins=64, nstart=20011, maxeval=5 * 20011)
    _assert_vegas_close(g, o, 1e-12)


@pytest.mark.parametrize("hist64", [0, 1])
@pytest.mark.parametrize("fam", range(5))
def test_families_fp32_eval(cc, fam, hist64):
    # both FP32-path histograms: 64-bit fixed point (with FP64 for the rest)
    # and FP64
    d = 5
    a, u = W.genz_params(fam, d, 4)
    c = cc.Context()
    c.config("hist64", hist64)
    g = cc.vegas(fam, a, u, ctx=c, flags=cc.FP32_EVAL, nbins=128, nstart=30000,
                 maxeval=6 * 30000, seed=3, trace=True)
    c.close()
    o32 = O.vegas(O.genz(fam, a, u, precision=O.FP32_EVAL), d, flags=O.FP32_EVAL, nbins=128,
                  nstart=30000, maxeval=6 * 30000, seed=3)
    o64 = O.vegas(O.genz(fam, a, u), d, nbins=128, nstart=30000, maxeval=6 * 30000, seed=3)
    assert g["neval"] == o32["neval"]
    assert _rel(g["integral"], o32["integral"]) < 1e-6
    assert _rel(g["error"], o32["error"]) < 1e-5  # see test_oracle_conditioning
    assert _rel(g["integral"], o64["integral"]) < 1e-6


def test_ragged_and_degenerate_sizes(cc, ctx):
    a, u = W.genz_params(2, 3, 9)
    # nstart = 2 (smallest), ragged counts, nincrease > 0
    for nstart, ninc, maxev in ((2, 0, 10), (257, 3, 5000), (99991, 1234, 5 * 10**5)):
        g = cc.vegas(2, a, u, ctx=ctx, nstart=nstart, nincrease=ninc, maxeval=maxev, nbins=16,
                     trace=True)
        o = O.vegas(O.genz(2, a, u), 3, nstart=nstart, nincrease=ninc, maxeval=maxev, nbins=16)
        _assert_vegas_close(g, o, 1e-12)
    # maxeval below nstart: no iteration at all
    g = cc.vegas(2, a, u, ctx=ctx, nstart=1000, maxeval=999)
    assert g["fail"] == 1 and g["neval"] == 0 and g["integral"] == 0.0


@pytest.mark.parametrize("d,N,prec", [(1, 2, 0), (1, 2, 1), (16, 256, 0), (16, 256, 1),
                                      (12, 100, 1), (9, 37, 0)])
def test_extreme_dims_and_bins(cc, ctx, d, N, prec):
    # smallest and largest dimension and bin count, odd bin counts (the
    # general map rather than the power-of-two one), and three Philox blocks
    a, u = W.genz_params(2, d, 5)
    n = 30011
    g = cc.vegas(2, a, u, ctx=ctx, flags=prec, nbins=N, nstart=n, maxeval=4 * n, seed=9,
                 trace=True)
    o = O.vegas(O.genz(2, a, u, precision=prec), d, flags=prec, nbins=N, nstart=n,
                maxeval=4 * n, seed=9)
    if prec == 0:
        _assert_vegas_close(g, o, 1e-12)
        assert np.max(np.abs(g["grid"] - o["grid"])) < 1e-12
    else:
        assert g["neval"] == o["neval"]
        assert _rel(g["integral"], o["integral"]) < 1e-6
        assert _rel(g["error"], o["error"]) < 1e-5


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32_eval", "fp64"])
@pytest.mark.parametrize("fam,d,N", [(0, 5, 128), (2, 8, 128), (1, 12, 50), (4, 3, 256),
                                     (2, 16, 256)])
def test_fixed_point_histogram_equals_fp64_histogram(cc, fam, d, N, prec):
    # The fixed-point histogram sums exactly what it holds and sends every
    # other v^2 to an FP64 histogram, so the two histograms of either
    # precision differ by summation order only: the runs agree to FP64
    # rounding.  (d = 16 with 256 bins in FP64 takes the FP64 histogram in
    # both runs: its fixed-point one would not fit the LDS.)
    a, u = W.genz_params(fam, d, 6)
    out = []
    for h in (1, 0):
        c = cc.Context()
        c.config("hist64", h)
        out.append(cc.vegas(fam, a, u, ctx=c, flags=prec, nbins=N, nstart=50021,
                            maxeval=8 * 50021, seed=5, trace=True))
        c.close()
    r64, rfx = out
    assert rfx["neval"] == r64["neval"]
    assert _rel(rfx["integral"], r64["integral"]) < 1e-12
    assert _rel(rfx["error"], r64["error"]) < 1e-12
    assert np.max(np.abs(rfx["grid"] - r64["grid"])) < 1e-12


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32_eval", "fp64"])
def test_rerun_is_bit_identical(cc, prec):
    # With every v^2 inside the fixed-point window (a flat product peak, whose
    # v^2 stay within a factor 2^23 of each other) the histogram is an
    # integer sum, independent of the order of the LDS adds, and every other
    # sum is taken in a fixed order: two runs give the same bits.  Each run
    # has its own context (and so its own buffers and graphs).  (FP64
    # evaluation takes the fixed-point histogram when asked: by default it
    # adds in FP64.)
    d = 6
    a, u = np.full(d, 0.5), W.genz_params(2, d, 3)[1]
    out = []
    for _ in range(2):
        c = cc.Context()
        c.config("hist64", 0)
        out.append(cc.vegas(2, a, u, ctx=c, flags=prec, nbins=128, nstart=300007,
                            maxeval=6 * 300007, seed=9, trace=True))
        c.close()
    r0, r1 = out
    for k in ("integral", "error", "prob", "neval", "chi2"):
        assert r0[k] == r1[k], k
    assert np.array_equal(r0["iter_I"], r1["iter_I"])
    assert np.array_equal(r0["iter_var"], r1["iter_var"])
    assert np.array_equal(r0["grid"], r1["grid"])


def test_zero_variance_frozen_grid(cc, ctx):
    # a = 0 makes the Gaussian the constant 1; on the frozen uniform grid with
    # N = 128 every weight is exactly 1, so sigma_t = 0 and the result is 1
    for prec in (cc.FP64, cc.FP32_EVAL):
        g = cc.vegas(0, np.zeros(3), np.full(3, 0.5), ctx=ctx, nbins=128, nstart=4096,
                     maxeval=3 * 4096, flags=prec | cc.FREEZE_GRID, trace=True)
        assert g["integral"] == 1.0 and g["error"] == 0.0 and g["fail"] == 0


def test_epsrel_convergence_matches_oracle(cc, ctx):
    g, o = _both(cc, ctx, 0, 3, pseed=2, epsrel=2e-4, nstart=5000, nincrease=2500,
                 maxeval=10**7, nbins=128)
    assert g["fail"] == 0
    _assert_vegas_close(g, o, 1e-12)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_eval"])
def test_geometry_invariance(cc, prec):
    # block size, blocks per CU and points per lane per trip (ILP) change the
    # tiles and the order of the sums, not the points
    a, u = W.genz_params(1, 8, 3)
    base = None
    for block, bpc, ilp in ((256, 4, 1), (128, 2, 2), (64, 8, 1), (256, 1, 2), (256, 3, 2)):
        c = cc.Context()
        c.config("block", block)
        c.config("blocks_per_cu", bpc)
        c.config("ilp", ilp)
        r = cc.vegas(1, a, u, ctx=c, flags=prec, nstart=200003, maxeval=3 * 200003)
        c.close()
        if base is None:
            base = r
        else:
            assert _rel(r["integral"], base["integral"]) < 1e-13
            assert _rel(r["error"], base["error"]) < 1e-12


def test_spin_semantics(cc):
    # NULL context, a context created by the call, and a reused one agree
    import ctypes as C
    a, u = W.genz_params(0, 3, 1)
    r0 = cc.vegas(0, a, u, ctx=None, nstart=5000, maxeval=15000)
    c = cc.Context()
    r1 = cc.vegas(0, a, u, ctx=c, nstart=5000, maxeval=15000)
    r2 = cc.vegas(0, a, u, ctx=c, nstart=5000, maxeval=15000)
    c.close()
    assert not c.handle
    for r in (r1, r2):
        assert _rel(r["integral"], r0["integral"]) < 1e-13
    del C


def test_dosample_raw_on_torch_stream(cc, ctx):
    import torch
    d, N, n = 6, 128, 300007
    a, u = W.genz_params(4, d, 2)
    grid = torch.tensor(np.tile(np.arange(N + 1) / N, (d, 1)), dtype=torch.float64,
                        device="cuda")
    sums = torch.zeros(2, dtype=torch.float64, device="cuda")
    hist = torch.zeros(d * N, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    cc.vegas_dosample_raw(ctx, 4, a, u, N, 0, n, grid.data_ptr(), sums.data_ptr(),
                          hist.data_ptr(), stream_ptr=s.cuda_stream)
    s.synchronize()
    o = O.vegas(O.genz(4, a, u), d, nbins=N, nstart=n, maxeval=n)
    S1 = o["iter_I"][0] * n
    assert _rel(sums[0].item(), S1) < 1e-12
    assert np.allclose(hist.cpu().numpy().reshape(d, N), o["hist"], rtol=1e-12, atol=0)


def test_full_size_first_iteration_fp64(cc, ctx):
    # d = 8 oscillatory, 128 bins, one full iteration of 10^7 points
    a, u = W.genz_params(1, 8, 1)
    n = 10**7
    g = cc.vegas(1, a, u, ctx=ctx, nbins=128, nstart=n, maxeval=n, seed=1, trace=True)
    o = O.vegas(O.genz(1, a, u), 8, nbins=128, nstart=n, maxeval=n, seed=1)
    assert _rel(g["iter_I"][0], o["iter_I"][0]) < 1e-12
    assert _rel(g["iter_var"][0], o["iter_var"][0]) < 1e-12
    assert np.max(np.abs(g["grid"] - o["grid"])) < 1e-12


def test_full_size_run_properties(cc, ctx):
    # 20 iterations x 10^7 points, FP32 evaluation and FP64: the closed form
    # lies within 5 sigma and the two precisions agree within 1e-6
    from closed_forms import exact
    for fam in (1, 2):
        a, u = W.genz_params(fam, 8, 1)
        ex = exact(fam, a, u)
        r64 = cc.vegas(fam, a, u, ctx=ctx, nbins=128, nstart=10**7, maxeval=20 * 10**7)
        r32 = cc.vegas(fam, a, u, ctx=ctx, nbins=128, nstart=10**7, maxeval=20 * 10**7,
                       flags=cc.FP32_EVAL)
        for r in (r64, r32):
            assert r["neval"] == 2 * 10**8 and r["fail"] == 1
            assert abs(r["integral"] - ex) < 5 * r["error"]
        assert _rel(r32["integral"], r64["integral"]) < 1e-6
