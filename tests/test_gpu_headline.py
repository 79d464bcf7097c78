"""Parity of the headline workload against the CPU oracle, on the path the
benchmark times.

The workload: Vegas in d = 8 with 128 bins per dimension, 20 iterations of
10^7 points, on the Genz oscillatory and product-peak integrands (parameter
seed 1, Philox seed 1, stream 0), in FP32 evaluation with FP64 accumulation
and in all-FP64.  The benchmark runs the two integrals as one batch
(ccuba_vegas_batch); here the same batch is compared with the oracle, and
each integral run alone with its iteration history (ccuba_vegas_ex) is
compared iteration by iteration.

Bars (relative unless stated):
  * FP64: integral and every I_t 1e-12; grid 1e-12 absolute.  Both sides
    take the iteration's sums about the previous estimate, so sigma_t^2
    keeps its digits although the variance is ~1e-4 of the mean of v^2 here.
    The grids drift apart by about an ulp per refinement (the device
    library's log and pow against the C library's, sums in another order):
    ~16 ulps of 0.5 after 20 iterations.  A drift delta moves the weight of
    every point of a bin of width h by delta/h, ~1e-12 in the narrowest
    (5e-3) bins of the product peak, and sigma_t^2 and the error estimate
    with it: sigma_t^2 1e-11, error 5e-12 (measured at most 1.9e-12 and
    1.05e-12).  chi^2 compares I_t - I with sigma_t, which is ~1e-5 I here,
    so a 1e-16 difference of the I_t is ~1e-11 of chi^2: bars 1e-9 on chi^2
    and 1e-9 absolute on prob.
  * FP32 evaluation: the two sides evaluate the integrand in binary32 by
    formulas that round differently (the device folds log2 e and 1/(2 pi)
    into its constants and calls the device library's exp2 and cospi, the
    oracle calls the C library's expf and cosf on the plain definition), so
    single values differ by a few ulps.  The integral and every I_t are held
    to 1e-6, the grid to 1e-6 absolute.  Such last-bit differences move the
    error estimate by a few 1e-6 (one rounding per factor of the product
    peak moves the oracle's own estimate by 2e-6: test_oracle_conditioning),
    so the error is held to 1e-5, and every sigma_t^2, which the same
    change moves by up to 8e-6 in an iteration where the grid is still
    moving, to 1e-4 (measured at most 4.3e-5).  The I_t differ by up to
    ~5e-8, which is ~1e-3 of sigma_t here: chi^2 1e-2, prob 1e-2 absolute.
The oracle runs of the full workload (2 x 10^8 evaluations each) go in
parallel threads: the oracle is plain C behind ctypes, which releases the
GIL.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

D, NBINS, NPTS, ITERS = 8, 128, 10**7, 20
FAMILIES = (W.OSCILLATORY, W.PRODUCT_PEAK)


@pytest.fixture(scope="module")
def cc():
    import paper_1408_6373_amd as cc
    return cc


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _maxrel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _oracle_runs(cases, **kw):
    """{(family, precision): oracle result} for the headline shape, in parallel."""
    def one(case):
        fam, prec = case
        a, u = W.genz_params(fam, D, 1)
        return O.vegas(O.genz(fam, a, u, precision=prec), D, flags=prec, seed=1, stream_id=0,
                       nbins=NBINS, **kw)
    with cf.ThreadPoolExecutor(max_workers=len(cases)) as ex:
        return dict(zip(cases, ex.map(one, cases)))


def _spec(fam, prec, **kw):
    a, u = W.genz_params(fam, D, 1)
    return dict(dict(method=0, ndim=D, family=fam, a=a, u=u, flags=prec, seed=1, stream_id=0,
                     nbins=NBINS), **kw)


def _check(tag, r, o, tr, bars):
    """Compare a device result (and its trace, if any) with the oracle."""
    d = dict(integral=_rel(r["integral"], o["integral"]),
             error=_rel(r["error"], o["error"]), prob=abs(r["prob"] - o["prob"]))
    if tr is not None:
        d.update(iter_I=_maxrel(tr["iter_I"], o["iter_I"]),
                 iter_var=_maxrel(tr["iter_var"], o["iter_var"]),
                 chi2=_rel(tr["chi2"], o["chi2"]),
                 grid=float(np.max(np.abs(tr["grid"] - o["grid"]))))
    print("PARITY %s %s" % (tag, " ".join("%s=%.3g" % kv for kv in sorted(d.items()))))
    assert r["neval"] == o["neval"] and r["fail"] == o["fail"], tag
    if tr is not None:
        assert len(tr["iter_I"]) == len(o["iter_I"]) and tr["dof"] == o["dof"], tag
    for k, v in d.items():
        assert v <= bars[k], (tag, k, v, bars[k])


BARS = {
    0: dict(integral=1e-12, error=5e-12, prob=1e-9, iter_I=1e-12, iter_var=1e-11, chi2=1e-9,
            grid=1e-12),
    1: dict(integral=1e-6, error=1e-5, prob=1e-2, iter_I=1e-6, iter_var=1e-4, chi2=1e-2,
            grid=1e-6),
}


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32_eval", "fp64"])
def test_headline_config_against_oracle(cc, prec):
    """The full headline workload: the bench's batch of both integrals, and
    each integral alone with its history, against the oracle."""
    oracle = _oracle_runs([(f, prec) for f in FAMILIES], nstart=NPTS, maxeval=ITERS * NPTS)
    ctx = cc.Context()
    try:
        specs = [_spec(f, prec, nstart=NPTS, maxeval=ITERS * NPTS) for f in FAMILIES]
        batch = cc.vegas_batch(ctx, specs)
        for f, s, r in zip(FAMILIES, specs, batch):
            assert r["status"] == 0
            _check("batch fam=%d prec=%d" % (f, prec), r, oracle[(f, prec)], None, BARS[prec])
            alone = cc.vegas(f, s["a"], s["u"], ctx=ctx, flags=prec, seed=1, nbins=NBINS,
                             nstart=NPTS, maxeval=ITERS * NPTS, trace=True)
            _check("alone fam=%d prec=%d" % (f, prec), alone, oracle[(f, prec)], alone,
                   BARS[prec])
    finally:
        ctx.close()


def test_multitrip_fp32_tiles_against_oracle(cc):
    """d = 8, 128 bins, FP32 evaluation with 2 points per lane per trip: the
    batch path's 16384-point tiles take 32 trips of a 256-thread block, and
    the single-integral path's tiles about 6; 3 iterations of 2 x 10^6 points,
    iteration by iteration against the oracle's FP32 emulation."""
    n, iters = 2 * 10**6, 3
    oracle = _oracle_runs([(f, 1) for f in FAMILIES], nstart=n, maxeval=iters * n)
    ctx = cc.Context()
    try:
        assert ctx.config_get("ilp", cc.FP32_EVAL) == 2
        assert ctx.config_get("block", cc.FP32_EVAL) == 256
        specs = [_spec(f, 1, nstart=n, maxeval=iters * n) for f in FAMILIES]
        for f, s, r in zip(FAMILIES, specs, cc.vegas_batch(ctx, specs)):
            assert r["status"] == 0
            _check("multitrip batch fam=%d" % f, r, oracle[(f, 1)], None, BARS[1])
            alone = cc.vegas(f, s["a"], s["u"], ctx=ctx, flags=1, seed=1, nbins=NBINS,
                             nstart=n, maxeval=iters * n, trace=True)
            _check("multitrip alone fam=%d" % f, alone, oracle[(f, 1)], alone, BARS[1])
    finally:
        ctx.close()
