"""GPU parity of Vegas with a device integrand compiled at run time into the
DoSample kernel (ccuba_vegas_source).

Bars: a source that computes a built-in Genz family with the same operations
gives that family's results (1e-13 relative: the runs differ only in the
order of FP64 histogram additions); any other source agrees with the oracle
calling the same function in Python within 1e-12 (FP64), or, with FP32
evaluation, the oracle's FP32 emulation of the family within 1e-6 (integral)
and 1e-5 (error: the two evaluate it in binary32 with different roundings,
which the error estimate is sensitive to); a bad source is refused with the
compiler's message.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

GAUSS_SRC = r"""
__device__ double ccuba_user(const double *x, int d, const double *a, const double *u) {
  double s = 0.0;
  for (int j = 0; j < d; ++j) {
    const double t = x[j] - u[j];
    s = fma(a[j] * a[j], t * t, s);
  }
  return exp(-s);
}
__device__ float ccuba_user(const float *x, int d, const float *a, const float *u) {
  float s = 0.0f;
  for (int j = 0; j < d; ++j) {
    const float t = x[j] - u[j];
    s = fmaf(a[j] * a[j], t * t, s);
  }
  return expf(-s);
}
"""

# not a Genz family: a product of sines and a sum inside a cosine
ODD_SRC = r"""
__device__ double ccuba_user(const double *x, int d, const double *a, const double *u) {
  double p = 1.0, s = 0.0;
  for (int j = 0; j < d; ++j) {
    p *= 1.0 + a[j] * sin(3.0 * x[j]);
    s += u[j] * x[j];
  }
  return p * cos(s);
}
"""


def _odd_py(a, u):
    def f(x):
        return np.prod(1.0 + a * np.sin(3.0 * x), axis=1) * np.cos(np.sum(u * x, axis=1))
    return f


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


@pytest.mark.parametrize("d,N", [(8, 128), (5, 100), (3, 64)])
def test_source_gaussian_equals_builtin_family(cc, ctx, d, N):
    a, u = W.genz_params(W.GAUSSIAN, d, d)
    kw = dict(ctx=ctx, nbins=N, nstart=50021, maxeval=6 * 50021, seed=4)
    s = cc.vegas_source(GAUSS_SRC, d, a, u, **kw)
    b = cc.vegas(W.GAUSSIAN, a, u, **kw)
    assert s["neval"] == b["neval"] and s["fail"] == b["fail"]
    assert _rel(s["integral"], b["integral"]) < 1e-13
    assert _rel(s["error"], b["error"]) < 1e-12
    assert abs(s["prob"] - b["prob"]) < 1e-11


def test_source_matches_oracle(cc, ctx):
    d = 4
    rng = np.random.default_rng(7)
    a, u = 0.5 * rng.random(d), rng.random(d)
    kw = dict(nbins=64, nstart=20011, maxeval=5 * 20011, seed=6)
    g = cc.vegas_source(ODD_SRC, d, a, u, ctx=ctx, **kw)
    o = O.vegas(O.python_integrand(_odd_py(a, u)), d, **kw)
    assert g["neval"] == o["neval"] and g["fail"] == o["fail"]
    assert _rel(g["integral"], o["integral"]) < 1e-12
    assert _rel(g["error"], o["error"]) < 1e-12


def test_source_fp32_evaluation(cc, ctx):
    d = 6
    a, u = W.genz_params(W.GAUSSIAN, d, 2)
    kw = dict(nbins=128, nstart=100003, maxeval=4 * 100003, seed=8)
    g = cc.vegas_source(GAUSS_SRC, d, a, u, ctx=ctx, flags=cc.FP32_EVAL, **kw)
    o = O.vegas(O.genz(W.GAUSSIAN, a, u, precision=O.FP32_EVAL), d, flags=O.FP32_EVAL, **kw)
    assert g["neval"] == o["neval"]
    assert _rel(g["integral"], o["integral"]) < 1e-6
    assert _rel(g["error"], o["error"]) < 1e-5


def test_source_converges(cc, ctx):
    a, u = W.genz_params(W.GAUSSIAN, 3, 5)
    g = cc.vegas_source(GAUSS_SRC, 3, a, u, ctx=ctx, epsrel=1e-4, nstart=10**5,
                        nincrease=10**4, maxeval=10**8)
    b = cc.vegas(W.GAUSSIAN, a, u, ctx=ctx, epsrel=1e-4, nstart=10**5, nincrease=10**4,
                 maxeval=10**8)
    assert g["fail"] == 0 and g["neval"] == b["neval"]
    assert g["error"] <= 1e-4 * abs(g["integral"])


def test_bad_source_is_refused_with_the_message(cc, ctx):
    bad = "__device__ double ccuba_user(const double *x, int d, const double *a, " \
          "const double *u) { return undefined_thing(x); }"
    with pytest.raises(cc.CcubaError) as e:
        cc.vegas_source(bad, 3, ctx=ctx, nstart=1000, maxeval=1000)
    assert e.value.rc == cc.EINVAL and "undefined_thing" in str(e.value)
    # FP32 evaluation needs the float version
    only64 = ODD_SRC
    with pytest.raises(cc.CcubaError):
        cc.vegas_source(only64, 3, ctx=ctx, flags=cc.FP32_EVAL, nstart=1000, maxeval=1000)
