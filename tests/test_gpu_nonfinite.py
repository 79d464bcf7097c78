"""GPU parity of the non-finite integrand rule (fail = -4, zero results)
against the oracle: Vegas through a device-source integrand and a batched
host integrand, Cuhre and Divonne's partitioning phase through a corner peak
whose base vanishes on the line x_0 = 1/2 (a = (-2, 0): f = (1 - 2 x_0)^-3)."""
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


INF_SOURCE = """
__device__ double ccuba_user(const double *x, int ndim, const double *a, const double *u) {
  return x[0] < 0.25 ? __builtin_inf() : 1.0;
}
"""


def _inf_quarter(x):
    return np.where(x[:, 0] < 0.25, np.inf, 1.0)


def test_vegas_device_source(cc, ctx):
    kw = dict(nstart=5000, maxeval=50000, nbins=32)
    g = cc.vegas_source(INF_SOURCE, 3, ctx=ctx, **kw)
    o = O.vegas(O.python_integrand(_inf_quarter), 3, **kw)
    assert g["fail"] == o["fail"] == -4 and g["neval"] == o["neval"] == 5000
    assert g["integral"] == g["error"] == g["prob"] == 0.0


def test_vegas_batched_host_integrand(cc, ctx):
    f = lambda x: np.where(x[:, 1] > 0.9, np.nan, np.exp(-np.sum(x * x, axis=1)))
    kw = dict(nstart=4000, maxeval=40000, nbins=32)
    g = cc.vegas_batched(f, 2, ctx=ctx, nvec=1000, **kw)
    o = O.vegas(O.python_integrand(f), 2, nvec=1000, **kw)
    assert g["fail"] == o["fail"] == -4 and g["neval"] == o["neval"]
    assert g["integral"] == 0.0


def test_cuhre_corner_peak_pole(cc, ctx):
    a, u = np.array([-2.0, 0.0]), np.zeros(2)
    g = cc.cuhre(W.CORNER_PEAK, a, u, ctx=ctx, epsrel=1e-3, maxeval=10**6)
    o = O.cuhre(O.genz(W.CORNER_PEAK, a, u), 2, epsrel=1e-3, maxeval=10**6)
    assert g["fail"] == o["fail"] == -4 and g["neval"] == o["neval"]
    assert g["integral"] == 0.0 and g["error"] == 0.0


def test_divonne_partition_corner_peak_pole(cc, ctx):
    # the first cut is at x_0 = 1/2; the lower child's maximum search is
    # clipped onto that face, where f is infinite
    a, u = np.array([-2.0, 0.0]), np.zeros(2)
    kw = dict(nsearch=64, niter=16, maxregions=20)
    g = cc.divonne_partition(W.CORNER_PEAK, a, u, ctx=ctx, **kw)
    o = O.divonne_partition(O.genz(W.CORNER_PEAK, a, u), 2, **kw)
    assert g["fail"] == o["fail"] == -4 and g["neval"] == o["neval"]
    assert g["total_spread"] == o["total_spread"] == 0.0
