"""GPU checks of the serving loop: requests admitted while others run share
the device launches, and each result is the one the request gets alone
(Vegas: same points; Cuhre: same subdivisions)."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import paper_1408_6373_amd as cc
    return cc


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _requests(n, seed):
    reqs = W.serving_requests(n, rate=1000.0, seed=seed, dmax=8, eps_lo=1e-4, eps_hi=1e-2)
    specs = []
    for q, r in enumerate(reqs):
        if r["method"] == 0:
            specs.append(dict(method=0, ndim=r["ndim"], family=r["family"], a=r["a"], u=r["u"],
                              seed=r["seed"], stream_id=r["stream_id"], epsrel=r["epsrel"],
                              nstart=20000, nincrease=10000, maxeval=2 * 10**6, nbins=128,
                              flags=q % 2))
        else:
            specs.append(dict(method=1, ndim=r["ndim"], family=r["family"], a=r["a"], u=r["u"],
                              epsrel=r["epsrel"], maxeval=3 * 10**6,
                              max_regions_per_batch=2000, flags=0))
    return specs


def _alone(cc, ctx, s):
    if s["method"] == 0:
        return cc.vegas(s["family"], s["a"], s["u"], ctx=ctx, flags=s["flags"], seed=s["seed"],
                        stream_id=s["stream_id"], epsrel=s["epsrel"], nstart=s["nstart"],
                        nincrease=s["nincrease"], maxeval=s["maxeval"], nbins=s["nbins"])
    return cc.cuhre(s["family"], s["a"], s["u"], ctx=ctx, epsrel=s["epsrel"],
                    maxeval=s["maxeval"], max_regions_per_batch=s["max_regions_per_batch"])


def _check(cc, ctx, specs, results):
    for s, r in zip(specs, results):
        assert r["status"] == 0 and r["t_done"] >= r["t_submit"]
        a = _alone(cc, ctx, s)
        assert r["neval"] == a["neval"] and r["fail"] == a["fail"]
        if s["method"] == 1:
            assert r["nregions"] == a["nregions"]
        assert _rel(r["integral"], a["integral"]) < 1e-12
        assert _rel(r["error"], a["error"]) < 1e-12


def test_mixed_requests_equal_alone(cc):
    ctx = cc.Context()
    specs = _requests(30, 7)
    tickets = [cc.submit(ctx, s) for s in specs]
    cc.drain(ctx)
    results = [cc.poll(ctx, t) for t in tickets]
    assert all(r is not None for r in results)
    _check(cc, ctx, specs, results)
    ctx.close()


def test_arrivals_while_running_join_the_batch(cc):
    ctx = cc.Context()
    first = _requests(10, 11)
    t1 = [cc.submit(ctx, s) for s in first]
    time.sleep(0.002)
    second = _requests(10, 12)
    t2 = [cc.submit(ctx, s) for s in second]
    got = {}
    for t in t1 + t2:  # results of requests that already finished
        r = cc.poll(ctx, t)
        if r is not None:
            got[t] = r
    cc.drain(ctx)
    for t in t1 + t2:
        if t not in got:
            got[t] = cc.poll(ctx, t)
    _check(cc, ctx, first + second, [got[t] for t in t1 + t2])
    ctx.close()


def test_poll_unknown_and_repeated(cc):
    ctx = cc.Context()
    s = _requests(1, 3)[0]
    t = cc.submit(ctx, s)
    cc.drain(ctx)
    assert cc.poll(ctx, t) is not None
    with pytest.raises(cc.CcubaError) as e:
        cc.poll(ctx, t)
    assert e.value.rc == cc.ENOENT
    with pytest.raises(cc.CcubaError):
        cc.poll(ctx, 10**9)
    ctx.close()


def test_small_budget_queues_or_refuses(cc):
    # 64 MiB budget: small requests queue until memory frees; a Cuhre request
    # whose region heap cannot fit alone is refused with ENOMEM
    ctx = cc.Context(hbm_budget=64 << 20)
    specs = _requests(12, 21)
    big = dict(method=1, ndim=3, family=0, a=np.full(3, 5.0), u=np.full(3, 0.3),
               epsrel=1e-12, maxeval=10**10, max_regions_per_batch=10**7, flags=0)
    tickets = [cc.submit(ctx, s) for s in specs] + [cc.submit(ctx, big)]
    cc.drain(ctx)
    res = [cc.poll(ctx, t) for t in tickets]
    assert res[-1]["status"] == cc.ENOMEM
    ok = [r for r in res[:-1] if r["status"] == 0]
    assert len(ok) == len(specs)
    ctx.close()


def test_invalid_request_status(cc):
    ctx = cc.Context()
    bad = dict(method=0, ndim=3, family=0, a=np.ones(3), u=np.ones(3) / 2, nstart=1,
               maxeval=100)
    t = cc.submit(ctx, bad)
    cc.drain(ctx)
    assert cc.poll(ctx, t)["status"] == cc.EINVAL
    ctx.close()
