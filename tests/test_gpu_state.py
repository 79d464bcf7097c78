"""GPU tests of Vegas checkpoint/resume (statefile) and grid reuse (gridno).

Bars: a run stopped by maxeval and resumed under a larger one equals the
uninterrupted run (neval, fail, history; integral and error within 1e-13,
as two uninterrupted runs agree) and the oracle (1e-12); grid reuse equals the
oracle started from the same grid (1e-12).
"""
import os

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


def _same(r, s, tol=1e-13):
    assert r["neval"] == s["neval"] and r["fail"] == s["fail"]
    assert _rel(r["integral"], s["integral"]) < tol
    assert _rel(r["error"], s["error"]) < tol * 100
    if "iter_I" in r and "iter_I" in s:
        assert len(r["iter_I"]) == len(s["iter_I"])
        assert np.allclose(r["iter_I"], s["iter_I"], rtol=tol, atol=0)


@pytest.mark.parametrize("flags", [0, 1])
def test_resume_equals_uninterrupted(cc, ctx, tmp_path, flags):
    fam, d, n = W.OSCILLATORY, 6, 30011
    a, u = W.genz_params(fam, d, 2)
    kw = dict(ctx=ctx, flags=flags, nbins=64, nstart=n, nincrease=1000, seed=7, trace=True)
    whole = cc.vegas(fam, a, u, maxeval=6 * n + 15000, **kw)
    path = str(tmp_path / "vegas.state")
    part = cc.vegas(fam, a, u, maxeval=3 * n + 3000, statefile=path, **kw)
    assert part["fail"] == 1 and len(part["iter_I"]) == 3 and os.path.exists(path)
    rest = cc.vegas(fam, a, u, maxeval=6 * n + 15000, statefile=path, **kw)
    _same(rest, whole, 1e-13 if flags == 0 else 1e-12)
    assert np.allclose(rest["grid"], whole["grid"], rtol=0, atol=1e-12)
    assert os.path.exists(path)  # stopped by maxeval again: kept
    if flags == 0:
        o = O.vegas(O.genz(fam, a, u), d, nbins=64, nstart=n, nincrease=1000, seed=7,
                    maxeval=6 * n + 15000)
        assert _rel(rest["integral"], o["integral"]) < 1e-12
    # the same budget again: nothing left to do, the stored result comes back
    again = cc.vegas(fam, a, u, maxeval=6 * n + 15000, statefile=path, **kw)
    _same(again, rest, 1e-15)


def test_converged_run_removes_its_state_file(cc, ctx, tmp_path):
    a, u = W.genz_params(W.GAUSSIAN, 3, 3)
    path = str(tmp_path / "conv.state")
    r = cc.vegas(W.GAUSSIAN, a, u, ctx=ctx, epsrel=1e-3, nstart=20000, maxeval=10**7,
                 statefile=path)
    assert r["fail"] == 0 and not os.path.exists(path)
    plain = cc.vegas(W.GAUSSIAN, a, u, ctx=ctx, epsrel=1e-3, nstart=20000, maxeval=10**7)
    _same(r, plain)


def test_state_file_of_other_settings_is_refused(cc, ctx, tmp_path):
    a, u = W.genz_params(W.C0, 4, 4)
    path = str(tmp_path / "other.state")
    cc.vegas(W.C0, a, u, ctx=ctx, nstart=5000, maxeval=10000, statefile=path, seed=1)
    for kw in (dict(seed=2), dict(nbins=64), dict(nstart=6000), dict(flags=cc.FP32_EVAL)):
        args = dict(ctx=ctx, nstart=5000, maxeval=10**5, statefile=path, seed=1)
        args.update(kw)
        with pytest.raises(cc.CcubaError) as e:
            cc.vegas(W.C0, a, u, **args)
        assert e.value.rc == cc.EINVAL
    with pytest.raises(cc.CcubaError):  # another integrand
        cc.vegas(W.C0, 2.0 * a, u, ctx=ctx, nstart=5000, maxeval=10**5, statefile=path, seed=1)


def test_grid_reuse_matches_oracle(cc, ctx):
    fam, d, N = W.PRODUCT_PEAK, 5, 32
    a, u = W.genz_params(fam, d, 5)
    first = cc.vegas(fam, a, u, ctx=ctx, nbins=N, nstart=20000, maxeval=80000, gridno=3,
                     trace=True)
    G = first["grid"]
    kw = dict(nbins=N, nstart=10007, maxeval=3 * 10007, seed=9)
    second = cc.vegas(fam, a, u, ctx=ctx, gridno=-3, trace=True, **kw)
    o = O.vegas(O.genz(fam, a, u), d, grid=G, **kw)
    assert second["neval"] == o["neval"] and second["fail"] == o["fail"]
    assert _rel(second["integral"], o["integral"]) < 1e-12
    assert np.allclose(second["iter_I"], o["iter_I"], rtol=1e-12, atol=0)
    # gridno < 0 reads the slot without writing it: the same start again
    third = cc.vegas(fam, a, u, ctx=ctx, gridno=-3, trace=True, **kw)
    _same(third, second)
    # a slot of another shape is not used: the uniform start
    other = cc.vegas(fam, a, u, ctx=ctx, gridno=3, **dict(kw, nbins=64))
    plain = cc.vegas(fam, a, u, ctx=ctx, **dict(kw, nbins=64))
    _same(other, plain)


def test_truncated_state_file_is_refused(cc, ctx, tmp_path):
    a, u = W.genz_params(W.C0, 4, 6)
    path = str(tmp_path / "cut.state")
    kw = dict(ctx=ctx, nstart=5000, maxeval=10000, statefile=path, seed=1)
    cc.vegas(W.C0, a, u, **kw)
    data = open(path, "rb").read()
    with open(path, "wb") as fh:
        fh.write(data[:-8])
    with pytest.raises(cc.CcubaError) as e:
        cc.vegas(W.C0, a, u, **dict(kw, maxeval=10**5))
    assert e.value.rc == cc.EINVAL
    with open(path, "wb") as fh:  # whole again: the run goes on
        fh.write(data)
    r = cc.vegas(W.C0, a, u, **dict(kw, maxeval=20000))
    assert r["neval"] > 10000
