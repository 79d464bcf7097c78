"""GPU checks of the batched Vegas launch: every integral of a batch gets the
result it gets alone (same points; only the order of FP64 sums may differ),
and sampled integrals of the full 4096-job workload match the CPU oracle."""
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


def _specs(n, seed, iters=4, nmax=6e4, prec_mix=True, eps=False):
    jobs = W.batch_jobs(n, seed=seed, nmin=2e3, nmax=nmax)
    specs = []
    for q, j in enumerate(jobs):
        s = dict(method=0, ndim=j["ndim"], family=j["family"], a=j["a"], u=j["u"],
                 seed=j["seed"], stream_id=j["stream_id"], nstart=j["nstart"],
                 maxeval=iters * j["nstart"], nbins=128,
                 flags=(q % 2) if prec_mix else 1)
        if eps:
            s.update(epsrel=10 ** (-2 - q % 3), nincrease=j["nstart"] // 2,
                     maxeval=40 * j["nstart"])
        specs.append(s)
    return specs


def _alone(cc, ctx, s):
    return cc.vegas(s["family"], s["a"], s["u"], ctx=ctx, flags=s["flags"], seed=s["seed"],
                    stream_id=s["stream_id"], nstart=s["nstart"], maxeval=s["maxeval"],
                    nbins=s["nbins"], epsrel=s.get("epsrel", 0.0),
                    nincrease=s.get("nincrease", 0))


def test_batch_equals_alone(cc, ctx):
    specs = _specs(48, 5)
    res = cc.vegas_batch(ctx, specs)
    for s, r in zip(specs, res):
        a = _alone(cc, ctx, s)
        assert r["status"] == 0 and r["neval"] == a["neval"] and r["fail"] == a["fail"]
        assert _rel(r["integral"], a["integral"]) < 1e-12
        assert _rel(r["error"], a["error"]) < 1e-12


def test_batch_with_convergence_drops_jobs(cc, ctx):
    specs = _specs(24, 9, eps=True)
    res = cc.vegas_batch(ctx, specs)
    conv = 0
    for s, r in zip(specs, res):
        a = _alone(cc, ctx, s)
        assert r["neval"] == a["neval"] and r["fail"] == a["fail"]
        assert _rel(r["integral"], a["integral"]) < 1e-12
        conv += r["fail"] == 0
    assert conv > 0


def test_batch_matches_oracle(cc, ctx):
    specs = _specs(12, 13, iters=3)
    res = cc.vegas_batch(ctx, specs)
    for s, r in zip(specs, res):
        o = O.vegas(O.genz(s["family"], s["a"], s["u"], precision=s["flags"]), s["ndim"],
                    flags=s["flags"], seed=s["seed"], stream_id=s["stream_id"],
                    nstart=s["nstart"], maxeval=s["maxeval"], nbins=128)
        tol = 1e-12 if s["flags"] == 0 else 1e-6
        assert _rel(r["integral"], o["integral"]) < tol
        assert _rel(r["error"], o["error"]) < (1e-12 if s["flags"] == 0 else 1e-5)


def test_invalid_job_gets_its_own_status(cc, ctx):
    specs = _specs(4, 3)
    specs[1] = dict(specs[1], nbins=1)
    specs[2] = dict(specs[2], method=1)
    res = cc.vegas_batch(ctx, specs)
    assert res[1]["status"] == cc.EINVAL and res[2]["status"] == cc.EINVAL
    assert res[0]["status"] == 0 and res[3]["status"] == 0


def test_full_4096_job_workload_sampled(cc, ctx):
    # 4096 integrals, d in 2..12, n log-uniform in [1e4, 1e6], 10 iterations,
    # FP32 evaluation: sampled integrals against the oracle's FP32 emulation
    jobs = W.batch_jobs(4096, seed=1000)
    specs = [dict(method=0, ndim=j["ndim"], family=j["family"], a=j["a"], u=j["u"],
                  seed=j["seed"], stream_id=j["stream_id"], nstart=j["nstart"],
                  maxeval=10 * j["nstart"], nbins=128, flags=1) for j in jobs]
    res = cc.vegas_batch(ctx, specs)
    assert all(r["status"] == 0 and r["neval"] == 10 * s["nstart"] for s, r in zip(specs, res))
    rng = np.random.default_rng(0)
    for q in rng.choice(4096, 6, replace=False):
        s, r = specs[q], res[q]
        if s["nstart"] > 3e5:
            continue
        o = O.vegas(O.genz(s["family"], s["a"], s["u"], precision=1), s["ndim"], flags=1,
                    seed=s["seed"], stream_id=s["stream_id"], nstart=s["nstart"],
                    maxeval=s["maxeval"], nbins=128)
        assert _rel(r["integral"], o["integral"]) < 1e-6


def test_autotuned_batch_equals_default(cc):
    # the tuner only changes launch settings: results agree to summation order
    jobs = W.batch_jobs(96, seed=77)
    specs = [dict(method=0, ndim=j["ndim"], family=j["family"], a=j["a"], u=j["u"],
                  seed=j["seed"], stream_id=j["stream_id"], nstart=j["nstart"],
                  maxeval=4 * j["nstart"], nbins=128, flags=cc.FP32_EVAL if q % 2 else 0)
             for q, j in enumerate(jobs)]
    c0 = cc.Context()
    base = cc.vegas_batch(c0, specs)
    c0.close()
    c1 = cc.Context()
    c1.config("autotune", 1)
    tuned = cc.vegas_batch(c1, specs)
    for prec in (cc.FP64, cc.FP32_EVAL):
        assert c1.config_get("blocks_per_cu", prec) in (2, 3, 4, 6)
        assert c1.config_get("ilp", prec) in (1, 2)
        assert c1.config_get("min_tile", prec) in (4096, 16384, 65536)
    c1.close()
    for r, b in zip(tuned, base):
        assert r["status"] == 0 and r["neval"] == b["neval"]
        assert _rel(r["integral"], b["integral"]) < 1e-12
        assert _rel(r["error"], b["error"]) < 1e-12



@pytest.mark.parametrize("eps", [False, True])
def test_two_halves_equal_one_stream(cc, eps):
    """The batch run as two halves on two streams (both launched from one
    thread when every job runs its budget, from two threads when jobs can
    stop early) gives each integral what the one-stream run gives, and in
    profile mode the sampling busy time (the union of the halves' launch
    intervals, which overlap) is positive and at most their summed time.
    The early-stopping jobs run up to 40 iterations; the values that fall
    outside the fixed-point window go to LDS FP64 adds, whose order varies
    from run to run, so their grids differ from a rerun's in the last bits
    and their (small) errors by up to ~1e-11 (1e-10 below), whatever the
    streams; the integral holds 1e-12."""
    specs = _specs(24, 11, eps=eps)
    out = {}
    for streams in (1, 2):
        c = cc.Context()
        c.config("batch_streams", streams)
        out[streams] = cc.vegas_batch(c, specs)
        c.close()
    for s, a, b in zip(specs, out[2], out[1]):
        assert a["status"] == 0 and a["neval"] == b["neval"] and a["fail"] == b["fail"]
        assert _rel(a["integral"], b["integral"]) < 1e-12
        # (FP32 evaluation: binary32 v^2 products summed in another order)
        tol = 1e-12 if s["flags"] == 0 and not eps else 1e-10
        assert _rel(a["error"], b["error"]) < tol, (s["flags"], a["error"], b["error"])
    import bench
    c = cc.Context()
    c.config("batch_streams", 2)
    c.config("profile", 1)
    bench._stats(cc, c)
    cc.vegas_batch(c, specs)
    st = bench._stats(cc, c)
    c.close()
    assert st.dosample_launches > 0 and st.dosample_ms > 0
    assert 0 < st.dosample_busy_ms <= st.dosample_ms * (1 + 1e-9)


def test_batch_streams_setting(cc):
    """batch_streams is a per-precision launch setting (2 by default), set for
    both precisions by ccuba_config and refused outside {1, 2}; a one-job
    batch never splits and gives the single call's result."""
    c = cc.Context()
    assert c.config_get("batch_streams", cc.FP32_EVAL) == 2
    assert c.config_get("batch_streams", cc.FP64) == 2
    c.config("batch_streams", 1)
    assert c.config_get("batch_streams", cc.FP32_EVAL) == 1
    assert c.config_get("batch_streams", cc.FP64) == 1
    for bad in (0, 3, -1):
        with pytest.raises(cc.CcubaError):
            c.config("batch_streams", bad)
    c.config("batch_streams", 2)
    s = _specs(1, 3, prec_mix=False)[0]
    r = cc.vegas_batch(c, [s])[0]
    a = _alone(cc, c, s)
    assert r["status"] == 0 and r["neval"] == a["neval"]
    assert _rel(r["integral"], a["integral"]) < 1e-12
    c.close()
