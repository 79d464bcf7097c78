"""The context's device memory pool: blocks freed by one call serve the next,
under a small budget, without changing any result."""
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


def test_repeated_calls_of_changing_shapes_reuse_memory(cc):
    ctx = cc.Context(hbm_budget=256 << 20)
    shapes = [(1, 8, 10**6, 128, cc.FP32_EVAL), (0, 3, 20011, 50, cc.FP64),
              (2, 12, 300007, 128, cc.FP32_EVAL), (4, 5, 65536, 64, cc.FP64)]
    first = {}
    for rep in range(3):
        for fam, d, n, N, prec in shapes:
            a, u = W.genz_params(fam, d, 2)
            r = cc.vegas(fam, a, u, ctx=ctx, flags=prec, nbins=N, nstart=n, maxeval=4 * n)
            key = (fam, d)
            if rep == 0:
                first[key] = r
            else:
                assert r["neval"] == first[key]["neval"]
                assert _rel(r["integral"], first[key]["integral"]) < 1e-13
                assert _rel(r["error"], first[key]["error"]) < 1e-12
        a, u = W.genz_params(3, 4, 2)
        c = cc.cuhre(3, a, u, ctx=ctx, epsrel=1e-6, max_regions_per_batch=10**4)
        if rep == 0:
            first["cuhre"] = c
        else:
            assert c["neval"] == first["cuhre"]["neval"]
            assert c["nregions"] == first["cuhre"]["nregions"]
            assert _rel(c["integral"], first["cuhre"]["integral"]) < 1e-13
    ctx.close()


def test_tight_budget_falls_back_to_a_one_batch_store(cc):
    # 4 batches of regions would not fit in 8 MiB; one batch does
    ctx = cc.Context(hbm_budget=8 << 20)
    a, u = W.genz_params(3, 6, 1)
    r = cc.cuhre(3, a, u, ctx=ctx, epsrel=1e-4, maxeval=10**8, max_regions_per_batch=8000)
    assert r["fail"] in (0, 1) and r["neval"] > 0
    ctx.close()
