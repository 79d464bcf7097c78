"""The allocation-free DoSample entry point (ccuba_vegas_dosample_raw_noalloc)
against the allocating one (ccuba_vegas_dosample_raw) on the same inputs:
two calls in a row, the second on a smaller input, in both precisions.

The two take the same tiles here (the scratch holds their rows), so their
FP64 sums and every fixed-point histogram bin are the same numbers summed in
the same order: sums within 1e-13 relative, histograms within 1e-12
relative (the FP64 LDS histogram's adds come in another order).  The first
call's sums are also checked against the oracle's first iteration."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import paper_1408_6373_amd as cc
    return cc


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(b), 1e-300))


def _pass(cc, ctx, torch, fam, d, N, n, it, prec, grid, noalloc, stream):
    a, u = W.genz_params(fam, d, 3)
    g = torch.tensor(grid, dtype=torch.float64, device="cuda")
    sums = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    hist = torch.full((d * N,), -1.0, dtype=torch.float64, device="cuda")
    cc.vegas_dosample_raw(ctx, fam, a, u, N, it, n, g.data_ptr(), sums.data_ptr(),
                          hist.data_ptr(), stream_ptr=stream.cuda_stream, flags=prec, seed=7,
                          stream_id=2, noalloc=noalloc)
    stream.synchronize()
    return sums.cpu().numpy(), hist.cpu().numpy().reshape(d, N), (a, u)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_eval"])
def test_noalloc_equals_allocating_entry_point(cc, prec):
    import torch
    ctx = cc.Context()
    s = torch.cuda.Stream()
    rng = np.random.default_rng(11)
    try:
        # a large call, then a smaller one (fewer points, a smaller grid)
        for fam, d, N, n, it in ((1, 8, 128, 3_000_017, 4), (2, 5, 64, 40_009, 1)):
            w = rng.random((d, N)) + 0.2
            grid = np.zeros((d, N + 1))
            grid[:, 1:] = np.cumsum(w, axis=1) / w.sum(axis=1, keepdims=True)
            grid[:, -1] = 1.0
            s0, h0, (a, u) = _pass(cc, ctx, torch, fam, d, N, n, it, prec, grid, False, s)
            s1, h1, _ = _pass(cc, ctx, torch, fam, d, N, n, it, prec, grid, True, s)
            assert _rel(s1, s0) <= 1e-13, (fam, d, s1, s0)
            assert _rel(h1, h0) <= 1e-12, (fam, d)
            assert np.all(h1 >= 0.0)
    finally:
        ctx.close()


def test_noalloc_first_iteration_against_oracle(cc):
    import torch
    ctx = cc.Context()
    s = torch.cuda.Stream()
    try:
        d, N, n = 6, 128, 300_007
        grid = np.tile(np.arange(N + 1) / N, (d, 1))
        sums, hist, (a, u) = _pass(cc, ctx, torch, 4, d, N, n, 0, 0, grid, True, s)
        o = O.vegas(O.genz(4, a, u), d, nbins=N, nstart=n, maxeval=n, seed=7, stream_id=2)
        assert abs(sums[0] - o["iter_I"][0] * n) <= 1e-12 * abs(o["iter_I"][0] * n)
        assert _rel(hist, o["hist"]) <= 1e-12
    finally:
        ctx.close()
