"""The accelerator batching example of Sect. 3.2.4 (tests/golden/
accelerator_batches.txt): 2400 points with p_accel = 1000 go out as batches
of 1000, 1000 and 400.  The oracle's integrand calls (CPU) and the device
path's caller-integrand batches (GPU) must both reproduce it."""
import os

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    out = []
    for line in open(os.path.join(HERE, "golden", "accelerator_batches.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        lhs, rhs = line.split("->")
        n, p = (int(v) for v in lhs.split())
        out.append((n, p, [int(v) for v in rhs.split()]))
    return out


def _recorder(sizes):
    def f(x):
        sizes.append(x.shape[0])
        return np.exp(-np.sum((x - 0.5) ** 2, axis=1))
    return f


@pytest.mark.parametrize("n,p,batches", _cases())
def test_oracle_sends_the_papers_batches(n, p, batches):
    sizes = []
    O.vegas(O.python_integrand(_recorder(sizes)), 3, nstart=n, maxeval=2 * n, nvec=p)
    assert sizes == batches * 2


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,batches", _cases())
def test_device_path_sends_the_papers_batches(n, p, batches):
    import paper_1408_6373_amd as cc
    ctx = cc.Context()
    try:
        sizes = []
        r = cc.vegas_batched(_recorder(sizes), 3, ctx=ctx, nvec=p, nstart=n, maxeval=2 * n,
                             nbins=32)
        assert sizes == batches * 2 and r["neval"] == 2 * n
    finally:
        ctx.close()
