"""The non-finite integrand rule (fail = -4): an integrand value that is not
finite makes the iteration's (or step's) sums non-finite, which ends the run
with fail -4 and zero results.  Pins on the oracle of every method."""
import numpy as np

import oracle as O


def _inf_low(x):
    return np.where(x[:, 0] < 0.01, np.inf, 1.0)


def test_vegas():
    r = O.vegas(O.python_integrand(_inf_low), 3, nstart=5000, maxeval=50000)
    assert r["fail"] == -4 and r["neval"] == 5000
    assert r["integral"] == 0 and r["error"] == 0 and r["prob"] == 0
    two = O.vegas(O.python_integrand(lambda x: np.stack([np.ones(len(x)), np.full(len(x), np.nan)], 1)),
                  2, ncomp=2, nstart=1000, maxeval=10000)
    assert two["fail"] == -4 and np.all(two["integral"] == 0)
    ok = O.vegas(O.python_integrand(lambda x: np.ones(len(x))), 3, nstart=5000, maxeval=50000)
    assert ok["fail"] == 0 and ok["integral"] == 1.0 and ok["error"] == 0.0


def test_cuhre():
    # the rule's centre point is (1/2, 1/2)
    f = O.python_integrand(lambda x: np.where(np.all(x == 0.5, axis=1), np.inf, 1.0))
    r = O.cuhre(f, 2, epsrel=1e-3, maxeval=10**5)
    assert r["fail"] == -4 and r["integral"] == 0 and r["error"] == 0
    assert r["neval"] == O.lib().oracle_gm_npoints(2)


def test_suave():
    r = O.suave(O.python_integrand(_inf_low), 3, nnew=2000, maxeval=50000)
    assert r["fail"] == -4 and r["neval"] == 2000 and r["nregions"] == 1
    assert r["integral"] == 0 and r["error"] == 0


def test_divonne_partition():
    # an infinite value becomes the maximum, and its spread is not finite
    r = O.divonne_partition(O.python_integrand(lambda x: np.where(x[:, 1] > 0.99, np.inf, 1.0)),
                            2, nsearch=512, niter=4, maxregions=50)
    assert r["fail"] == -4 and r["total_spread"] == 0.0
    # NaN compares false with everything: the extremum searches pass it by
    r = O.divonne_partition(O.python_integrand(lambda x: np.where(x[:, 1] > 0.99, np.nan, 1.0)),
                            2, nsearch=512, niter=4, maxregions=50)
    assert r["fail"] == 0 and r["total_spread"] == 0.0
