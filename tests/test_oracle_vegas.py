"""Pins of the oracle's Vegas: closed-form integrals (statistical), the
zero-variance invariant on a frozen grid, chi^2 calibration, and the paper's
interface semantics (nvec, -999 abort, nbatch, mineval/maxeval)."""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from closed_forms import exact
import workloads as W


@pytest.mark.parametrize("fam", [0, 1, 2, 4])
def test_closed_forms_within_4_sigma(fam):
    zs = []
    for seed in range(1, 21):
        a, u = W.genz_params(fam, 4, seed)
        r = O.vegas(O.genz(fam, a, u), 4, nbins=50, nstart=5000, maxeval=5 * 5000, seed=seed)
        assert r["fail"] == 1 and r["neval"] == 25000
        z = (r["integral"] - exact(fam, a, u)) / r["error"]
        zs.append(z)
        assert abs(z) < 4.5
    zs = np.array(zs)
    # the z-scores of an unbiased estimator with a correct error are ~N(0,1)
    assert abs(zs.mean()) < 1.0 and 0.4 < zs.std() < 1.8


def test_corner_peak_d6():
    a, u = W.genz_params(3, 6, 5)
    r = O.vegas(O.genz(3, a, u), 6, nstart=20000, maxeval=10 * 20000, seed=3)
    assert abs(r["integral"] - exact(3, a, u)) < 4.5 * r["error"]


def test_fp32_eval_close_to_fp64():
    a, u = W.genz_params(2, 8, 1)
    r64 = O.vegas(O.genz(2, a, u), 8, nstart=20000, maxeval=5 * 20000, seed=2)
    r32 = O.vegas(O.genz(2, a, u, precision=O.FP32_EVAL), 8, nstart=20000,
                  maxeval=5 * 20000, seed=2, flags=O.FP32_EVAL)
    assert abs(r32["integral"] / r64["integral"] - 1) < 1e-5
    assert abs(r32["error"] / r64["error"] - 1) < 1e-3


def test_zero_variance_on_frozen_grid():
    # f = 1, N a power of two and a frozen (uniform) grid: every v is exactly
    # 1, so S1 = S2 = n, every sigma_t = 0 and the result is exactly 1
    one = O.python_integrand(lambda x: np.ones(len(x)))
    for prec in (O.FP64, O.FP32_EVAL):
        r = O.vegas(one, 3, nbins=128, nstart=4096, maxeval=3 * 4096,
                    flags=O.FREEZE_GRID | prec, nvec=4096)
        assert r["integral"] == 1.0 and r["error"] == 0.0
        assert np.all(r["iter_var"] == 0.0) and np.all(r["iter_I"] == 1.0)


def test_chi2_probability_is_calibrated():
    # with a frozen grid the iterations are independent draws of the same
    # estimator, so prob = P(chi^2 <= observed) is uniform on [0,1]
    probs = []
    for seed in range(40):
        a, u = W.genz_params(0, 3, seed)
        r = O.vegas(O.genz(0, a, u), 3, nbins=16, nstart=2000, maxeval=6 * 2000,
                    seed=seed, flags=O.FREEZE_GRID)
        assert r["dof"] == 5
        probs.append(r["prob"])
    assert stats.kstest(probs, "uniform").pvalue > 1e-3


def test_gauss_legendre_d2():
    # brute force at d = 2 with 64x64 Gauss-Legendre nodes of the same f
    x, w = np.polynomial.legendre.leggauss(64)
    x = (x + 1) / 2
    w = w / 2
    a, u = W.genz_params(2, 2, 9)
    X0, X1 = np.meshgrid(x, x, indexing="ij")
    f = O.genz_eval(2, a, u, np.stack([X0.ravel(), X1.ravel()], 1))
    I_gl = float((np.outer(w, w).ravel() * f).sum())
    r = O.vegas(O.genz(2, a, u), 2, nstart=20000, maxeval=8 * 20000, seed=4)
    assert abs(r["integral"] - I_gl) < 4.5 * r["error"]


def test_nvec_does_not_change_results():
    a, u = W.genz_params(1, 5, 2)
    base = None
    for nvec in (1, 7, 1000):
        r = O.vegas(O.genz(1, a, u), 5, nstart=3000, maxeval=3 * 3000, nvec=nvec)
        key = (r["integral"], r["error"], r["prob"])
        base = base or key
        assert key == base


def test_nvec_batches_seen_by_integrand():
    seen = []

    def f(x):
        seen.append(len(x))
        return np.ones(len(x))

    O.vegas(O.python_integrand(f), 2, nstart=2500, maxeval=2500, nvec=1000)
    assert seen == [1000, 1000, 500]


def test_nbatch_does_not_change_results():
    a, u = W.genz_params(0, 3, 2)
    r1 = O.vegas(O.genz(0, a, u), 3, nstart=3000, maxeval=6000, nbatch=1)
    r2 = O.vegas(O.genz(0, a, u), 3, nstart=3000, maxeval=6000, nbatch=10**6)
    assert r1["integral"] == r2["integral"] and r1["error"] == r2["error"]


def test_abort_minus_999():
    calls = []

    def f(x):
        calls.append(1)
        if len(calls) == 3:
            return -999
        return np.ones(len(x))

    r = O.vegas(O.python_integrand(f), 2, nstart=5000, maxeval=10**5, nvec=1000)
    assert r["fail"] == -99 and len(calls) == 3 and r["neval"] == 3000


def test_epsrel_stops_and_mineval():
    a, u = W.genz_params(0, 2, 1)
    r = O.vegas(O.genz(0, a, u), 2, epsrel=1e-3, nstart=5000, nincrease=1000,
                maxeval=10**7)
    assert r["fail"] == 0 and r["error"] <= 1e-3 * abs(r["integral"])
    # n_t = nstart + t nincrease
    T = len(r["iter_I"])
    assert r["neval"] == sum(5000 + 1000 * t for t in range(T))
    r2 = O.vegas(O.genz(0, a, u), 2, epsrel=1e-3, nstart=5000, nincrease=1000,
                 maxeval=10**7, mineval=r["neval"] + 1)
    assert r2["neval"] > r["neval"]


def test_maxeval_stops_before_overrun():
    a, u = W.genz_params(0, 2, 1)
    r = O.vegas(O.genz(0, a, u), 2, epsrel=0, nstart=1000, maxeval=3500)
    assert r["fail"] == 1 and r["neval"] == 3000 and len(r["iter_I"]) == 3
    # a constant on the first (uniform) grid has zero variance, which meets
    # any tolerance, including epsrel = epsabs = 0, after one iteration
    one = O.python_integrand(lambda x: np.ones(len(x)))
    r = O.vegas(one, 2, epsrel=0, nstart=1024, maxeval=4096)
    assert r["fail"] == 0 and r["neval"] == 1024 and r["error"] == 0.0


def test_stream_id_and_seed_change_points():
    a, u = W.genz_params(0, 3, 1)
    base = O.vegas(O.genz(0, a, u), 3, nstart=2000, maxeval=2000)
    assert O.vegas(O.genz(0, a, u), 3, nstart=2000, maxeval=2000, seed=2)["integral"] != base["integral"]
    assert O.vegas(O.genz(0, a, u), 3, nstart=2000, maxeval=2000, stream_id=1)["integral"] != base["integral"]


def test_bad_arguments():
    one = O.python_integrand(lambda x: np.ones(len(x)))
    for kw in (dict(nbins=1), dict(nbins=257), dict(nstart=1)):
        with pytest.raises(ValueError):
            O.vegas(one, 2, **kw)
    with pytest.raises(ValueError):
        O.vegas(one, 17)


# ---------------------------------------------------------------------------
# Several components (ncomp > 1): one set of points, per-component sums,
# results and chi^2, the grid adapted to component 0, and an accuracy test
# that needs every component.

def _genz_py(fam, a, u):
    return lambda x: O.genz_eval(fam, a, u, x)


def test_components_scaled_by_two_are_exactly_twice():
    # v_1 = w (2 g) = 2 v_0 exactly, so every sum, estimate, weight and error
    # scales by a power of two (exact in binary floating point)
    a, u = W.genz_params(1, 3, 4)
    g = _genz_py(1, a, u)
    one = O.vegas(O.python_integrand(g), 3, nstart=2000, maxeval=10000, nbins=32)
    two = O.vegas(O.python_integrand(lambda x: np.stack([g(x), 2.0 * g(x)], 1)), 3,
                  nstart=2000, maxeval=10000, nbins=32, ncomp=2)
    assert two["integral"][0] == one["integral"] and two["error"][0] == one["error"]
    assert two["integral"][1] == 2.0 * two["integral"][0]
    assert two["error"][1] == 2.0 * two["error"][0]
    assert two["prob"][1] == two["prob"][0]
    assert np.array_equal(two["grid"], one["grid"])  # component 0 drives the grid
    assert np.array_equal(two["iter_I"], one["iter_I"])


def test_constant_component_is_exact():
    # on the first (uniform) grid every weight is exactly 1, so a constant
    # component has zero variance there, and the combination of a
    # zero-variance iteration is exact: 1 with error 0, whatever the grid
    # does afterwards
    a, u = W.genz_params(0, 4, 5)
    g = _genz_py(0, a, u)
    r = O.vegas(O.python_integrand(lambda x: np.stack([g(x), np.ones(len(x))], 1)), 4,
                nstart=1000, maxeval=5000, nbins=16, ncomp=2)
    assert r["integral"][1] == 1.0 and r["error"][1] == 0.0 and r["prob"][1] == 0.0
    assert r["neval"] == 5000 and r["fail"] == 1  # component 0 never met epsrel = 0


def test_every_component_must_converge():
    # component 0 alone stops early; a hard second component keeps the run
    # going, and component 0's iterations are the same as far as both go
    a, u = W.genz_params(2, 2, 6)
    g = _genz_py(2, a, u)
    h = lambda x: g(x) ** 1.5  # the same peak, sharper: needs more points
    alone = O.vegas(O.python_integrand(g), 2, epsrel=1e-3, nstart=2000, maxeval=10**6,
                    nbins=32)
    both = O.vegas(O.python_integrand(lambda x: np.stack([g(x), h(x)], 1)), 2,
                   epsrel=1e-3, nstart=2000, maxeval=10**6, nbins=32, ncomp=2)
    n1 = len(alone["iter_I"])
    assert alone["fail"] == 0 and both["fail"] == 0
    assert len(both["iter_I"]) > n1
    assert np.array_equal(both["iter_I"][:n1], alone["iter_I"])
    for c in range(2):
        assert both["error"][c] <= 1e-3 * abs(both["integral"][c])


def test_abort_reports_every_component_zero():
    calls = []

    def f(x):
        calls.append(1)
        return -999 if len(calls) == 2 else np.ones((len(x), 3))

    r = O.vegas(O.python_integrand(f), 2, nstart=3000, maxeval=10**5, nvec=1000, ncomp=3)
    assert r["fail"] == -99 and r["neval"] == 2000
    assert np.all(r["integral"] == 0) and np.all(r["error"] == 0)


# ---------------------------------------------------------------------------
# A run started from a given grid (a grid reused from an earlier integration)

def test_uniform_start_grid_is_the_ordinary_run():
    a, u = W.genz_params(1, 3, 8)
    N = 32
    uni = np.tile(np.arange(N + 1) / N, (3, 1))
    r0 = O.vegas(O.genz(1, a, u), 3, nstart=3000, maxeval=9000, nbins=N)
    r1 = O.vegas(O.genz(1, a, u), 3, nstart=3000, maxeval=9000, nbins=N, grid=uni)
    assert r0["integral"] == r1["integral"] and r0["error"] == r1["error"]
    assert np.array_equal(r0["grid"], r1["grid"])


def test_first_iteration_from_a_grid_is_the_plain_mean():
    # iteration 0 from grid G: I_0 = (1/n) sum w f over the points mapped
    # through G, sigma_0^2 from the same sum of squares (brute force here)
    import math
    d, N, n = 3, 16, 4000
    a, u = W.genz_params(0, d, 9)
    prev = O.vegas(O.genz(0, a, u), d, nstart=2000, maxeval=6000, nbins=N)
    G = prev["grid"]
    r = O.vegas(O.genz(0, a, u), d, nstart=n, maxeval=n, nbins=N, grid=G, seed=3)
    pts = O.vegas_points(d, N, G, 3, 0, 0, 0, n)
    v = pts["w"] * O.genz_eval(0, a, u, pts["x"])
    I = math.fsum(v) / n
    var = (math.fsum(v * v) / n - I * I) / (n - 1)
    assert abs(r["iter_I"][0] - I) <= 1e-15 * abs(I)
    assert abs(r["iter_var"][0] - var) <= 1e-12 * var


@pytest.mark.parametrize("t", [4, 8])
def test_later_iteration_variance_is_the_sample_variance(t):
    # iteration t of a product peak in d = 8 whose grid has adapted, so that
    # the variance is about 1/2000 of the mean of v^2: I_t and sigma_t^2 equal
    # the mean and the two-pass sample variance of the iteration's v = w f,
    # summed by brute force (math.fsum) over the points mapped through the
    # grid that enters iteration t.  Evaluating sigma_t^2 from plain sums of v
    # and v^2 loses about 3 of its digits to cancellation here (off by about
    # 1e-13); the bar 1e-14 needs the cancellation-free form.
    import math
    d, N, n, seed = 8, 64, 100000, 5
    a, u = W.genz_params(2, d, 1)
    G = O.vegas(O.genz(2, a, u), d, nstart=n, maxeval=t * n, nbins=N, seed=seed)["grid"]
    r = O.vegas(O.genz(2, a, u), d, nstart=n, maxeval=(t + 1) * n, nbins=N, seed=seed)
    pts = O.vegas_points(d, N, G, seed, 0, t, 0, n)
    v = pts["w"] * O.genz_eval(2, a, u, pts["x"])
    I = math.fsum(v) / n
    dv = v - I
    var = (math.fsum(dv * dv) / n - (math.fsum(dv) / n) ** 2) / (n - 1)
    assert math.fsum(v * v) / n > 1000 * var * (n - 1)  # the cancellation is there
    assert abs(r["iter_I"][t] - I) <= 1e-15 * abs(I)
    assert abs(r["iter_var"][t] - var) <= 1e-14 * var
