"""Pins of the oracle's grid refinement (Lepage 1978).  The smoothing and
damping constants are a reading (3-point smoothing, alpha = 1.5), so what is
pinned is the set of invariants any correct rebinning must keep; beyond these
the refinement is parity unpinned."""
import numpy as np

import oracle as O


def _mass_density(H):
    # the damped, smoothed weights m_k recomputed from their definition
    N = len(H)
    d = np.empty(N)
    d[0] = (H[0] + H[1]) / 2
    d[-1] = (H[-2] + H[-1]) / 2
    d[1:-1] = (H[:-2] + H[1:-1] + H[2:]) / 3
    r = d / d.sum()
    m = np.zeros(N)
    nz = r > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        m[nz] = np.where(r[nz] == 1, 1.0, ((r[nz] - 1) / np.log(r[nz])) ** 1.5)
    return m


def test_invariants_random_histograms():
    rng = np.random.default_rng(0)
    for N in (2, 3, 50, 128, 256):
        E = np.concatenate([[0.0], np.sort(rng.random(N - 1)), [1.0]])
        H = rng.random(N) ** 4
        En = O.refine_dim(H, E)
        assert En[0] == 0.0 and En[-1] == 1.0
        assert np.all(np.diff(En) >= 0)
        # each new bin holds the same share of sum m, with m_k spread
        # uniformly over old bin k: integrate the piecewise-constant density
        m = _mass_density(H)
        dens = m / np.diff(E)
        cum = np.concatenate([[0.0], np.cumsum(m)])
        def M(x):
            k = np.clip(np.searchsorted(E, x, side="right") - 1, 0, N - 1)
            return cum[k] + dens[k] * (x - E[k])
        shares = np.diff([M(x) for x in En])
        assert np.allclose(shares, m.sum() / N, rtol=1e-10, atol=1e-13 * m.sum())


def test_uniform_histogram_keeps_grid():
    N = 64
    E = np.concatenate([[0.0], np.sort(np.random.default_rng(1).random(N - 1)), [1.0]])
    # a flat histogram on a uniform grid leaves the uniform grid
    U = np.arange(N + 1) / N
    assert np.allclose(O.refine_dim(np.ones(N), U), U, atol=1e-15)
    # an all-zero histogram leaves any grid unchanged
    assert np.array_equal(O.refine_dim(np.zeros(N), E), E)


def test_concentrates_where_the_histogram_is():
    N = 50
    U = np.arange(N + 1) / N
    H = np.zeros(N)
    H[10] = 1.0
    En = O.refine_dim(H, U)
    # bins 9..11 carry mass after smoothing; most new edges fall inside them
    inside = np.sum((En > U[9]) & (En < U[12]))
    assert inside > N // 2


def test_mirror_symmetry():
    # The refinement has no preferred direction: reflecting the grid and the
    # histogram (x -> 1 - x) reflects the refined grid.  A one-sided
    # smoothing or an edge placed from the wrong end breaks this.
    rng = np.random.default_rng(2)
    for N in (3, 7, 64, 129):
        E = np.concatenate([[0.0], np.sort(rng.random(N - 1)), [1.0]])
        H = rng.random(N) ** 3
        En = O.refine_dim(H, E)
        Er = O.refine_dim(H[::-1].copy(), (1.0 - E[::-1]).copy())
        assert np.allclose(Er, 1.0 - En[::-1], atol=1e-13)


def test_scale_invariance():
    # Only the histogram's shape steers the grid: scaling it by any positive
    # factor leaves the refined grid unchanged (the damping acts on the
    # normalized weights).  Powers of two scale exactly.
    rng = np.random.default_rng(3)
    N = 100
    E = np.concatenate([[0.0], np.sort(rng.random(N - 1)), [1.0]])
    H = rng.random(N) ** 2
    En = O.refine_dim(H, E)
    for c in (2.0 ** -40, 0.5, 8.0, 2.0 ** 60):
        assert np.array_equal(O.refine_dim(H * c, E), En)
    assert np.allclose(O.refine_dim(H * 3.7, E), En, atol=1e-14)
