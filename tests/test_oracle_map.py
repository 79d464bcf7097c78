"""Pins of the oracle's point generation and grid map (uniform draw, map,
Jacobian; Lepage 1978 change of variables)."""
import numpy as np

import oracle as O


def _uniform_grid(d, N):
    return np.tile(np.arange(N + 1) / N, (d, 1))


def test_words_follow_counter_layout():
    d, N, seed, sid, t = 7, 50, 0x1234_5678_9ABC_DEF0, 11, 3
    p = O.vegas_points(d, N, _uniform_grid(d, N), seed, sid, t, 1000, 5)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for q in range(5):
        for b in range(2):
            want = O.philox([1000 + q, (t << 8) | b, sid, 0], key)
            assert list(p["words"][q, 4 * b:4 * b + 4]) == want


def test_fp64_uniform_is_exact_and_open():
    # on the uniform grid with N a power of two the map is the identity and
    # w == 1 exactly, so x exposes y: y * 2^32 - 1/2 must be the Philox word
    d, N = 8, 128
    p = O.vegas_points(d, N, _uniform_grid(d, N), 99, 0, 0, 0, 4096)
    y = p["x"]
    assert np.all(p["w"] == 1.0)
    assert np.all(y * 2.0**32 - 0.5 == p["words"][:, :d].astype(np.float64))
    assert np.all((y > 0) & (y < 1))
    assert np.all(p["bin"] == (p["words"][:, :d] >> 25))


def test_fp32_uniform_is_exact_and_open():
    d, N = 8, 128
    p = O.vegas_points(d, N, _uniform_grid(d, N), 99, 0, 0, 0, 4096, precision=O.FP32_EVAL)
    y = p["x"]
    assert np.all(p["w"] == 1.0)
    m = (p["words"][:, :d] >> 9).astype(np.float64)
    assert np.all(y * 2.0**23 - 0.5 == m)
    assert np.all((y > 0) & (y < 1))
    assert np.all(y.astype(np.float32).astype(np.float64) == y)


def test_extreme_words_stay_inside():
    # y of the largest and smallest words is strictly inside (0,1): checked
    # through the closed formula's endpoints on both precisions
    for prec in (O.FP64, O.FP32_EVAL):
        p = O.vegas_points(4, 2, _uniform_grid(4, 2), 5, 0, 0, 0, 20000, precision=prec)
        assert p["x"].min() > 0 and p["x"].max() < 1


def _random_grid(rng, d, N):
    g = np.zeros((d, N + 1))
    for j in range(d):
        w = rng.random(N) ** 3 + 1e-3
        g[j, 1:] = np.cumsum(w) / w.sum()
        g[j, -1] = 1.0
    return g


def test_map_on_adapted_grid_is_measure_preserving():
    # for any grid, E[w] = 1 and E[w g(x)] = int g: the map is a change of
    # variables with Jacobian w (statistical, 6 sigma)
    rng = np.random.default_rng(3)
    d, N, n = 3, 20, 200000
    g = _random_grid(rng, d, N)
    p = O.vegas_points(d, N, g, 7, 0, 0, 0, n)
    w, x = p["w"], p["x"]
    for vals, exact in ((w, 1.0), (w * x[:, 0] ** 2, 1 / 3),
                        (w * x[:, 1] * x[:, 2], 1 / 4)):
        assert abs(vals.mean() - exact) < 6 * vals.std() / np.sqrt(n)
    # every point lies in the bin the oracle reports
    for j in range(d):
        k = p["bin"][:, j]
        assert np.all(x[:, j] >= g[j, k]) and np.all(x[:, j] <= g[j, k + 1])


def test_fp32_map_close_to_fp64():
    rng = np.random.default_rng(4)
    d, N = 5, 50
    g = _random_grid(rng, d, N)
    p64 = O.vegas_points(d, N, g, 7, 1, 2, 0, 5000)
    p32 = O.vegas_points(d, N, g, 7, 1, 2, 0, 5000, precision=O.FP32_EVAL)
    assert np.max(np.abs(p64["x"] - p32["x"])) < 1e-6
    # FP32 edges carry an absolute rounding of at most 2^-25 each, so a bin
    # width (and the Jacobian factor) moves by at most 3 2^-25 / width; w also
    # jumps where the precisions put a coordinate in adjacent bins, which is
    # rare (|y32 - y64| <= 2^-24)
    widths = np.take_along_axis(np.diff(g, axis=1), p64["bin"].T, axis=1).T
    bound = (3 * 2.0**-25 / widths).sum(axis=1) + d * 2.0**-23
    rel = np.abs(p64["w"] / p32["w"] - 1)
    assert np.mean(rel > bound) < 1e-3
