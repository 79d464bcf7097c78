"""Seeded synthetic workloads: Genz-family parameters, batch job lists and
serving arrival streams.

This module holds none of the integration method's arithmetic.  It draws the
inputs that the device library and the CPU oracle are both given, with numpy's
PCG64 generator keyed by (seed, job), so that a workload is reproduced
exactly from its seed.

Families (Genz 1987): 0 Gaussian, 1 oscillatory, 2 product peak,
3 corner peak, 4 C0.  Parameter recipe:
  * Gaussian: a_i = 5, u_i ~ U(0,1);
  * oscillatory, product peak, C0: r_i ~ U(0,1), a_i = 9 r_i / sum r (so the
    a_i sum to 9, mean 9/d), u_i ~ U(0,1);
  * corner peak: a_i = 5 r_i / sum r, u unused (zeros);
  * oscillatory: u_1 is drawn again while |cos(2 pi u_1 + sum a / 2)| < 0.1,
    so that the integral stays away from zero and a relative target is
    reachable.
"""
import math

import numpy as np

GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, C0 = range(5)
FAMILY_NAMES = ["gaussian", "oscillatory", "product_peak", "corner_peak", "c0"]


def _rng(seed, job=0, stream=0):
    return np.random.Generator(np.random.PCG64([int(seed), int(job), int(stream)]))


def genz_params(family, ndim, seed, job=0):
    """Return (a, u) float64 arrays of length ndim for one integrand."""
    rng = _rng(seed, job, 1)
    r = rng.random(ndim)
    u = rng.random(ndim)
    if family == GAUSSIAN:
        a = np.full(ndim, 5.0)
    elif family == CORNER_PEAK:
        a = 5.0 * r / r.sum()
        u = np.zeros(ndim)
    else:
        a = 9.0 * r / r.sum()
    if family == OSCILLATORY:
        half = a.sum() / 2.0
        while abs(math.cos(2.0 * math.pi * u[0] + half)) < 0.1:
            u[0] = rng.random()
    return a.astype(np.float64), u.astype(np.float64)


def batch_jobs(njobs=4096, seed=1000, dmin=2, dmax=12, nmin=1e4, nmax=1e6,
               families=(GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, C0)):
    """Independent Vegas jobs: d ~ U{dmin..dmax}, points per iteration
    log-uniform in [nmin, nmax], family uniform over ``families``; job j has
    parameter seed ``seed + j``."""
    rng = _rng(seed, 0, 2)
    jobs = []
    for j in range(njobs):
        d = int(rng.integers(dmin, dmax + 1))
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        fam = int(families[rng.integers(0, len(families))])
        a, u = genz_params(fam, d, seed + j, j)
        jobs.append(dict(ndim=d, nstart=n, family=fam, a=a, u=u, seed=seed + j,
                         stream_id=j))
    return jobs


def serving_requests(count, rate, seed=7, dmin=2, dmax=16, vegas_share=0.7,
                     eps_lo=1e-5, eps_hi=1e-3):
    """Poisson arrivals at ``rate`` requests/s.  Each request: method Vegas
    (probability ``vegas_share``) or Cuhre, d ~ U{dmin..dmax}, target relative
    error log-uniform in [eps_lo, eps_hi], a Genz family and its parameters
    (Vegas: Gaussian/oscillatory/product peak/C0; Cuhre: all five)."""
    rng = _rng(seed, 0, 3)
    t = 0.0
    reqs = []
    for q in range(count):
        t += rng.exponential(1.0 / rate)
        method = 0 if rng.random() < vegas_share else 1
        d = int(rng.integers(dmin, dmax + 1))
        eps = math.exp(rng.uniform(math.log(eps_lo), math.log(eps_hi)))
        fams = (GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, C0) if method == 0 else (
            GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, C0)
        fam = int(fams[rng.integers(0, len(fams))])
        a, u = genz_params(fam, d, seed * 100003 + q, q)
        reqs.append(dict(arrival=t, method=method, ndim=d, epsrel=eps, family=fam,
                         a=a, u=u, seed=seed * 100003 + q, stream_id=q))
    return reqs
