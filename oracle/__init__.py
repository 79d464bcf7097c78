"""ctypes binding of the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the plain serial FP64 integrator the HIP path is
checked against.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  It never imports the product package.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

FP64 = 0
FP32_EVAL = 1
FREEZE_GRID = 1 << 4
GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, C0 = range(5)

INTEGRAND_T = C.CFUNCTYPE(C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double),
                          C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_void_p,
                          C.POINTER(C.c_int), C.POINTER(C.c_int))


class _Genz(C.Structure):
    _fields_ = [("family", C.c_int), ("ndim", C.c_int),
                ("a", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_double)),
                ("precision", C.c_int)]


class _VegasTrace(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("n_iter", C.c_int),
                ("iter_I", C.POINTER(C.c_double)),
                ("iter_var", C.POINTER(C.c_double)),
                ("chi2", C.c_double), ("dof", C.c_int),
                ("grid", C.POINTER(C.c_double)),
                ("hist", C.POINTER(C.c_double))]


class _SuaveTrace(C.Structure):
    _fields_ = [("max_regions", C.c_int), ("max_splits", C.c_int),
                ("nregions", C.c_int), ("nsplits", C.c_int),
                ("chi2", C.c_double), ("dof", C.c_int),
                ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double)),
                ("I", C.POINTER(C.c_double)), ("var", C.POINTER(C.c_double)),
                ("inh_I", C.POINTER(C.c_double)), ("inh_var", C.POINTER(C.c_double)),
                ("grid", C.POINTER(C.c_double)), ("cut", C.POINTER(C.c_int))]


class _PartitionTrace(C.Structure):
    _fields_ = [("max_regions", C.c_int), ("max_splits", C.c_int),
                ("nregions", C.c_int), ("nsplits", C.c_int),
                ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double)),
                ("xmin", C.POINTER(C.c_double)), ("xmax", C.POINTER(C.c_double)),
                ("fmin", C.POINTER(C.c_double)), ("fmax", C.POINTER(C.c_double)),
                ("spread", C.POINTER(C.c_double)), ("cut", C.POINTER(C.c_int))]


class _CuhreTrace(C.Structure):
    _fields_ = [("n_batches", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # ORACLE_SANITIZE=1: the AddressSanitizer/UBSan build (oracle/sanitize.py)
        san = os.environ.get("ORACLE_SANITIZE") == "1"
        path = _build.SAN_LIB if san else _build.LIB
        if not os.path.exists(path):
            _build.build(sanitize=san)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
        L.oracle_genz_eval.argtypes = [C.POINTER(_Genz), dp]
        L.oracle_genz_eval.restype = C.c_double
        L.oracle_vegas_points.argtypes = [C.c_int, C.c_int, C.c_int, C.c_ulonglong,
                                          C.c_uint, C.c_int, dp, C.c_longlong,
                                          C.c_longlong, C.POINTER(C.c_uint32), dp, dp,
                                          C.POINTER(C.c_int)]
        L.oracle_vegas_refine_dim.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_vegas.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_double, C.c_double, C.c_int, C.c_ulonglong,
                                   C.c_longlong, C.c_longlong, C.c_longlong,
                                   C.c_longlong, C.c_longlong, C.c_int, C.c_uint,
                                   C.POINTER(C.c_longlong), C.POINTER(C.c_int), dp, dp,
                                   dp, C.POINTER(_VegasTrace)]
        L.oracle_vegas_from.argtypes = [dp] + L.oracle_vegas.argtypes
        L.oracle_gm_rule.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int, dp, dp,
                                     dp, dp, dp, C.POINTER(C.c_int), dp]
        L.oracle_gm_npoints.argtypes = [C.c_int]
        L.oracle_gm_npoints.restype = C.c_longlong
        L.oracle_cuhre.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_double, C.c_double, C.c_int, C.c_longlong,
                                   C.c_longlong, C.c_int, C.c_longlong,
                                   C.POINTER(C.c_int), C.POINTER(C.c_longlong),
                                   C.POINTER(C.c_int), dp, dp, dp,
                                   C.POINTER(_CuhreTrace)]
        L.oracle_suave.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_double, C.c_double, C.c_int, C.c_ulonglong,
                                   C.c_longlong, C.c_longlong, C.c_longlong, C.c_double,
                                   C.c_int, C.c_int, C.c_uint, C.POINTER(C.c_int),
                                   C.POINTER(C.c_longlong), C.POINTER(C.c_int), dp, dp, dp,
                                   C.POINTER(_SuaveTrace)]
        L.oracle_divonne_partition.argtypes = [
            C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_ulonglong, C.c_uint, C.c_int,
            C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int),
            C.POINTER(C.c_longlong), C.POINTER(C.c_int), dp, C.POINTER(_PartitionTrace)]
        L.oracle_gammainc_lower.argtypes = [C.c_double, C.c_double]
        L.oracle_gammainc_lower.restype = C.c_double
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox(ctr, key):
    """Philox4x32-10 block: four uint32 words."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


class Integrand:
    """Holds a ctypes integrand_t plus its userdata for the oracle calls."""

    def __init__(self, fn_ptr, userdata, keep=()):
        self.fn = fn_ptr
        self.userdata = userdata
        self._keep = keep


def genz(family, a, u, precision=FP64):
    """Built-in Genz integrand (C callback inside the oracle)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = _Genz(int(family), len(a), _dptr(a), _dptr(u), int(precision))
    fn = C.cast(lib().oracle_genz_integrand, C.c_void_p)
    return Integrand(fn, C.cast(C.pointer(g), C.c_void_p), keep=(a, u, g))


def python_integrand(func):
    """Wrap ``func(x[nvec, ndim]) -> f[nvec]`` or ``f[nvec, ncomp]`` (or -999 to
    abort) as integrand_t."""

    def cb(ndim, x, ncomp, f, userdata, nvec, core):
        nd, nv, nc = ndim[0], nvec[0], ncomp[0]
        xs = np.ctypeslib.as_array(x, shape=(nv * nd,)).reshape(nv, nd)
        r = func(xs.copy())
        if isinstance(r, int) and r == -999:
            return -999
        r = np.asarray(r, dtype=np.float64).reshape(nv, nc)
        fs = np.ctypeslib.as_array(f, shape=(nv * nc,))
        fs[:] = r.reshape(-1)
        return 0

    cfn = INTEGRAND_T(cb)
    return Integrand(C.cast(cfn, C.c_void_p), None, keep=(cfn,))


def genz_eval(family, a, u, x, precision=FP64):
    a = np.ascontiguousarray(a, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = _Genz(int(family), len(a), _dptr(a), _dptr(u), int(precision))
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    out = np.empty(x.shape[0])
    for p in range(x.shape[0]):
        row = np.ascontiguousarray(x[p])
        out[p] = lib().oracle_genz_eval(C.byref(g), _dptr(row))
    return out


def vegas_points(ndim, nbins, grid, seed, stream_id, iteration, i0, npts,
                 precision=FP64):
    grid = np.ascontiguousarray(grid, dtype=np.float64).reshape(ndim, nbins + 1)
    nblk = (ndim + 3) // 4
    words = np.zeros((npts, 4 * nblk), dtype=np.uint32)
    x = np.zeros((npts, ndim))
    w = np.zeros(npts)
    k = np.zeros((npts, ndim), dtype=np.int32)
    rc = lib().oracle_vegas_points(ndim, nbins, precision, seed, stream_id, iteration,
                                   _dptr(grid), i0, npts,
                                   words.ctypes.data_as(C.POINTER(C.c_uint32)),
                                   _dptr(x), _dptr(w),
                                   k.ctypes.data_as(C.POINTER(C.c_int)))
    if rc != 0:
        raise ValueError("oracle_vegas_points: bad arguments")
    return dict(words=words, x=x, w=w, bin=k)


def refine_dim(H, E):
    H = np.ascontiguousarray(H, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    out = np.zeros_like(E)
    lib().oracle_vegas_refine_dim(len(H), _dptr(H), _dptr(E), _dptr(out))
    return out


def vegas(integrand, ndim, *, epsrel=0.0, epsabs=0.0, flags=0, seed=1,
          mineval=0, maxeval=10**5, nstart=10**4, nincrease=0, nbatch=1000,
          nbins=128, stream_id=0, nvec=1000, max_iter=4096, ncomp=1, grid=None):
    """Serial Vegas.  With ncomp > 1 integral/error/prob are arrays of ncomp
    values; iter_I, iter_var, chi2, dof and the grid are component 0's.  grid
    (ndim x (nbins + 1)) starts the run from that grid instead of the uniform one."""
    gin = None
    if grid is not None:
        gin = np.ascontiguousarray(grid, dtype=np.float64).reshape(ndim * (nbins + 1))
    neval = C.c_longlong()
    fail = C.c_int()
    integral = np.zeros(ncomp)
    error = np.zeros(ncomp)
    prob = np.zeros(ncomp)
    It = np.zeros(max_iter)
    Vt = np.zeros(max_iter)
    grid = np.zeros(ndim * (nbins + 1))
    hist = np.zeros(ndim * nbins)
    tr = _VegasTrace(max_iter, 0, _dptr(It), _dptr(Vt), 0.0, 0, _dptr(grid), _dptr(hist))
    rc = lib().oracle_vegas_from(None if gin is None else _dptr(gin),
                                 ndim, ncomp, integrand.fn, integrand.userdata, nvec, epsrel,
                            epsabs, flags, seed, mineval, maxeval, nstart, nincrease,
                            nbatch, nbins, stream_id, C.byref(neval), C.byref(fail),
                            _dptr(integral), _dptr(error), _dptr(prob), C.byref(tr))
    if rc != 0:
        raise ValueError("oracle_vegas: bad arguments")
    n = tr.n_iter
    one = ncomp == 1
    return dict(neval=neval.value, fail=fail.value,
                integral=float(integral[0]) if one else integral.copy(),
                error=float(error[0]) if one else error.copy(),
                prob=float(prob[0]) if one else prob.copy(), iter_I=It[:n].copy(),
                iter_var=Vt[:n].copy(), chi2=tr.chi2, dof=tr.dof,
                grid=grid.reshape(ndim, nbins + 1), hist=hist.reshape(ndim, nbins))


def gm_npoints(ndim):
    return int(lib().oracle_gm_npoints(ndim))


def gm_rule(integrand, c, h, nvec=1000):
    c = np.ascontiguousarray(c, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    d = len(c)
    I7 = np.zeros(1)
    I5 = np.zeros(1)
    err = np.zeros(1)
    axis = C.c_int()
    dfour = np.zeros(d)
    rc = lib().oracle_gm_rule(d, integrand.fn, integrand.userdata, nvec, _dptr(c),
                              _dptr(h), _dptr(I7), _dptr(I5), _dptr(err),
                              C.byref(axis), _dptr(dfour))
    if rc != 0:
        raise ValueError("oracle_gm_rule: rc=%d" % rc)
    return dict(I7=float(I7[0]), I5=float(I5[0]), err=float(err[0]),
                axis=axis.value, dfour=dfour)


def cuhre(integrand, ndim, *, epsrel=1e-3, epsabs=0.0, flags=0, mineval=0,
          maxeval=10**7, key=7, max_regions_per_batch=10**5, nvec=1000):
    nreg = C.c_int()
    neval = C.c_longlong()
    fail = C.c_int()
    integral = np.zeros(1)
    error = np.zeros(1)
    prob = np.zeros(1)
    tr = _CuhreTrace(0)
    rc = lib().oracle_cuhre(ndim, 1, integrand.fn, integrand.userdata, nvec, epsrel,
                            epsabs, flags, mineval, maxeval, key,
                            max_regions_per_batch, C.byref(nreg), C.byref(neval),
                            C.byref(fail), _dptr(integral), _dptr(error), _dptr(prob),
                            C.byref(tr))
    if rc != 0:
        raise ValueError("oracle_cuhre: bad arguments")
    return dict(nregions=nreg.value, neval=neval.value, fail=fail.value,
                integral=float(integral[0]), error=float(error[0]),
                prob=float(prob[0]), n_batches=tr.n_batches)


def gammainc_lower(a, x):
    return float(lib().oracle_gammainc_lower(a, x))


def suave(integrand, ndim, *, epsrel=0.0, epsabs=0.0, flags=0, seed=1, mineval=0,
          maxeval=10**5, nnew=1000, flatness=25.0, nbins=128, nsplit=1, stream_id=0,
          nvec=1000):
    """Serial Suave (ncomp = 1).  Returns the results plus every region in
    position order (bounds, estimates, inherited estimates, grids) and the
    dimension of every split."""
    max_regions = 1 + max(0, maxeval // (2 * nnew))
    d, N = ndim, nbins
    lo = np.zeros((max_regions, d))
    hi = np.zeros((max_regions, d))
    I = np.zeros(max_regions)
    var = np.zeros(max_regions)
    inh_I = np.zeros(max_regions)
    inh_var = np.zeros(max_regions)
    grid = np.zeros((max_regions, d, N + 1))
    cut = np.zeros(max_regions, dtype=np.int32)
    tr = _SuaveTrace(max_regions, max_regions, 0, 0, 0.0, 0, _dptr(lo), _dptr(hi), _dptr(I),
                     _dptr(var), _dptr(inh_I), _dptr(inh_var), _dptr(grid),
                     cut.ctypes.data_as(C.POINTER(C.c_int)))
    nreg, neval, fail = C.c_int(), C.c_longlong(), C.c_int()
    integral, error, prob = np.zeros(1), np.zeros(1), np.zeros(1)
    rc = lib().oracle_suave(ndim, 1, integrand.fn, integrand.userdata, nvec, epsrel, epsabs,
                            flags, seed, mineval, maxeval, nnew, flatness, nbins, nsplit,
                            stream_id, C.byref(nreg), C.byref(neval), C.byref(fail),
                            _dptr(integral), _dptr(error), _dptr(prob), C.byref(tr))
    if rc != 0:
        raise ValueError("oracle_suave: bad arguments")
    R = nreg.value
    ns = tr.nsplits
    return dict(integral=float(integral[0]), error=float(error[0]), prob=float(prob[0]),
                neval=neval.value, fail=fail.value, nregions=R, chi2=tr.chi2, dof=tr.dof,
                lo=lo[:R].copy(), hi=hi[:R].copy(), I=I[:R].copy(), var=var[:R].copy(),
                inh_I=inh_I[:R].copy(), inh_var=inh_var[:R].copy(), grid=grid[:R].copy(),
                cut=cut[:ns].copy())


def divonne_partition(integrand, ndim, *, seed=1, stream_id=0, nsearch=256, niter=32,
                      maxregions=64, nsplit=1, spread_tol=0.0, nvec=1000):
    """Divonne's partitioning phase.  Returns the regions in position order with
    their extrema and spreads, and the dimension of every split."""
    d, m = ndim, maxregions
    arr = dict(lo=np.zeros((m, d)), hi=np.zeros((m, d)), xmin=np.zeros((m, d)),
               xmax=np.zeros((m, d)), fmin=np.zeros(m), fmax=np.zeros(m), spread=np.zeros(m),
               cut=np.zeros(m, dtype=np.int32))
    tr = _PartitionTrace(m, m, 0, 0, *[_dptr(arr[k]) for k in
                                       ("lo", "hi", "xmin", "xmax", "fmin", "fmax", "spread")],
                         arr["cut"].ctypes.data_as(C.POINTER(C.c_int)))
    nreg, neval, fail, tot = C.c_int(), C.c_longlong(), C.c_int(), C.c_double()
    rc = lib().oracle_divonne_partition(ndim, integrand.fn, integrand.userdata, nvec, seed,
                                        stream_id, nsearch, niter, maxregions, nsplit,
                                        spread_tol, C.byref(nreg), C.byref(neval),
                                        C.byref(fail), C.byref(tot), C.byref(tr))
    if rc != 0:
        raise ValueError("oracle_divonne_partition: bad arguments")
    R = nreg.value
    out = dict(nregions=R, neval=neval.value, fail=fail.value, total_spread=tot.value,
               cut=arr["cut"][:tr.nsplits].copy())
    for k in ("lo", "hi", "xmin", "xmax", "fmin", "fmax", "spread"):
        out[k] = arr[k][:R].copy()
    return out
