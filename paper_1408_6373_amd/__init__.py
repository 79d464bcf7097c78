"""Python binding of libccuba (include/ccuba.h): argument marshalling only.

Every step of the integration runs in the HIP library; this module converts
Python/numpy arguments to the C ABI and back.  It raises at import time if
``libccuba.so`` has not been built: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

try:
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one; loading it first makes the process use a single runtime, so that
    # device pointers and streams from torch are valid in the library.
    import torch  # noqa: F401
except ImportError:  # the library itself does not need torch
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccuba.so")

OK, EINVAL, EHIP, ENOMEM, ENOENT, ESTATE = 0, -1, -2, -3, -4, -5
GAUSSIAN, OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, C0 = range(5)
FP64, FP32_EVAL, FREEZE_GRID = 0, 1, 1 << 4

if not os.path.exists(LIB_PATH):
    raise ImportError("libccuba.so is not built: run `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (or paper_1408_6373_amd/build.py) first")

_lib = C.CDLL(LIB_PATH)
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_llp = C.POINTER(C.c_longlong)


class Integrand(C.Structure):
    _fields_ = [("family", C.c_int), ("a", _dp), ("u", _dp)]


class VegasTrace(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("n_iter", C.c_int), ("iter_I", _dp),
                ("iter_var", _dp), ("chi2", C.c_double), ("dof", C.c_int), ("grid", _dp)]


class Job(C.Structure):
    _fields_ = [("method", C.c_int), ("ndim", C.c_int), ("f", Integrand),
                ("epsrel", C.c_double), ("epsabs", C.c_double), ("flags", C.c_int),
                ("seed", C.c_ulonglong), ("stream_id", C.c_uint),
                ("mineval", C.c_longlong), ("maxeval", C.c_longlong),
                ("nstart", C.c_longlong), ("nincrease", C.c_longlong),
                ("nbins", C.c_int), ("max_regions_per_batch", C.c_longlong)]


class Result(C.Structure):
    _fields_ = [("neval", C.c_longlong), ("nregions", C.c_int), ("fail", C.c_int),
                ("status", C.c_int), ("integral", C.c_double), ("error", C.c_double),
                ("prob", C.c_double), ("t_submit", C.c_double), ("t_done", C.c_double)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_CTXP = C.c_void_p
_sig("ccuba_init", C.c_int, [C.POINTER(_CTXP), C.c_int, C.c_size_t])
_sig("ccuba_shutdown", C.c_int, [C.POINTER(_CTXP)])
_sig("ccuba_config", C.c_int, [_CTXP, C.c_char_p, C.c_longlong])
_sig("ccuba_config_get", C.c_int, [_CTXP, C.c_char_p, C.c_int, C.POINTER(C.c_longlong)])
_sig("ccuba_strerror", C.c_char_p, [C.c_int])
_VEGAS_ARGS = [C.POINTER(_CTXP), C.c_int, C.c_int, C.POINTER(Integrand), C.c_double,
               C.c_double, C.c_int, C.c_ulonglong, C.c_longlong, C.c_longlong, C.c_longlong,
               C.c_longlong, C.c_longlong, C.c_int, C.c_uint, _llp, _ip, _dp, _dp, _dp]
_sig("ccuba_vegas", C.c_int, _VEGAS_ARGS)
_sig("ccuba_vegas_ex", C.c_int, _VEGAS_ARGS + [C.POINTER(VegasTrace)])
_sig("ccuba_vegas_stateful", C.c_int, _VEGAS_ARGS[:13] + [C.c_int, C.c_char_p] +
     _VEGAS_ARGS[13:] + [C.POINTER(VegasTrace)])
_sig("ccuba_vegas_points", C.c_int, [_CTXP, C.c_int, C.c_int, C.c_int, C.c_ulonglong, C.c_uint,
                                     C.c_int, _dp, C.c_longlong, C.c_longlong,
                                     C.POINTER(C.c_uint32), _dp, _dp, _ip])
_sig("ccuba_vegas_refine", C.c_int, [_CTXP, C.c_int, C.c_int, _dp, _dp, _dp])
_RAW_ARGS = [_CTXP, C.c_int, C.c_int, C.POINTER(Integrand), C.c_int, C.c_ulonglong, C.c_uint,
             C.c_int, C.c_longlong, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_sig("ccuba_vegas_dosample_raw", C.c_int, _RAW_ARGS)
_sig("ccuba_vegas_dosample_raw_noalloc", C.c_int, _RAW_ARGS)
_sig("ccuba_vegas_batch", C.c_int, [_CTXP, C.c_int, C.POINTER(Job), C.POINTER(Result)])
_sig("ccuba_vegas_source", C.c_int, [C.POINTER(_CTXP), C.c_int, C.c_char_p, _dp, _dp,
                                     C.c_double, C.c_double, C.c_int, C.c_ulonglong,
                                     C.c_longlong, C.c_longlong, C.c_longlong, C.c_longlong,
                                     C.c_longlong, C.c_int, C.c_uint, _llp, _ip, _dp, _dp, _dp])
_sig("ccuba_rtc_log", C.c_int, [_CTXP, C.c_char_p, C.c_size_t])
# int integrand(const int *ndim, const double x[], const int *ncomp, double f[],
#               void *userdata, const int *nvec, const int *core)
BATCH_INTEGRAND = C.CFUNCTYPE(C.c_int, _ip, C.c_void_p, _ip, C.c_void_p, C.c_void_p, _ip, _ip)
POINTS_HOST, POINTS_DEVICE = 0, 1
_sig("ccuba_vegas_batched", C.c_int, [C.POINTER(_CTXP), C.c_int, C.c_int, BATCH_INTEGRAND,
                                      C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                      C.c_int, C.c_ulonglong, C.c_longlong, C.c_longlong,
                                      C.c_longlong, C.c_longlong, C.c_int, C.c_uint, _llp, _ip,
                                      _dp, _dp, _dp])
if hasattr(_lib, "ccuba_cuhre"):
    _sig("ccuba_cuhre", C.c_int, [C.POINTER(_CTXP), C.c_int, C.c_int, C.POINTER(Integrand),
                                  C.c_double, C.c_double, C.c_int, C.c_longlong, C.c_longlong,
                                  C.c_int, C.c_longlong, _ip, _llp, _ip, _dp, _dp, _dp])
    _sig("ccuba_cuhre_rule", C.c_int, [_CTXP, C.c_int, C.POINTER(Integrand), C.c_longlong,
                                       _dp, _dp, _dp, _dp, _dp, _ip])


class SuaveTrace(C.Structure):
    _fields_ = [("max_regions", C.c_int), ("max_splits", C.c_int), ("nregions", C.c_int),
                ("nsplits", C.c_int), ("chi2", C.c_double), ("dof", C.c_int),
                ("lo", _dp), ("hi", _dp), ("I", _dp), ("var", _dp), ("grid", _dp),
                ("cut", _ip)]


if hasattr(_lib, "ccuba_suave"):
    _sig("ccuba_suave", C.c_int, [C.POINTER(_CTXP), C.c_int, C.c_int, C.POINTER(Integrand),
                                  C.c_double, C.c_double, C.c_int, C.c_ulonglong,
                                  C.c_longlong, C.c_longlong, C.c_longlong, C.c_double,
                                  C.c_int, C.c_int, C.c_uint, _ip, _llp, _ip, _dp, _dp, _dp,
                                  C.POINTER(SuaveTrace)])


class PartitionTrace(C.Structure):
    _fields_ = [("max_regions", C.c_int), ("max_splits", C.c_int), ("nregions", C.c_int),
                ("nsplits", C.c_int), ("lo", _dp), ("hi", _dp), ("xmin", _dp), ("xmax", _dp),
                ("fmin", _dp), ("fmax", _dp), ("spread", _dp), ("cut", _ip)]


if hasattr(_lib, "ccuba_divonne_partition"):
    _sig("ccuba_divonne_partition", C.c_int,
         [C.POINTER(_CTXP), C.c_int, C.POINTER(Integrand), C.c_ulonglong, C.c_uint, C.c_int,
          C.c_int, C.c_int, C.c_int, C.c_double, _ip, _llp, _ip, _dp,
          C.POINTER(PartitionTrace)])
if hasattr(_lib, "ccuba_submit"):
    _sig("ccuba_submit", C.c_int, [_CTXP, C.POINTER(Job), C.POINTER(C.c_ulonglong)])
    _sig("ccuba_poll", C.c_int, [_CTXP, C.c_ulonglong, C.POINTER(Result)])
    _sig("ccuba_drain", C.c_int, [_CTXP])

SYMBOLS = ["ccuba_init", "ccuba_shutdown", "ccuba_config", "ccuba_config_get",
           "ccuba_strerror", "ccuba_vegas",
           "ccuba_vegas_ex", "ccuba_cuhre", "ccuba_cuhre_rule", "ccuba_vegas_batch",
           "ccuba_submit", "ccuba_poll", "ccuba_drain", "ccuba_vegas_dosample_raw",
           "ccuba_vegas_dosample_raw_noalloc",
           "ccuba_vegas_points", "ccuba_vegas_refine", "ccuba_vegas_batched",
           "ccuba_vegas_source", "ccuba_rtc_log", "ccuba_vegas_stateful", "ccuba_suave",
           "ccuba_divonne_partition"]


class CcubaError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__("%s: %s (%d)" % (what, strerror(rc), rc))
        self.rc = rc


def strerror(rc):
    return _lib.ccuba_strerror(rc).decode()


def _check(rc, what):
    if rc != 0:
        raise CcubaError(rc, what)
    return rc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_dp)


class Context:
    """A library context (the analog of the paper's spinning-cores handle)."""

    def __init__(self, device=-1, hbm_budget=0):
        self._h = _CTXP()
        _check(_lib.ccuba_init(C.byref(self._h), device, hbm_budget), "ccuba_init")

    @property
    def handle(self):
        return self._h

    def config(self, key, value):
        _check(_lib.ccuba_config(self._h, key.encode(), int(value)), "ccuba_config(%s)" % key)

    def config_get(self, key, precision=FP32_EVAL):
        v = C.c_longlong()
        _check(_lib.ccuba_config_get(self._h, key.encode(), int(precision), C.byref(v)),
               "ccuba_config_get(%s)" % key)
        return v.value

    def close(self):
        if self._h:
            _lib.ccuba_shutdown(C.byref(self._h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _integrand(family, a, u):
    a = _f64(a)
    u = _f64(u)
    return Integrand(int(family), _ptr(a), _ptr(u)), (a, u)


def _ctx_arg(ctx):
    """ctx=None -> NULL (temporary context); Context -> its handle."""
    if ctx is None:
        return None
    return C.byref(ctx.handle)


def vegas(family, a, u, *, ctx=None, epsrel=0.0, epsabs=0.0, flags=FP64, seed=1, mineval=0,
          maxeval=10**5, nstart=10**4, nincrease=0, nbatch=1000, nbins=128, stream_id=0,
          trace=False, max_iter=4096, gridno=0, statefile=None):
    """ccuba_vegas(_ex), or ccuba_vegas_stateful with gridno / statefile: returns a
    dict with neval, fail, integral, error, prob (and iter_I, iter_var, chi2, dof,
    grid when trace=True)."""
    f, keep = _integrand(family, a, u)
    ndim = len(keep[0])
    neval = C.c_longlong()
    fail = C.c_int()
    out = np.zeros(3)
    res = [np.zeros(1) for _ in range(3)]
    args = [_ctx_arg(ctx), ndim, 1, C.byref(f), epsrel, epsabs, flags, seed, mineval, maxeval,
            nstart, nincrease, nbatch, nbins, stream_id, C.byref(neval), C.byref(fail),
            _ptr(res[0]), _ptr(res[1]), _ptr(res[2])]
    r = dict()
    stateful = gridno != 0 or bool(statefile)
    if stateful:
        sargs = args[:13] + [int(gridno), statefile.encode() if statefile else None] + args[13:]
    if trace:
        It = np.zeros(max_iter)
        Vt = np.zeros(max_iter)
        grid = np.zeros(ndim * (nbins + 1))
        tr = VegasTrace(max_iter, 0, _ptr(It), _ptr(Vt), 0.0, 0, _ptr(grid))
        if stateful:
            _check(_lib.ccuba_vegas_stateful(*sargs, C.byref(tr)), "ccuba_vegas_stateful")
        else:
            _check(_lib.ccuba_vegas_ex(*args, C.byref(tr)), "ccuba_vegas_ex")
        n = tr.n_iter
        r.update(iter_I=It[:n].copy(), iter_var=Vt[:n].copy(), chi2=tr.chi2, dof=tr.dof,
                 grid=grid.reshape(ndim, nbins + 1))
    elif stateful:
        _check(_lib.ccuba_vegas_stateful(*sargs, None), "ccuba_vegas_stateful")
    else:
        _check(_lib.ccuba_vegas(*args), "ccuba_vegas")
    del out
    r.update(neval=neval.value, fail=fail.value, integral=float(res[0][0]),
             error=float(res[1][0]), prob=float(res[2][0]))
    return r


def vegas_points(ctx, ndim, nbins, grid, seed, stream_id, iteration, i0, npts, flags=FP64):
    grid = _f64(grid).reshape(-1)
    nblk = (ndim + 3) // 4
    words = np.zeros((npts, 4 * nblk), dtype=np.uint32)
    x = np.zeros((npts, ndim))
    w = np.zeros(npts)
    k = np.zeros((npts, ndim), dtype=np.int32)
    _check(_lib.ccuba_vegas_points(ctx.handle, ndim, nbins, flags, seed, stream_id, iteration,
                                   _ptr(grid), i0, npts,
                                   words.ctypes.data_as(C.POINTER(C.c_uint32)), _ptr(x),
                                   _ptr(w), k.ctypes.data_as(_ip)), "ccuba_vegas_points")
    return dict(words=words, x=x, w=w, bin=k)


def vegas_refine(ctx, hist, grid):
    hist = _f64(hist)
    grid = _f64(grid)
    ndim, nbins = hist.shape
    out = np.zeros_like(grid)
    _check(_lib.ccuba_vegas_refine(ctx.handle, ndim, nbins, _ptr(hist), _ptr(grid), _ptr(out)),
           "ccuba_vegas_refine")
    return out


def vegas_dosample_raw(ctx, family, a, u, nbins, iteration, npts, grid_ptr, sums_ptr, hist_ptr,
                       stream_ptr=None, flags=FP64, seed=1, stream_id=0, noalloc=False):
    """Device-buffer DoSample: pointers are device addresses (e.g. torch
    tensor .data_ptr()), stream_ptr a HIP stream handle (or None).  noalloc
    calls ccuba_vegas_dosample_raw_noalloc, which allocates nothing and
    returns without waiting for the stream."""
    f, keep = _integrand(family, a, u)
    name = "ccuba_vegas_dosample_raw_noalloc" if noalloc else "ccuba_vegas_dosample_raw"
    _check(getattr(_lib, name)(ctx.handle, len(keep[0]), nbins, C.byref(f), flags, seed,
                               stream_id, iteration, npts, C.c_void_p(grid_ptr),
                               C.c_void_p(sums_ptr), C.c_void_p(hist_ptr),
                               C.c_void_p(stream_ptr) if stream_ptr else None), name)


def rtc_log(ctx):
    """The compiler's message of the context's last run-time compilation."""
    buf = C.create_string_buffer(1 << 16)
    _check(_lib.ccuba_rtc_log(ctx.handle, buf, len(buf)), "ccuba_rtc_log")
    return buf.value.decode(errors="replace")


def vegas_source(source, ndim, a=None, u=None, *, ctx=None, epsrel=0.0, epsabs=0.0, flags=FP64,
                 seed=1, mineval=0, maxeval=10**5, nstart=10**4, nincrease=0, nbatch=1000,
                 nbins=128, stream_id=0):
    """ccuba_vegas_source: Vegas of a device integrand given as HIP source, which
    defines ``__device__ double ccuba_user(const double *x, int ndim, const double *a,
    const double *u)`` (and the float version for FP32_EVAL).  The library compiles
    it into its DoSample kernel at run time.  A source that does not compile raises
    CcubaError with the compiler's message."""
    a = _f64(np.zeros(ndim) if a is None else a)
    u = _f64(np.zeros(ndim) if u is None else u)
    neval = C.c_longlong()
    fail = C.c_int()
    res = [np.zeros(1) for _ in range(3)]
    rc = _lib.ccuba_vegas_source(_ctx_arg(ctx), ndim, source.encode(), _ptr(a), _ptr(u), epsrel,
                                 epsabs, flags, seed, mineval, maxeval, nstart, nincrease,
                                 nbatch, nbins, stream_id, C.byref(neval), C.byref(fail),
                                 _ptr(res[0]), _ptr(res[1]), _ptr(res[2]))
    if rc == EINVAL and ctx is not None:
        log = rtc_log(ctx)
        if log:
            raise CcubaError(rc, "ccuba_vegas_source: the source does not compile:\n" + log)
    _check(rc, "ccuba_vegas_source")
    return dict(neval=neval.value, fail=fail.value, integral=float(res[0][0]),
                error=float(res[1][0]), prob=float(res[2][0]))


class _DeviceArray:
    """A library-owned device buffer, seen through the array interface that
    torch.as_tensor accepts (no copy)."""

    def __init__(self, ptr, shape):
        self.__cuda_array_interface__ = {"shape": shape, "typestr": "<f8",
                                         "data": (ptr, False), "version": 2, "strides": None}


def vegas_batched(func, ndim, ncomp=1, *, where="host", nvec=10000, ctx=None, epsrel=0.0,
                  epsabs=0.0, flags=FP64, seed=1, mineval=0, maxeval=10**5, nstart=10**4,
                  nincrease=0, nbins=128, stream_id=0):
    """ccuba_vegas_batched: Vegas of a caller's integrand, in batches of nvec points.

    where="host": ``func(x)`` gets a numpy array x of shape (m, ndim) and returns
    f of shape (m,) or (m, ncomp), or -999 to abort.  where="device": ``func(x, f)``
    gets torch tensors on the GPU, x of shape (m, ndim) and f of shape (m, ncomp),
    fills f in place and may return -999; the binding waits for torch's current
    stream after the call.  An exception raised by func aborts the run and is
    raised again here.  Returns a dict with neval, fail, integral, error, prob
    (floats for ncomp == 1, arrays otherwise)."""
    if where not in ("host", "device"):
        raise ValueError("where must be 'host' or 'device'")
    raised = []

    def cb(nd_p, x, nc_p, f, userdata, nv_p, core):
        try:
            nd, nc, nv = nd_p[0], nc_p[0], nv_p[0]
            if where == "host":
                xs = np.ctypeslib.as_array(C.cast(C.c_void_p(x), _dp), shape=(nv, nd))
                r = func(xs)
                if isinstance(r, int) and r == -999:
                    return -999
                fs = np.ctypeslib.as_array(C.cast(C.c_void_p(f), _dp), shape=(nv, nc))
                fs[:] = np.asarray(r, dtype=np.float64).reshape(nv, nc)
                return 0
            import torch
            xt = torch.as_tensor(_DeviceArray(x, (nv, nd)), device="cuda")
            ft = torch.as_tensor(_DeviceArray(f, (nv, nc)), device="cuda")
            r = func(xt, ft)
            torch.cuda.current_stream().synchronize()
            return -999 if (isinstance(r, int) and r == -999) else 0
        except BaseException as e:  # reported after the library returns
            raised.append(e)
            return -999

    cfn = BATCH_INTEGRAND(cb)
    neval = C.c_longlong()
    fail = C.c_int()
    res = [np.zeros(ncomp) for _ in range(3)]
    rc = _lib.ccuba_vegas_batched(_ctx_arg(ctx), ndim, ncomp, cfn, None, nvec,
                                  POINTS_HOST if where == "host" else POINTS_DEVICE, epsrel,
                                  epsabs, flags, seed, mineval, maxeval, nstart, nincrease,
                                  nbins, stream_id, C.byref(neval), C.byref(fail),
                                  _ptr(res[0]), _ptr(res[1]), _ptr(res[2]))
    if raised:
        raise raised[0]
    _check(rc, "ccuba_vegas_batched")
    one = ncomp == 1
    out = dict(neval=neval.value, fail=fail.value)
    for k, v in zip(("integral", "error", "prob"), res):
        out[k] = float(v[0]) if one else v.copy()
    return out


def _struct_dtype(st):
    """numpy dtype with the layout of a ctypes structure (pointers as uint64)."""
    names, formats, offsets = [], [], []
    for name, typ in st._fields_:
        if isinstance(typ, type) and issubclass(typ, C.Structure):
            fmt = _struct_dtype(typ)
        elif hasattr(typ, "contents"):
            fmt = np.uint64
        else:
            fmt = np.dtype(typ)
        names.append(name)
        formats.append(fmt)
        offsets.append(getattr(st, name).offset)
    return np.dtype(dict(names=names, formats=formats, offsets=offsets,
                         itemsize=C.sizeof(st)))


_JOB_DTYPE = _struct_dtype(Job)


def make_jobs(specs):
    """Build a ctypes Job array from dicts (method, ndim, family, a, u, epsrel,
    epsabs, flags, seed, stream_id, mineval, maxeval, nstart, nincrease,
    nbins, max_regions_per_batch).  Returns (array, keep): keep holds the
    parameter arrays the jobs point into and must outlive the call."""
    n = len(specs)
    dmax = max((len(s["a"]) for s in specs), default=1)
    A = np.zeros((max(n, 1), dmax))
    U = np.zeros((max(n, 1), dmax))
    nd = np.zeros(n, dtype=np.int32)
    for q, s in enumerate(specs):
        a, u = _f64(s["a"]), _f64(s["u"])
        if len(u) != len(a):
            raise ValueError("a and u differ in length")
        nd[q] = len(a)
        A[q, :len(a)] = a
        U[q, :len(u)] = u
    rec = np.zeros(n, dtype=_JOB_DTYPE)

    def col(key, dflt, typ=int):
        return np.fromiter((typ(s.get(key, dflt)) for s in specs), dtype=np.float64 if typ is float
                           else np.int64, count=n)
    rec["method"] = col("method", 0)
    rec["ndim"] = nd
    rec["f"]["family"] = np.fromiter((int(s["family"]) for s in specs), dtype=np.int64, count=n)
    rec["f"]["a"] = A.ctypes.data + np.arange(n, dtype=np.uint64) * (8 * dmax)
    rec["f"]["u"] = U.ctypes.data + np.arange(n, dtype=np.uint64) * (8 * dmax)
    rec["epsrel"] = col("epsrel", 0.0, float)
    rec["epsabs"] = col("epsabs", 0.0, float)
    rec["flags"] = col("flags", 0)
    rec["seed"] = np.fromiter((int(s.get("seed", 1)) for s in specs), dtype=np.uint64, count=n)
    rec["stream_id"] = col("stream_id", 0)
    rec["mineval"] = col("mineval", 0)
    rec["maxeval"] = col("maxeval", 10**5)
    rec["nstart"] = col("nstart", 10**4)
    rec["nincrease"] = col("nincrease", 0)
    rec["nbins"] = col("nbins", 128)
    rec["max_regions_per_batch"] = col("max_regions_per_batch", 0)
    arr = (Job * n).from_buffer(rec)
    return arr, (A, U, rec)


def _result_dict(r):
    return dict(neval=r.neval, nregions=r.nregions, fail=r.fail, status=r.status,
                integral=r.integral, error=r.error, prob=r.prob, t_submit=r.t_submit,
                t_done=r.t_done)


def vegas_batch(ctx, specs):
    """Many independent Vegas integrals in one engine.  specs: a list of job
    dicts (see make_jobs), or the (array, keep) pair make_jobs returns."""
    arr, keep = specs if isinstance(specs, tuple) else make_jobs(specs)
    out = (Result * len(arr))()
    _check(_lib.ccuba_vegas_batch(ctx.handle, len(arr), arr, out), "ccuba_vegas_batch")
    return [_result_dict(r) for r in out]


def cuhre(family, a, u, *, ctx=None, epsrel=1e-3, epsabs=0.0, flags=0, mineval=0,
          maxeval=10**7, key=7, max_regions_per_batch=10**5):
    f, keep = _integrand(family, a, u)
    nreg = C.c_int()
    neval = C.c_longlong()
    fail = C.c_int()
    res = [np.zeros(1) for _ in range(3)]
    _check(_lib.ccuba_cuhre(_ctx_arg(ctx), len(keep[0]), 1, C.byref(f), epsrel, epsabs, flags,
                            mineval, maxeval, key, max_regions_per_batch, C.byref(nreg),
                            C.byref(neval), C.byref(fail), _ptr(res[0]), _ptr(res[1]),
                            _ptr(res[2])), "ccuba_cuhre")
    return dict(nregions=nreg.value, neval=neval.value, fail=fail.value,
                integral=float(res[0][0]), error=float(res[1][0]), prob=float(res[2][0]))


def suave(family, a, u, *, ctx=None, epsrel=0.0, epsabs=0.0, flags=0, seed=1, mineval=0,
          maxeval=10**5, nnew=1000, flatness=25.0, nbins=128, nsplit=1, stream_id=0,
          trace=False):
    """Suave of a Genz integrand.  With trace=True the result also holds every
    region in position order (bounds, estimates, grids) and the cut dimensions."""
    f, keep = _integrand(family, a, u)
    d = len(keep[0])
    nreg, neval, fail = C.c_int(), C.c_longlong(), C.c_int()
    res = [np.zeros(1) for _ in range(3)]
    tr = None
    if trace:
        m = 1 + max(0, int(maxeval) // (2 * int(nnew)))
        arrs = dict(lo=np.zeros((m, d)), hi=np.zeros((m, d)), I=np.zeros(m), var=np.zeros(m),
                    grid=np.zeros((m, d, nbins + 1)), cut=np.zeros(m, dtype=np.int32))
        tr = SuaveTrace(m, m, 0, 0, 0.0, 0, _ptr(arrs["lo"]), _ptr(arrs["hi"]),
                        _ptr(arrs["I"]), _ptr(arrs["var"]), _ptr(arrs["grid"]),
                        arrs["cut"].ctypes.data_as(_ip))
    _check(_lib.ccuba_suave(_ctx_arg(ctx), d, 1, C.byref(f), epsrel, epsabs, flags, seed,
                            mineval, maxeval, nnew, flatness, nbins, nsplit, stream_id,
                            C.byref(nreg), C.byref(neval), C.byref(fail), _ptr(res[0]),
                            _ptr(res[1]), _ptr(res[2]), C.byref(tr) if tr is not None else None),
           "ccuba_suave")
    out = dict(nregions=nreg.value, neval=neval.value, fail=fail.value,
               integral=float(res[0][0]), error=float(res[1][0]), prob=float(res[2][0]))
    if tr is not None:
        R = tr.nregions
        out.update(chi2=tr.chi2, dof=tr.dof, lo=arrs["lo"][:R].copy(), hi=arrs["hi"][:R].copy(),
                   I=arrs["I"][:R].copy(), var=arrs["var"][:R].copy(),
                   grid=arrs["grid"][:R].copy(), cut=arrs["cut"][:tr.nsplits].copy())
    return out


def divonne_partition(family, a, u, *, ctx=None, seed=1, stream_id=0, nsearch=256, niter=32,
                      maxregions=64, nsplit=1, spread_tol=0.0, trace=False):
    """Divonne's partitioning phase for a Genz integrand.  With trace=True the
    result also holds every region (bounds, extrema and their points, spread)
    and the cut dimensions."""
    f, keep = _integrand(family, a, u)
    d = len(keep[0])
    nreg, neval, fail, tot = C.c_int(), C.c_longlong(), C.c_int(), C.c_double()
    tr = None
    if trace:
        m = int(maxregions)
        arrs = dict(lo=np.zeros((m, d)), hi=np.zeros((m, d)), xmin=np.zeros((m, d)),
                    xmax=np.zeros((m, d)), fmin=np.zeros(m), fmax=np.zeros(m),
                    spread=np.zeros(m), cut=np.zeros(m, dtype=np.int32))
        tr = PartitionTrace(m, m, 0, 0, *[_ptr(arrs[k]) for k in
                                          ("lo", "hi", "xmin", "xmax", "fmin", "fmax",
                                           "spread")], arrs["cut"].ctypes.data_as(_ip))
    _check(_lib.ccuba_divonne_partition(_ctx_arg(ctx), d, C.byref(f), seed, stream_id, nsearch,
                                        niter, maxregions, nsplit, spread_tol, C.byref(nreg),
                                        C.byref(neval), C.byref(fail), C.byref(tot),
                                        C.byref(tr) if tr is not None else None),
           "ccuba_divonne_partition")
    out = dict(nregions=nreg.value, neval=neval.value, fail=fail.value,
               total_spread=tot.value)
    if tr is not None:
        R = tr.nregions
        for k in ("lo", "hi", "xmin", "xmax", "fmin", "fmax", "spread"):
            out[k] = arrs[k][:R].copy()
        out["cut"] = arrs["cut"][:tr.nsplits].copy()
    return out


def cuhre_rule(ctx, family, a, u, c, h):
    """Rule on a batch of regions: c, h arrays of shape (nreg, ndim)."""
    f, keep = _integrand(family, a, u)
    c = np.atleast_2d(_f64(c))
    h = np.atleast_2d(_f64(h))
    nreg, ndim = c.shape
    cs = np.ascontiguousarray(c.T)
    hs = np.ascontiguousarray(h.T)
    I7 = np.zeros(nreg)
    I5 = np.zeros(nreg)
    err = np.zeros(nreg)
    axis = np.zeros(nreg, dtype=np.int32)
    _check(_lib.ccuba_cuhre_rule(ctx.handle, ndim, C.byref(f), nreg, _ptr(cs), _ptr(hs),
                                 _ptr(I7), _ptr(I5), _ptr(err), axis.ctypes.data_as(_ip)),
           "ccuba_cuhre_rule")
    return dict(I7=I7, I5=I5, err=err, axis=axis)


def submit(ctx, spec):
    arr, keep = make_jobs([spec])
    t = C.c_ulonglong()
    _check(_lib.ccuba_submit(ctx.handle, arr, C.byref(t)), "ccuba_submit")
    return t.value


def poll(ctx, ticket):
    """None while pending, else the result dict."""
    r = Result()
    rc = _lib.ccuba_poll(ctx.handle, ticket, C.byref(r))
    if rc == 1:
        return None
    _check(rc, "ccuba_poll")
    return _result_dict(r)


def drain(ctx):
    _check(_lib.ccuba_drain(ctx.handle), "ccuba_drain")
