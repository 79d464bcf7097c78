"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ccuba.h declares, names its status codes, and rejects
malformed arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccuba.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccuba_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def cc():
    import paper_1408_6373_amd as cc
    return cc


def test_every_declared_symbol_is_exported(cc):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(cc._lib, n), n
    assert set(cc.SYMBOLS) <= set(names)


def test_config_get_rejects_bad_arguments_on_the_host(cc):
    v = C.c_longlong()
    assert cc._lib.ccuba_config_get(None, b"ilp", 1, C.byref(v)) == cc.EINVAL


def test_strerror_names_codes(cc):
    for rc in (0, -1, -2, -3, -4, -5):
        assert cc.strerror(rc) not in ("", "unknown status")
    assert cc.strerror(-99) == "unknown status"


def test_bad_arguments_are_rejected_on_the_host(cc):
    a = np.ones(3)
    u = np.full(3, 0.5)
    f, keep = cc._integrand(0, a, u)
    n, fl = C.c_longlong(), C.c_int()
    r = [np.zeros(1) for _ in range(3)]
    ptrs = [cc._ptr(x) for x in r]
    L = cc._lib
    # ndim out of range, ncomp != 1, bins out of range, nstart < 2, nbatch < 1
    for nd, nc, nb, ns, nbatch in ((0, 1, 128, 100, 1), (17, 1, 128, 100, 1),
                                   (3, 2, 128, 100, 1), (3, 1, 1, 100, 1),
                                   (3, 1, 257, 100, 1), (3, 1, 128, 1, 1),
                                   (3, 1, 128, 100, 0)):
        rc = L.ccuba_vegas(None, nd, nc, C.byref(f), 0.0, 0.0, 0, 1, 0, 1000, ns, 0, nbatch,
                           nb, 0, C.byref(n), C.byref(fl), *ptrs)
        assert rc == cc.EINVAL
    # precision bits 2 and 3 are not defined
    rc = L.ccuba_vegas(None, 3, 1, C.byref(f), 0.0, 0.0, 2, 1, 0, 1000, 100, 0, 1, 128, 0,
                       C.byref(n), C.byref(fl), *ptrs)
    assert rc == cc.EINVAL
    # Cuhre: ndim 1, key 9, batch 1
    nr = C.c_int()
    for nd, key, b in ((1, 7, 100), (3, 9, 100), (3, 7, 1)):
        rc = L.ccuba_cuhre(None, nd, 1, C.byref(f), 1e-3, 0.0, 0, 0, 10**6, key, b,
                           C.byref(nr), C.byref(n), C.byref(fl), *ptrs)
        assert rc == cc.EINVAL
    # caller-evaluated integrand: ndim, ncomp, nbins, nvec, where, precision
    cb = cc.BATCH_INTEGRAND(lambda *args: 0)
    r3 = [np.zeros(17) for _ in range(3)]
    p3 = [cc._ptr(x) for x in r3]
    for nd, nc, nb, nv, wh, fl_ in ((0, 1, 64, 10, 0, 0), (3, 0, 64, 10, 0, 0),
                                    (3, 17, 64, 10, 0, 0), (3, 1, 1, 10, 0, 0),
                                    (3, 1, 64, 0, 0, 0), (3, 1, 64, 10, 2, 0),
                                    (3, 1, 64, 10, 0, 2)):
        rc = L.ccuba_vegas_batched(None, nd, nc, cb, None, nv, wh, 0.0, 0.0, fl_, 1, 0, 1000,
                                   100, 0, nb, 0, C.byref(n), C.byref(fl), *p3)
        assert rc == cc.EINVAL
    # device source: NULL source, ndim out of range
    for nd, src in ((3, None), (0, b"x"), (17, b"x")):
        rc = L.ccuba_vegas_source(None, nd, src, None, None, 0.0, 0.0, 0, 1, 0, 1000, 100, 0,
                                  1, 64, 0, C.byref(n), C.byref(fl), *ptrs)
        assert rc == cc.EINVAL
    # checkpointed Vegas: the checks of ccuba_vegas, before any file is touched
    for nd, nb in ((0, 64), (3, 1)):
        rc = L.ccuba_vegas_stateful(None, nd, 1, C.byref(f), 0.0, 0.0, 0, 1, 0, 1000, 100, 0, 1,
                                    2, b"/nonexistent/dir/state", nb, 0, C.byref(n),
                                    C.byref(fl), *ptrs, None)
        assert rc == cc.EINVAL
    rc = L.ccuba_vegas_stateful(None, 3, 1, C.byref(f), 0.0, 0.0, 0, 1, 0, 1000, 100, 0, 1, 0,
                                None, 64, 0, None, C.byref(fl), *ptrs, None)
    assert rc == cc.EINVAL
    # Suave: ndim, ncomp, nnew, flatness, nsplit, nbins, precision
    nr = C.c_int()
    for nd, nc, nn, fl_, ns, nb, flg in ((0, 1, 100, 25.0, 1, 64, 0), (17, 1, 100, 25.0, 1, 64, 0),
                                          (3, 2, 100, 25.0, 1, 64, 0), (3, 1, 1, 25.0, 1, 64, 0),
                                          (3, 1, 100, 0.0, 1, 64, 0), (3, 1, 100, 25.0, 0, 64, 0),
                                          (3, 1, 100, 25.0, 1025, 64, 0),
                                          (3, 1, 100, 25.0, 1, 1, 0), (3, 1, 100, 25.0, 1, 64, 1)):
        rc = L.ccuba_suave(None, nd, nc, C.byref(f), 0.0, 0.0, flg, 1, 0, 1000, nn, fl_, nb, ns, 0,
                           C.byref(nr), C.byref(n), C.byref(fl), *ptrs, None)
        assert rc == cc.EINVAL
    # Divonne partition: ndim, nsearch, niter, maxregions, nsplit, spread_tol
    tot = C.c_double()
    for nd, nse, nit, mr, ns, tol in ((0, 10, 1, 4, 1, 0.0), (17, 10, 1, 4, 1, 0.0),
                                      (3, 0, 1, 4, 1, 0.0), (3, 10, -1, 4, 1, 0.0),
                                      (3, 10, 1, 0, 1, 0.0), (3, 10, 1, 4, 0, 0.0),
                                      (3, 10, 1, 4, 1, -1.0), (3, (1 << 30) + 1, 1, 4, 1, 0.0)):
        rc = L.ccuba_divonne_partition(None, nd, C.byref(f), 1, 0, nse, nit, mr, ns, tol,
                                       C.byref(nr), C.byref(n), C.byref(fl), C.byref(tot), None)
        assert rc == cc.EINVAL
    # device-buffer DoSample, both entry points: no context, no buffers, npts < 2
    for name in ("ccuba_vegas_dosample_raw", "ccuba_vegas_dosample_raw_noalloc"):
        fn = getattr(L, name)
        assert fn(None, 3, 64, C.byref(f), 0, 1, 0, 0, 1000, 8, 8, 8, None) == cc.EINVAL
        hc = C.c_void_p(1)  # never dereferenced: the buffer checks come first
        assert fn(hc, 3, 64, C.byref(f), 0, 1, 0, 0, 1000, None, 8, 8, None) == cc.EINVAL
        assert fn(hc, 3, 64, C.byref(f), 0, 1, 0, 0, 1, 8, 8, 8, None) == cc.EINVAL
    assert L.ccuba_rtc_log(None, C.create_string_buffer(8), 8) == cc.EINVAL
    assert L.ccuba_init(None, 0, 0) == cc.EINVAL
    assert L.ccuba_config(None, b"block", 256) == cc.EINVAL
    h = C.c_void_p()
    assert L.ccuba_shutdown(C.byref(h)) == cc.OK  # a NULL handle is accepted


def test_structures_match_the_header(cc):
    # the ctypes mirrors have the C sizes (x86-64 System V layout)
    assert C.sizeof(cc.Integrand) == 24
    assert C.sizeof(cc.Result) == 8 + 4 * 4 + 8 * 5
    assert C.sizeof(cc.VegasTrace) == 48
