"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/mgme.h declares, and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2303_18244_amd", "libmgme.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmgme.so not built")


def declared_functions():
    with open(os.path.join(ROOT, "include", "mgme.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mgme_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    import paper_2303_18244_amd as M

    assert declared_functions() == sorted(M.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(L, name), name


def _lib():
    import paper_2303_18244_amd as M

    return M.lib()


def test_null_and_size_checks_return_einval():
    import paper_2303_18244_amd as M

    L = _lib()
    out = ctypes.c_void_p()
    par = M.Params(**M.DEFAULT_PARAMS)
    assert L.mgme_process_create(2, 2, None, ctypes.byref(par), 0, ctypes.byref(out)) == M.MGME_EINVAL
    pdg = (ctypes.c_int * 4)(21, 21, 6, -6)
    assert L.mgme_process_create(2, 2, pdg, None, 0, ctypes.byref(out)) == M.MGME_EINVAL
    assert L.mgme_process_create(2, 2, pdg, ctypes.byref(par), 0, None) == M.MGME_EINVAL
    assert L.mgme_process_create(1, 2, pdg, ctypes.byref(par), 0, ctypes.byref(out)) == M.MGME_EINVAL
    assert b"" != L.mgme_last_error()
    info = M.Info()
    assert L.mgme_process_info(None, ctypes.byref(info)) == M.MGME_EINVAL
    assert L.mgme_matrix_element(None, None, 10, 10, 0, None, None) == M.MGME_EINVAL
    assert L.mgme_rambo(None, 1500.0, 1, 0, 10, 10, None, None, None) == M.MGME_EINVAL
    assert L.mgme_process_destroy(None) == M.MGME_OK


def test_unsupported_process_and_width():
    import paper_2303_18244_amd as M

    L = _lib()
    out = ctypes.c_void_p()
    par = M.Params(**M.DEFAULT_PARAMS)
    pdg = (ctypes.c_int * 4)(21, 21, 5, -5)
    assert L.mgme_process_create(2, 2, pdg, ctypes.byref(par), 0, ctypes.byref(out)) == M.MGME_EUNSUPPORTED
    wide = dict(M.DEFAULT_PARAMS, wt=1.5)
    pdg = (ctypes.c_int * 4)(21, 21, 6, -6)
    assert (L.mgme_process_create(2, 2, pdg, ctypes.byref(M.Params(**wide)), 0, ctypes.byref(out))
            == M.MGME_EUNSUPPORTED)
    bad = dict(M.DEFAULT_PARAMS, alpha_s=-1.0)
    assert (L.mgme_process_create(2, 2, pdg, ctypes.byref(M.Params(**bad)), 0, ctypes.byref(out))
            == M.MGME_EINVAL)


def test_last_error_is_thread_local():
    import threading

    import paper_2303_18244_amd as M

    L = _lib()
    L.mgme_process_info(None, None)
    main_msg = L.mgme_last_error()
    seen = []

    def worker():
        seen.append(L.mgme_last_error())

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert main_msg != b"" and seen == [b""]


def test_event_level_entry_points_reject_bad_arguments():
    """mgme_select, mgme_event_weights and mgme_unweight validate their
    arguments before any device call."""
    import paper_2303_18244_amd as M

    L = _lib()
    EINVAL = M.MGME_EINVAL
    assert L.mgme_select(None, None, 10, 10, 0, None, None, None, None, None, None) == EINVAL
    stats = (ctypes.c_double * 3)()
    buf = (ctypes.c_double * 16)()
    assert L.mgme_event_weights(1500.0, buf, buf, -1, None, stats, None) == EINVAL
    assert L.mgme_event_weights(1500.0, None, buf, 10, None, stats, None) == EINVAL
    assert L.mgme_event_weights(1500.0, buf, buf, 10, None, None, None) == EINVAL
    assert L.mgme_event_weights(0.0, buf, buf, 10, None, stats, None) == EINVAL
    assert L.mgme_event_weights(float("nan"), buf, buf, 10, None, stats, None) == EINVAL
    idx = (ctypes.c_longlong * 16)()
    n = (ctypes.c_longlong * 1)()
    assert L.mgme_unweight(buf, buf, -1, buf, idx, n, None) == EINVAL
    assert L.mgme_unweight(buf, buf, 10, None, idx, n, None) == EINVAL
    assert L.mgme_unweight(buf, None, 10, buf, idx, n, None) == EINVAL
    assert L.mgme_unweight(buf, buf, 10, buf, None, n, None) == EINVAL
    assert L.mgme_unweight(buf, buf, 10, buf, idx, None, None) == EINVAL
    assert b"NULL" in L.mgme_last_error() or b"nevt" in L.mgme_last_error()
