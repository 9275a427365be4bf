"""mgme: tree-level |M|^2, summed over helicities and colours, on MI355X.

Thin Python binding of libmgme.so (see include/mgme.h): argument marshalling
only.  Device memory and streams come from PyTorch; every step of the
computation runs in the library's HIP kernels.  Importing works without the
library; the first call that needs it raises MgmeError if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgme.so")

MGME_OK, MGME_EINVAL, MGME_EUNSUPPORTED, MGME_ENOMEM, MGME_EDEVICE = 0, -1, -2, -3, -4
FP64, FP32, MIXED, FP64_FP32COLOUR = 0, 1, 2, 3

PROCESSES = {
    "ee_mumu": [-11, 11, -13, 13],
    "gg_tt": [21, 21, 6, -6],
    "gg_ttg": [21, 21, 6, -6, 21],
    "gg_ttgg": [21, 21, 6, -6, 21, 21],
    "gg_ttggg": [21, 21, 6, -6, 21, 21, 21],
}

DEFAULT_PARAMS = dict(alpha_s=0.118, alpha_em=1.0 / 132.5, sin2w=0.2222, mz=91.188, wz=2.441,
                      mt=173.0, wt=0.0, z_enabled=1)

# Entry points declared in include/mgme.h.
EXPORTS = ["mgme_process_create", "mgme_process_destroy", "mgme_process_info", "mgme_good_helicities",
           "mgme_set_helicities",
           "mgme_colour_matrix", "mgme_rambo", "mgme_matrix_element", "mgme_matrix_element_noalloc",
           "mgme_matrix_element_per_helicity",
           "mgme_workspace_bytes", "mgme_select", "mgme_event_weights", "mgme_unweight",
           "mgme_last_error", "mgme_server_create", "mgme_server_submit",
           "mgme_server_wait", "mgme_server_drain", "mgme_server_get_stats", "mgme_server_destroy",
           "mgme_server_last_error"]


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_longlong), ("use_graphs", ctypes.c_int),
                ("slot_workspace_bytes", ctypes.c_longlong), ("max_pass_over", ctypes.c_int),
                ("fake_executor", ctypes.c_int), ("fake_ns_per_event", ctypes.c_double),
                ("fake_bytes_per_event", ctypes.c_longlong), ("fake_fail_nevt", ctypes.c_longlong)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("events", ctypes.c_longlong), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("max_concurrent", ctypes.c_int), ("peak_footprint_bytes", ctypes.c_longlong),
                ("budget_bytes", ctypes.c_longlong), ("split_requests", ctypes.c_longlong),
                ("graph_launches", ctypes.c_longlong), ("graph_instantiations", ctypes.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MgmeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mgme error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("alpha_s", ctypes.c_double), ("alpha_em", ctypes.c_double), ("sin2w", ctypes.c_double),
                ("mz", ctypes.c_double), ("wz", ctypes.c_double), ("mt", ctypes.c_double),
                ("wt", ctypes.c_double), ("z_enabled", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("n_ext", ctypes.c_int), ("n_diagrams", ctypes.c_int), ("n_amp_terms", ctypes.c_int),
                ("n_colour", ctypes.c_int), ("n_hel", ctypes.c_int), ("n_good_hel", ctypes.c_int),
                ("n_currents", ctypes.c_int), ("n_amp_vertices", ctypes.c_int),
                ("norm_factor", ctypes.c_double), ("flops_per_hel", ctypes.c_double),
                ("flops_per_event", ctypes.c_double), ("kernel_hash", ctypes.c_ulonglong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libmgme.so; raises MgmeError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MgmeError(MGME_EUNSUPPORTED, f"{LIB_PATH} is missing: run paper_2303_18244_amd.build first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u64, dp = ctypes.c_void_p, ctypes.c_longlong, ctypes.c_ulonglong, ctypes.c_void_p
        L.mgme_process_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(vp)]
        L.mgme_process_destroy.argtypes = [vp]
        L.mgme_process_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.mgme_good_helicities.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.mgme_set_helicities.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.mgme_colour_matrix.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_int)]
        L.mgme_rambo.argtypes = [vp, ctypes.c_double, u64, u64, i64, i64, dp, dp, vp]
        L.mgme_matrix_element.argtypes = [vp, dp, i64, i64, ctypes.c_int, dp, vp]
        L.mgme_matrix_element_noalloc.argtypes = [vp, dp, i64, i64, ctypes.c_int, dp, vp]
        L.mgme_matrix_element_per_helicity.argtypes = [vp, dp, i64, i64, ctypes.c_int, dp, i64, vp]
        L.mgme_workspace_bytes.argtypes = [vp, i64, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
        L.mgme_select.argtypes = [vp, dp, i64, i64, ctypes.c_int, dp, dp, dp, vp, vp, vp]
        L.mgme_event_weights.argtypes = [ctypes.c_double, dp, dp, i64, dp, dp, vp]
        L.mgme_unweight.argtypes = [dp, dp, i64, dp, vp, vp, vp]
        L.mgme_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.c_int, ctypes.POINTER(vp)]
        L.mgme_server_submit.argtypes = [vp, vp, dp, i64, i64, ctypes.c_int, dp, vp,
                                         ctypes.POINTER(ctypes.c_ulonglong)]
        L.mgme_server_wait.argtypes = [vp, ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_double)]
        L.mgme_server_drain.argtypes = [vp]
        L.mgme_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.mgme_server_destroy.argtypes = [vp]
        L.mgme_last_error.restype = ctypes.c_char_p
        L.mgme_server_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if not name.endswith("last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != MGME_OK:
        raise MgmeError(rc, lib().mgme_last_error().decode())


def _scheck(rc: int) -> None:
    if rc != MGME_OK:
        raise MgmeError(rc, lib().mgme_server_last_error().decode())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Process:
    """A compiled process on one GPU."""

    def __init__(self, pdg: Sequence[int], device: int = 0, **params):
        par = dict(DEFAULT_PARAMS)
        par.update(params)
        self.pdg = list(pdg)
        self.device = device
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_int * len(self.pdg))(*self.pdg)
        _check(lib().mgme_process_create(2, len(self.pdg) - 2, arr, ctypes.byref(Params(**par)), device,
                                         ctypes.byref(self._h)))
        info = Info()
        _check(lib().mgme_process_info(self._h, ctypes.byref(info)))
        self.info = info.as_dict()
        self.n_ext = info.n_ext

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().mgme_process_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def good_helicities(self):
        codes = (ctypes.c_int * (1 << self.n_ext))()
        n = ctypes.c_int()
        _check(lib().mgme_good_helicities(self._h, codes, ctypes.byref(n)))
        return list(codes[: n.value])

    def set_helicities(self, codes=None):
        """Sums only the helicity codes given (strictly increasing); None or
        an empty list restores the good helicities."""
        codes = list(codes or [])
        arr = (ctypes.c_int * max(len(codes), 1))(*codes)
        _check(lib().mgme_set_helicities(self._h, arr if codes else None, len(codes)))
        info = Info()
        _check(lib().mgme_process_info(self._h, ctypes.byref(info)))
        self.info = info.as_dict()

    def colour_matrix(self):
        """(numerators [n][n], denominator, basis [n][k])."""
        n = self.info["n_colour"]
        k = sum(1 for x in self.pdg if x == 21)
        num = (ctypes.c_longlong * (n * n))()
        den = ctypes.c_longlong()
        basis = (ctypes.c_int * max(1, n * k))()
        _check(lib().mgme_colour_matrix(self._h, num, ctypes.byref(den), basis))
        return ([list(num[r * n:(r + 1) * n]) for r in range(n)], den.value,
                [list(basis[r * k:(r + 1) * k]) for r in range(n)])

    def rambo(self, sqrt_s: float, seed: int, first_event: int, nevt: int, ld: Optional[int] = None,
              mom=None, wgt=None, stream=None):
        """RAMBO events on the device: returns (mom [n_ext, 4, ld] float64, wgt [nevt])."""
        import torch
        ld = nevt if ld is None else ld
        dev = torch.device("cuda", self.device)
        if mom is None:
            mom = torch.empty((self.n_ext, 4, max(ld, 1)), dtype=torch.float64, device=dev)
        if wgt is None:
            wgt = torch.empty(max(nevt, 1), dtype=torch.float64, device=dev)
        _check(lib().mgme_rambo(self._h, float(sqrt_s), int(seed), int(first_event), int(nevt), int(ld),
                                mom.data_ptr(), wgt.data_ptr(), _stream_handle(stream)))
        return mom, wgt

    def matrix_element(self, mom, nevt: Optional[int] = None, precision: int = FP64, out=None, stream=None):
        """|M|^2 per event for momenta mom [n_ext, 4, ld] (float64, on the device)."""
        import torch
        ld = mom.shape[-1]
        nevt = ld if nevt is None else nevt
        if mom.dtype != torch.float64 or not mom.is_contiguous() or mom.shape[:2] != (self.n_ext, 4):
            raise MgmeError(MGME_EINVAL, "momenta must be a contiguous float64 tensor [n_ext, 4, ld]")
        if out is None:
            out = torch.empty(max(nevt, 1), dtype=torch.float64, device=mom.device)
        _check(lib().mgme_matrix_element(self._h, mom.data_ptr(), int(nevt), int(ld), int(precision),
                                         out.data_ptr(), _stream_handle(stream)))
        return out[:nevt]

    def matrix_element_noalloc(self, mom, nevt: Optional[int] = None, precision: int = FP64, out=None,
                               stream=None):
        """As matrix_element, through mgme_matrix_element_noalloc (no device
        allocation inside the call; `out` should then be given)."""
        import torch
        ld = mom.shape[-1]
        nevt = ld if nevt is None else nevt
        if mom.dtype != torch.float64 or not mom.is_contiguous() or mom.shape[:2] != (self.n_ext, 4):
            raise MgmeError(MGME_EINVAL, "momenta must be a contiguous float64 tensor [n_ext, 4, ld]")
        if out is None:
            out = torch.empty(max(nevt, 1), dtype=torch.float64, device=mom.device)
        _check(lib().mgme_matrix_element_noalloc(self._h, mom.data_ptr(), int(nevt), int(ld), int(precision),
                                                 out.data_ptr(), _stream_handle(stream)))
        return out[:nevt]

    def matrix_element_per_helicity(self, mom, nevt: Optional[int] = None, precision: int = FP64, stream=None):
        import torch
        ld = mom.shape[-1]
        nevt = ld if nevt is None else nevt
        out = torch.empty((1 << self.n_ext, max(nevt, 1)), dtype=torch.float64, device=mom.device)
        _check(lib().mgme_matrix_element_per_helicity(self._h, mom.data_ptr(), int(nevt), int(ld),
                                                      int(precision), out.data_ptr(), int(out.shape[1]),
                                                      _stream_handle(stream)))
        return out[:, :nevt]

    def select(self, mom, r_hel, r_col, nevt: Optional[int] = None, precision: int = FP64, stream=None):
        """|M|^2 and a random helicity code and colour flow per event, from the
        uniform numbers r_hel, r_col (float64 device tensors of nevt):
        returns (me [nevt] float64, hel [nevt] int32, col [nevt] int32)."""
        import torch
        ld = mom.shape[-1]
        nevt = ld if nevt is None else nevt
        if mom.dtype != torch.float64 or not mom.is_contiguous() or mom.shape[:2] != (self.n_ext, 4):
            raise MgmeError(MGME_EINVAL, "momenta must be a contiguous float64 tensor [n_ext, 4, ld]")
        for r in (r_hel, r_col):
            if r.dtype != torch.float64 or not r.is_contiguous() or r.numel() < nevt:
                raise MgmeError(MGME_EINVAL, "random numbers must be contiguous float64 tensors of nevt")
        n1 = max(nevt, 1)
        me = torch.empty(n1, dtype=torch.float64, device=mom.device)
        hel = torch.empty(n1, dtype=torch.int32, device=mom.device)
        col = torch.empty(n1, dtype=torch.int32, device=mom.device)
        _check(lib().mgme_select(self._h, mom.data_ptr(), int(nevt), int(ld), int(precision), r_hel.data_ptr(),
                                 r_col.data_ptr(), me.data_ptr(), hel.data_ptr(), col.data_ptr(),
                                 _stream_handle(stream)))
        return me[:nevt], hel[:nevt], col[:nevt]


def event_weights(sqrt_s: float, wgt, me, nevt: Optional[int] = None, want_weights: bool = True, stream=None):
    """Cross-section weights in pb and (sum w, sum w^2, max w) as a device
    tensor of 3 doubles; see mgme_event_weights."""
    import torch
    nevt = me.shape[0] if nevt is None else nevt
    for t in (wgt, me):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < nevt:
            raise MgmeError(MGME_EINVAL, "weights and matrix elements must be contiguous float64 tensors")
    w = torch.empty(max(nevt, 1), dtype=torch.float64, device=me.device) if want_weights else None
    stats = torch.empty(3, dtype=torch.float64, device=me.device)
    _check(lib().mgme_event_weights(float(sqrt_s), wgt.data_ptr(), me.data_ptr(), int(nevt),
                                    w.data_ptr() if w is not None else None, stats.data_ptr(),
                                    _stream_handle(stream)))
    return (w[:nevt] if w is not None else None), stats


def unweight(w, r, w_ref, nevt: Optional[int] = None, stream=None):
    """Hit-or-miss unweighting against the device scalar w_ref (a 1-element
    float64 tensor, or a view such as stats[2:]): returns the kept event
    indices (int64 device tensor, increasing); reads the count back to size
    the result, so this synchronises the stream."""
    import torch
    nevt = w.shape[0] if nevt is None else nevt
    for t in (w, r, w_ref):
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise MgmeError(MGME_EINVAL, "weights, random numbers and w_ref must be contiguous float64 tensors")
    if w.numel() < nevt or r.numel() < nevt or w_ref.numel() < 1:
        raise MgmeError(MGME_EINVAL, "tensor too short")
    idx = torch.empty(max(nevt, 1), dtype=torch.int64, device=w.device)
    nkept = torch.empty(1, dtype=torch.int64, device=w.device)
    _check(lib().mgme_unweight(w.data_ptr(), r.data_ptr(), int(nevt), w_ref.data_ptr(), idx.data_ptr(),
                               nkept.data_ptr(), _stream_handle(stream)))
    return idx[: int(nkept.item())]


class Server:
    """Continuous-batching request loop on one GPU (see mgme_server_* in
    include/mgme.h).  Tensors passed to submit() are kept referenced until
    their request has been waited for."""

    def __init__(self, n_slots: int = 4, hbm_budget_bytes: int = 0, device: int = 0, use_graphs: bool = False,
                 slot_workspace_bytes: int = 0, max_pass_over: int = 0, fake_ns_per_event: Optional[float] = None,
                 fake_bytes_per_event: int = 0, fake_fail_nevt: int = 0):
        cfg = ServerConfig(n_slots, hbm_budget_bytes, 1 if use_graphs else 0, slot_workspace_bytes, max_pass_over,
                           1 if fake_ns_per_event is not None else 0, float(fake_ns_per_event or 0.0),
                           int(fake_bytes_per_event), int(fake_fail_nevt))
        self._h = ctypes.c_void_p()
        _scheck(lib().mgme_server_create(ctypes.byref(cfg), device, ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, proc: Optional[Process], mom=None, nevt: Optional[int] = None, precision: int = FP64,
               out=None, stream=None) -> int:
        """Queues one batch; returns the request id.  The request starts after
        the work already enqueued on `stream` (default: torch's current
        stream), which produced `mom` and `out`.  With the test double, proc,
        mom and out may be None (only nevt is used)."""
        rid = ctypes.c_ulonglong()
        if mom is None:
            _scheck(lib().mgme_server_submit(self._h, None, None, int(nevt), int(nevt), int(precision), None, None,
                                             ctypes.byref(rid)))
            return rid.value
        ld = mom.shape[-1]
        nevt = ld if nevt is None else nevt
        _scheck(lib().mgme_server_submit(self._h, proc._h, mom.data_ptr(), int(nevt), int(ld), int(precision),
                                         out.data_ptr(), _stream_handle(stream), ctypes.byref(rid)))
        self._keep[rid.value] = (proc, mom, out)
        return rid.value

    def wait(self, rid: int) -> float:
        """Blocks until the request completed; returns its latency in ms."""
        lat = ctypes.c_double()
        rc = lib().mgme_server_wait(self._h, rid, ctypes.byref(lat))
        self._keep.pop(rid, None)
        _scheck(rc)
        return lat.value

    def drain(self) -> None:
        _scheck(lib().mgme_server_drain(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _scheck(lib().mgme_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().mgme_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
