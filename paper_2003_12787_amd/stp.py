"""Python binding of libstp.so (include/stp.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the predictor runs in the library's
HIP kernels. The binding raises if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstp.so")

# stp_status
OK, PENDING, E_INVAL, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_BUSY, E_TIMEOUT = 0, 1, -1, -2, -3, -4, -5, -6
# stp_physics / stp_prec
ACOUSTIC, ELASTIC, GENERIC, ELASTIC_CURV = 0, 1, 2, 3
FP64, FP32, BF16X3 = 0, 1, 2
# class flags
PARAM_PER_ELEMENT, A_PRESENT, COEF_PER_ELEMENT, FAVG_SUM, SRC_POINT = 1, 2, 4, 8, 16
# node families
GAUSS_LEGENDRE, GAUSS_LOBATTO = 0, 1
# kernel variants
VARIANT_AUTO, VARIANT_PLAIN, VARIANT_FUSED, VARIANT_MFMA = 0, 1, 2, 3

# Exported symbols declared in include/stp.h.
SYMBOLS = ("stp_plan", "stp_plan_free", "stp_run", "stp_run_noalloc", "stp_sync", "stp_reserve", "stp_submit", "stp_submit_deadline", "stp_poll", "stp_drain",
           "stp_class_cost", "stp_correct", "stp_face_params", "stp_plan_describe", "stp_last_error")


class StpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"stp status {status}: {msg}")
        self.status = status


class Class(C.Structure):
    _fields_ = [("order", C.c_int), ("nquant", C.c_int), ("physics", C.c_int), ("flags", C.c_uint)]


class PlanDesc(C.Structure):
    _fields_ = [("nclass", C.c_int), ("classes", C.POINTER(Class)), ("prec", C.c_int),
                ("acc64_min_order", C.c_int), ("device", C.c_int), ("variant", C.c_int),
                ("serve_mem_budget", C.c_size_t), ("autotune", C.c_int), ("nodes", C.c_int)]


class Batch(C.Structure):
    _fields_ = [("nelem", C.c_int64), ("cls", C.c_void_p), ("off_q", C.c_void_p), ("off_coef", C.c_void_p),
                ("off_face", C.c_void_p), ("off_src", C.c_void_p), ("dt", C.c_void_p), ("h", C.c_void_p),
                ("dt_h_scalar", C.c_int), ("Q", C.c_void_p), ("params", C.c_void_p), ("A", C.c_void_p),
                ("B", C.c_void_p), ("src", C.c_void_p), ("qavg", C.c_void_p), ("favg", C.c_void_p),
                ("qface", C.c_void_p), ("fface", C.c_void_p)]


class Step(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dt", C.c_double), ("h", C.c_double),
                ("Q", C.c_void_p), ("params", C.c_void_p), ("A", C.c_void_p), ("B", C.c_void_p),
                ("favg", C.c_void_p), ("qface", C.c_void_p), ("fface", C.c_void_p), ("Qnew", C.c_void_p),
                ("fparams", C.c_void_p)]


class TicketInfo(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double), ("status", C.c_int)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def lib():
    """Load libstp.so; raise if it is not built (the product never falls back to another path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        L.stp_plan.argtypes = [C.POINTER(PlanDesc), C.POINTER(C.c_void_p)]
        L.stp_plan_free.argtypes = [C.c_void_p]
        L.stp_plan_free.restype = None
        L.stp_run.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_void_p]
        L.stp_run_noalloc.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_void_p]
        L.stp_sync.argtypes = [C.c_void_p, C.c_void_p]
        L.stp_submit.argtypes = [C.c_void_p, C.POINTER(Batch), C.POINTER(C.c_uint64)]
        L.stp_submit_deadline.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_double, C.POINTER(C.c_uint64)]
        L.stp_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(TicketInfo)]
        L.stp_drain.argtypes = [C.c_void_p]
        L.stp_class_cost.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.stp_reserve.argtypes = [C.c_void_p, C.c_int64]
        L.stp_plan_describe.argtypes = [C.c_void_p, C.c_char_p, C.c_size_t]
        L.stp_correct.argtypes = [C.c_void_p, C.POINTER(Step), C.c_void_p]
        L.stp_face_params.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.stp_last_error.argtypes = []
        L.stp_last_error.restype = C.c_char_p
        for f in ("stp_plan", "stp_run", "stp_run_noalloc", "stp_sync", "stp_reserve", "stp_submit", "stp_submit_deadline", "stp_poll",
                  "stp_drain", "stp_class_cost",
                  "stp_plan_describe", "stp_correct"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().stp_last_error().decode()


def _check(status):
    if status not in (OK, PENDING):
        raise StpError(status, last_error())
    return status


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    """A raw HIP stream handle from a torch.cuda.Stream, a handle, or None (torch's current stream)."""
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


class Plan:
    """A predictor plan (owns its device tables). classes: list of (order, nquant, physics, flags)."""

    def __init__(self, classes, prec=FP32, acc64_min_order=0, device=0, variant=VARIANT_AUTO,
                 serve_mem_budget=0, autotune=0, nodes=GAUSS_LEGENDRE):
        arr = (Class * len(classes))(*[Class(*c) for c in classes])
        self.classes = [tuple(c) for c in classes]
        self.prec = prec
        desc = PlanDesc(len(classes), arr, prec, acc64_min_order, device, variant, serve_mem_budget, autotune,
                        nodes)
        h = C.c_void_p()
        _check(lib().stp_plan(C.byref(desc), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().stp_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_nelem):
        """Preallocate heterogeneous scratch so that run() allocates nothing (graph capture)."""
        _check(lib().stp_reserve(self.handle, int(max_nelem)))

    def describe(self):
        """The plan's kernel choices (variant per class, tiling, persistent grid) as a dict."""
        import json
        buf = C.create_string_buffer(1 << 16)
        _check(lib().stp_plan_describe(self.handle, buf, len(buf)))
        return json.loads(buf.value.decode())

    def cost(self, cls=0):
        """Algorithmic (bytes, flops) of one element of class `cls`."""
        b, f = C.c_double(), C.c_double()
        _check(lib().stp_class_cost(self.handle, cls, C.byref(b), C.byref(f)))
        return b.value, f.value

    def batch(self, nelem, Q, qavg, favg, qface, dt, h, params=None, A=None, B=None, src=None, fface=None,
              cls=None, off_q=None, off_coef=None, off_face=None, off_src=None):
        """Build a stp_batch. Tensors are device tensors; dt and h are floats (host scalars) or device
        float64 tensors [nelem]."""
        b = Batch()
        b.nelem = int(nelem)
        keep = []
        if isinstance(dt, (int, float)):
            dts, hs = (C.c_double * 1)(float(dt)), (C.c_double * 1)(float(h))
            keep += [dts, hs]
            b.dt, b.h = C.cast(dts, C.c_void_p), C.cast(hs, C.c_void_p)
            b.dt_h_scalar = 1
        else:
            b.dt, b.h = _ptr(dt), _ptr(h)
            b.dt_h_scalar = 0
        for name, t in (("cls", cls), ("off_q", off_q), ("off_coef", off_coef), ("off_face", off_face),
                        ("off_src", off_src), ("Q", Q), ("params", params), ("A", A), ("B", B), ("src", src),
                        ("qavg", qavg), ("favg", favg), ("qface", qface), ("fface", fface)):
            setattr(b, name, _ptr(t))
        b._keep = keep
        return b

    def run(self, batch, stream=None):
        """Queue the predictor on `stream` (a torch.cuda.Stream, a raw handle, or None = current)."""
        return _check(lib().stp_run(self.handle, C.byref(batch), C.c_void_p(_stream(stream))))

    def sync_status(self, stream=None):
        """stp_sync: wait for `stream` and return the raw status (STP_E_INVAL if a heterogeneous batch since the
        last sync had out-of-range class ids)."""
        return lib().stp_sync(self.handle, C.c_void_p(_stream(stream)))

    def run_noalloc(self, batch, stream=None):
        """stp_run_noalloc: as run(), with the heterogeneous scratch taken from the library's static array."""
        return _check(lib().stp_run_noalloc(self.handle, C.byref(batch), C.c_void_p(_stream(stream))))

    def run_noalloc_status(self, batch, stream=0):
        """stp_run_noalloc returning the raw status (for error-path tests)."""
        return lib().stp_run_noalloc(self.handle, C.byref(batch), C.c_void_p(stream))

    def run_status(self, batch, stream=0):
        """stp_run returning the raw status (for error-path tests)."""
        return lib().stp_run(self.handle, C.byref(batch), C.c_void_p(stream))

    def correct(self, grid, dt, h, Q, favg, qface, Qnew, params=None, A=None, B=None, fface=None, fparams=None,
                stream=None):
        """Queue the corrector step on a periodic nx x ny x nz mesh (stp_correct); tensors are device tensors.
        fparams: the face-point parameters of curved curvilinear elements from face_params, or None."""
        st = Step(int(grid[0]), int(grid[1]), int(grid[2]), float(dt), float(h), _ptr(Q), _ptr(params), _ptr(A),
                  _ptr(B), _ptr(favg), _ptr(qface), _ptr(fface), _ptr(Qnew), _ptr(fparams))
        return _check(lib().stp_correct(self.handle, C.byref(st), C.c_void_p(_stream(stream))))

    def face_params(self, nelem, params, fparams=None, stream=None):
        """stp_face_params: the per-node parameters [e][n^3][12] of curved curvilinear elements at their face
        points, [e][6][n^2][12]; allocates fparams (torch, like params) when it is None."""
        if fparams is None:
            n = self.classes[0][0] + 1
            fparams = params.new_empty((int(nelem), 6, n * n, 12))
        _check(lib().stp_face_params(self.handle, C.c_int64(int(nelem)), C.c_void_p(_ptr(params)),
                                     C.c_void_p(_ptr(fparams)), C.c_void_p(_stream(stream))))
        return fparams

    def correct_status(self, step, stream=0):
        """stp_correct returning the raw status (for error-path tests)."""
        return lib().stp_correct(self.handle, C.byref(step), C.c_void_p(stream))

    def submit(self, batch):
        t = C.c_uint64()
        _check(lib().stp_submit(self.handle, C.byref(batch), C.byref(t)))
        return t.value

    def submit_deadline(self, batch, timeout_s):
        """stp_submit_deadline: parts not launched within timeout_s seconds are dropped (ticket: E_TIMEOUT)."""
        t = C.c_uint64()
        _check(lib().stp_submit_deadline(self.handle, C.byref(batch), C.c_double(timeout_s), C.byref(t)))
        return t.value

    def poll(self, ticket):
        """Returns (status, TicketInfo)."""
        info = TicketInfo()
        st = lib().stp_poll(self.handle, ticket, C.byref(info))
        return st, info

    def drain(self):
        _check(lib().stp_drain(self.handle))
