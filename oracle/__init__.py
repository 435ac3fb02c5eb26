"""FP64 CPU oracle for the linear ADER-DG space-time predictor (arXiv:2003.12787).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package. The HIP product path never imports it, and the two share no code.

The arithmetic lives in ``stp_oracle.c`` (plain C, FP64, one element at a time, pthreads across
elements). This module only marshals numpy arrays into it. See the header of ``stp_oracle.c`` for the
equations and the reading of the paper that each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ACOUSTIC, ELASTIC, GENERIC, ELASTIC_CURV = 0, 1, 2, 3
NPARAM = {ACOUSTIC: 2, ELASTIC: 3, ELASTIC_CURV: 12}
NQUANT = {ACOUSTIC: 4, ELASTIC: 9, ELASTIC_CURV: 9}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no BLAS, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Args(C.Structure):
    _fields_ = [
        ("N", C.c_int), ("m", C.c_int), ("physics", C.c_int),
        ("has_A", C.c_int), ("coef_per_element", C.c_int), ("has_src", C.c_int),
        ("nelem", C.c_long),
        ("Q", C.c_void_p), ("params", C.c_void_p), ("A", C.c_void_p), ("B", C.c_void_p),
        ("src", C.c_void_p), ("dt", C.c_void_p), ("h", C.c_void_p),
        ("qavg", C.c_void_p), ("favg", C.c_void_p), ("qface", C.c_void_p), ("fface", C.c_void_p),
        ("favg_fig5", C.c_void_p), ("nthreads", C.c_int), ("nodes", C.c_int),
    ]


_lib = None


def _load(path):
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.oracle_gl_nodes.argtypes = [C.c_int, dp, dp]
    L.oracle_dmatrix.argtypes = [C.c_int, dp, dp]
    L.oracle_lagrange_at.argtypes = [C.c_int, dp, C.c_double, dp]
    L.oracle_contract.argtypes = [C.c_int, C.c_int, dp, C.c_int, dp, dp]
    L.oracle_preset_B.argtypes = [C.c_int, C.c_int, dp, dp]
    L.oracle_gll_nodes.argtypes = [C.c_int, dp, dp]
    L.oracle_apply_Vd.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p, dp, dp, dp]
    L.oracle_stp.argtypes = [C.POINTER(_Args)]
    L.oracle_default_threads.argtypes = []
    for f in ("oracle_gl_nodes", "oracle_gll_nodes", "oracle_dmatrix", "oracle_lagrange_at", "oracle_contract",
              "oracle_preset_B", "oracle_apply_Vd", "oracle_stp", "oracle_default_threads"):
        getattr(L, f).restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _load(_LIB)
    return _lib


class using:
    """Context manager that routes this module's functions through another build of the oracle
    source (used by the mutation tests, which compile deliberately broken copies)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} failed with status {rc}")


def gll_nodes(n: int):
    """Gauss-Lobatto nodes (ascending, including 0 and 1) and weights on [0, 1]; n >= 2."""
    xi, w = np.zeros(n), np.zeros(n)
    _check(lib().oracle_gll_nodes(n, _p(xi), _p(w)), "gll_nodes")
    return xi, w


def nodes_of(n: int, family: int = 0):
    """Nodes and weights of the family: 0 Gauss-Legendre, 1 Gauss-Lobatto."""
    return gll_nodes(n) if family == 1 else gl_nodes(n)


def gl_nodes(n: int):
    """Gauss-Legendre nodes (ascending) and weights on [0, 1]."""
    xi, w = np.zeros(n), np.zeros(n)
    _check(lib().oracle_gl_nodes(n, _p(xi), _p(w)), "gl_nodes")
    return xi, w


def dmatrix(n: int):
    """D[i, j] = l_j'(xi_i) on the n Gauss-Legendre nodes of [0, 1]."""
    xi, _ = gl_nodes(n)
    D = np.zeros((n, n))
    _check(lib().oracle_dmatrix(n, _p(xi), _p(D)), "dmatrix")
    return D


def lagrange_at(n: int, x: float):
    xi, _ = gl_nodes(n)
    out = np.zeros(n)
    _check(lib().oracle_lagrange_at(n, _p(xi), float(x), _p(out)), "lagrange_at")
    return out


def contract(M, axis: int, u):
    """out[..i..][s] = sum_j M[i, j] u[..j..][s] along spatial axis 0=x, 1=y, 2=z of u[z, y, x, s]."""
    M = _f64(M)
    u = _f64(u)
    n, m = u.shape[0], u.shape[3]
    out = np.zeros_like(u)
    _check(lib().oracle_contract(n, m, _p(M), axis, _p(u), _p(out)), "contract")
    return out


def preset_B(physics: int, par):
    """B_d matrices [3, m, m] of one node for a physics preset."""
    m = NQUANT[physics]
    par = _f64(par)
    B = np.zeros((3, m, m))
    _check(lib().oracle_preset_B(physics, m, _p(par), _p(B)), "preset_B")
    return B


def apply_Vd(N: int, h: float, d: int, B3, u, A3=None):
    """V_d(u) of one element; B3/A3 are per-node matrices [3, n^3, m, m]; u is [n^3, m]."""
    B3 = _f64(B3)
    u = _f64(u)
    m = u.shape[-1]
    out = np.zeros_like(u)
    Ap = None
    if A3 is not None:
        A3 = _f64(A3)
        Ap = A3.ctypes.data
    _check(lib().oracle_apply_Vd(N, m, float(h), d, Ap, _p(B3), _p(u), _p(out)), "apply_Vd")
    return out


def stp(N: int, physics: int, Q, dt, h, params=None, A=None, B=None, src=None,
        coef_per_element: bool = False, fig5: bool = False, nthreads: int = 0, nodes: int = 0):
    """Batched FP64 STP. Q is [E, n^3, m] (any shape with that size). dt and h are scalars or [E].

    Returns a dict with qavg [E, n^3, m], favg [E, 3, n^3, m], qface [E, 6, n^2, m], and fface
    (if A is given) and favg_fig5 (if fig5).
    """
    n = N + 1
    nn = n ** 3
    Q = _f64(Q)
    E = Q.shape[0]
    m = Q.size // max(E, 1) // nn if E else (NQUANT.get(physics) or B.shape[-1])
    Q = Q.reshape(E, nn, m)
    dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (E,)).copy())
    h = _f64(np.broadcast_to(np.asarray(h, dtype=np.float64), (E,)).copy())
    out = {
        "qavg": np.zeros((E, nn, m)),
        "favg": np.zeros((E, 3, nn, m)),
        "qface": np.zeros((E, 6, n * n, m)),
    }
    keep = [Q, dt, h]
    a = _Args()
    a.N, a.m, a.physics = N, m, physics
    a.has_A = int(A is not None)
    a.coef_per_element = int(bool(coef_per_element))
    a.has_src = int(src is not None)
    a.nelem = E
    a.Q = Q.ctypes.data
    for name, arr in (("params", params), ("A", A), ("B", B), ("src", src)):
        if arr is not None:
            arr = _f64(arr)
            keep.append(arr)
            setattr(a, name, arr.ctypes.data)
    a.dt, a.h = dt.ctypes.data, h.ctypes.data
    a.qavg, a.favg, a.qface = (out[k].ctypes.data for k in ("qavg", "favg", "qface"))
    if A is not None:
        out["fface"] = np.zeros((E, 6, n * n, m))
        a.fface = out["fface"].ctypes.data
    if fig5:
        out["favg_fig5"] = np.zeros((E, 3, nn, m))
        a.favg_fig5 = out["favg_fig5"].ctypes.data
    a.nthreads = int(nthreads)
    a.nodes = int(nodes)  # 0 Gauss-Legendre, 1 Gauss-Lobatto
    _check(lib().oracle_stp(C.byref(a)), "stp")
    del keep
    return out


def default_threads() -> int:
    return int(lib().oracle_default_threads())
