"""FP64 CPU oracle of the 3-D helical cone-beam path (test infrastructure only).

ctypes bindings to ``ct_oracle3.c``: the separable distance-driven helical projector, its brute-force
weight evaluator, the 13-direction (26-neighbour) regularizer, D_L, the cost and the relaxed OS-LALM
iteration. Only the tests and the benchmark's CPU leg use it; the HIP library never loads it.

Volumes are float64 ``[nz][ny][nx]``, sinograms ``[views][rows][bins]``; geometry comes from any object
with the ``synth.HelicalGeometry`` fields.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ct_oracle3.c")
_LIB = os.path.join(_HERE, "liboracle3.so")


def build() -> str:
    """Compile the 3-D oracle with gcc (-O2, OpenMP). Always recompiles."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dz", ctypes.c_double), ("zc", ctypes.c_double), ("nb", ctypes.c_int),
                ("du", ctypes.c_double), ("u_offset", ctypes.c_double), ("nr", ctypes.c_int),
                ("dw", ctypes.c_double), ("w_offset", ctypes.c_double), ("nviews", ctypes.c_int),
                ("views_per_turn", ctypes.c_int), ("beta0", ctypes.c_double), ("z0", ctypes.c_double),
                ("feed", ctypes.c_double), ("dso", ctypes.c_double), ("dsd", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("niters", ctypes.c_int), ("nsubsets", ctypes.c_int),
                ("rho_mode", ctypes.c_int), ("rho_fixed", ctypes.c_double), ("potential", ctypes.c_int),
                ("delta", ctypes.c_double), ("beta", ctypes.c_double), ("huber", ctypes.c_int),
                ("algorithm", ctypes.c_int), ("init_full", ctypes.c_int), ("dl_scale", ctypes.c_double),
                ("subset_order", ctypes.c_int), ("kappa", ctypes.c_int)]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        G, P = ctypes.POINTER(_Geom), ctypes.POINTER(_Params)
        L.h3_forward.argtypes = [G, _I, ctypes.c_int, _D, _D]
        L.h3_back.argtypes = [G, _I, ctypes.c_int, _D, _D]
        L.h3_weights_dense.argtypes = [G, ctypes.c_int, _D]
        L.h3_row_sweep.argtypes = [G, ctypes.c_int]
        L.h3_row_sweep.restype = ctypes.c_int
        L.h3_reg_cost.argtypes = [G, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.h3_reg_cost.restype = ctypes.c_double
        L.h3_reg_grad.argtypes = [G, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D, _D]
        L.h3_cost.argtypes = [G, _D, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.h3_cost.restype = ctypes.c_double
        L.h3_dl.argtypes = [G, _D, _D]
        L.h3_rho.argtypes = [ctypes.c_longlong, ctypes.c_double]
        L.h3_rho.restype = ctypes.c_double
        L.h3_rlalm_init.argtypes = [G, P, _D, _D, _D, _D, _D, _D]
        L.h3_rlalm_iterate.argtypes = [G, P, _D, _D, _D, _D, _D, _D, ctypes.c_longlong, ctypes.c_longlong]
        L.h3_rlalm_solve.argtypes = [G, P, _D, _D, _D, _D]
        _lib = L
    return _lib


POTENTIALS = {"hyperbola": 0, "fair": 1, "qggmrf": 2}
ORDERS = {"sequential": 0, "bitrev": 1}


def _geom(g) -> _Geom:
    return _Geom(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.zc, g.nb, g.du, g.u_offset, g.nr, g.dw, g.w_offset,
                 g.nviews, g.views_per_turn, g.beta0, g.z0, g.feed, g.dso, g.dsd)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _views(g, views):
    v = np.arange(g.nviews, dtype=np.int32) if views is None else np.ascontiguousarray(views, dtype=np.int32)
    return v, v.ctypes.data_as(_I)


def params(alpha=1.999, niters=10, nsubsets=12, rho_mode="continuation", rho_fixed=0.05, potential="hyperbola",
           delta=1e-4, beta=1024.0, huber=True, init_full=False, dl_scale=1.0, subset_order="sequential") -> _Params:
    return _Params(alpha, niters, nsubsets, {"continuation": 0, "fixed": 1}[rho_mode], rho_fixed,
                   POTENTIALS[potential], delta, beta, int(huber), 1, int(init_full), dl_scale,
                   ORDERS[subset_order], 0)


def forward(g, x, views=None) -> np.ndarray:
    v, vp = _views(g, views)
    out = np.zeros((len(v), g.nr, g.nb))
    lib().h3_forward(ctypes.byref(_geom(g)), vp, len(v), _dp(_f64(x).reshape(g.nz, g.ny, g.nx)), _dp(out))
    return out


def back(g, r, views=None) -> np.ndarray:
    v, vp = _views(g, views)
    out = np.zeros((g.nz, g.ny, g.nx))
    lib().h3_back(ctypes.byref(_geom(g)), vp, len(v), _dp(_f64(r).reshape(len(v), g.nr, g.nb)), _dp(out))
    return out


def weights_dense(g, v: int) -> np.ndarray:
    """Brute-force weights of view v: ``[nr * nb][nz * ny * nx]``."""
    out = np.zeros((g.nr * g.nb, g.nz * g.ny * g.nx))
    lib().h3_weights_dense(ctypes.byref(_geom(g)), int(v), _dp(out))
    return out


def row_sweep(g, v: int) -> bool:
    return bool(lib().h3_row_sweep(ctypes.byref(_geom(g)), int(v)))


def reg_cost(g, x, potential="hyperbola", delta=1e-4, beta=1024.0) -> float:
    return lib().h3_reg_cost(ctypes.byref(_geom(g)), _dp(_f64(x)), POTENTIALS[potential], delta, beta)


def reg_grad(g, x, potential="hyperbola", delta=1e-4, beta=1024.0, huber=True):
    x = _f64(x)
    gr, dr = np.zeros_like(x), np.zeros_like(x)
    lib().h3_reg_grad(ctypes.byref(_geom(g)), _dp(x), POTENTIALS[potential], delta, beta, int(huber), _dp(gr), _dp(dr))
    return gr, dr


def cost(g, y, w, x, potential="hyperbola", delta=1e-4, beta=1024.0) -> float:
    return lib().h3_cost(ctypes.byref(_geom(g)), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(x)), POTENTIALS[potential],
                         delta, beta)


def dl(g, w) -> np.ndarray:
    out = np.zeros((g.nz, g.ny, g.nx))
    lib().h3_dl(ctypes.byref(_geom(g)), _dp(_f64(w)), _dp(out))
    return out


def rho(k: int, alpha: float) -> float:
    return lib().h3_rho(k, alpha)


def rlalm_init(g, p: _Params, y, w, dlv, x0):
    x = _f64(x0).reshape(g.nz, g.ny, g.nx).copy()
    gv, h = np.zeros_like(x), np.zeros_like(x)
    lib().h3_rlalm_init(ctypes.byref(_geom(g)), ctypes.byref(p), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(dlv)), _dp(x),
                        _dp(gv), _dp(h))
    return x, gv, h


def rlalm_iterate(g, p: _Params, y, w, dlv, x, gv, h, t0: int, nsub: int):
    lib().h3_rlalm_iterate(ctypes.byref(_geom(g)), ctypes.byref(p), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(dlv)),
                           _dp(x), _dp(gv), _dp(h), int(t0), int(nsub))


def rlalm_solve(g, p: _Params, y, w, x0):
    """Whole solve: returns (x^(K), D_L)."""
    x = _f64(x0).reshape(g.nz, g.ny, g.nx).copy()
    dlv = np.zeros_like(x)
    lib().h3_rlalm_solve(ctypes.byref(_geom(g)), ctypes.byref(p), _dp(_f64(y)), _dp(_f64(w)), _dp(x), _dp(dlv))
    return x, dlv
