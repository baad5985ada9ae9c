"""FP64 CPU oracle (test infrastructure only).

Python bindings (ctypes) to ``ct_oracle.c``: the plain, slow reference that the HIP path is checked
against. Only the tests, the smoke check and the benchmark's CPU-baseline leg use it; the HIP library
never loads it, and it shares no code with the HIP library.

Each wrapper takes and returns float64 numpy arrays; geometry comes from any object with the
``synth.ScanGeometry`` fields.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Always recompiles."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nb", ctypes.c_int), ("du", ctypes.c_double), ("u_offset", ctypes.c_double),
                ("det", ctypes.c_int), ("nviews", ctypes.c_int), ("beta0", ctypes.c_double),
                ("span", ctypes.c_double), ("dso", ctypes.c_double), ("dsd", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("niters", ctypes.c_int), ("nsubsets", ctypes.c_int),
                ("rho_mode", ctypes.c_int), ("rho_fixed", ctypes.c_double), ("potential", ctypes.c_int),
                ("delta", ctypes.c_double), ("beta", ctypes.c_double), ("huber", ctypes.c_int),
                ("algorithm", ctypes.c_int), ("init_full", ctypes.c_int), ("dl_scale", ctypes.c_double),
                ("subset_order", ctypes.c_int), ("kappa", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def _declare(L):
    G = ctypes.POINTER(_Geom)
    P = ctypes.POINTER(_Params)
    L.or_forward.argtypes = [G, _I, ctypes.c_int, _D, _D]
    L.or_back.argtypes = [G, _I, ctypes.c_int, _D, _D]
    L.or_view_scale.argtypes = [G, ctypes.c_int, _D, _I]
    L.or_line_boundaries.argtypes = [G, ctypes.c_int, ctypes.c_int, _D]
    L.or_row_sweep.argtypes = [G, ctypes.c_int]
    L.or_row_sweep.restype = ctypes.c_int
    L.or_reg_cost.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.or_reg_cost.restype = ctypes.c_double
    L.or_reg_grad.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, _D, _D]
    L.or_subset_views.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I]
    L.or_subset_views.restype = ctypes.c_int
    L.or_cost.argtypes = [G, _D, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.or_cost.restype = ctypes.c_double
    L.or_dl.argtypes = [G, _D, _D]
    L.or_data_grad.argtypes = [G, _D, _D, _D, _D]
    L.or_rho.argtypes = [ctypes.c_longlong, ctypes.c_double]
    L.or_rho.restype = ctypes.c_double
    L.or_rlalm_init.argtypes = [G, P, _D, _D, _D, _D, _D, _D]
    L.or_rlalm_iterate.argtypes = [G, P, _D, _D, _D, _D, _D, _D, _D, ctypes.c_longlong, ctypes.c_longlong]
    L.or_kappa.argtypes = [G, _D, _D]
    L.or_subset_order.argtypes = [ctypes.c_int, ctypes.c_int, _I]
    L.or_reg_grad_k.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, _D, _D, _D]
    L.or_reg_cost_k.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
    L.or_reg_cost_k.restype = ctypes.c_double
    L.or_rlalm_solve.argtypes = [G, P, _D, _D, _D, _D, _D, _U8, ctypes.c_double, _D]
    L.or_xstar.argtypes = [G, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, ctypes.c_int,
                           ctypes.c_double, ctypes.c_double, _D]
    L.or_xstar.restype = ctypes.c_int
    L.or_fbp.argtypes = [G, _D, _D]
    L.or_num_threads.restype = ctypes.c_int
    L.or_set_num_threads.argtypes = [ctypes.c_int]
    L.or_set_num_threads.restype = None


def _geom(g) -> _Geom:
    det = {"flat": 0, "arc": 1}[g.det]
    return _Geom(g.nx, g.ny, g.dx, g.dy, g.nb, g.du, g.u_offset, det, g.nviews, g.beta0, g.span, g.dso, g.dsd)


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing legs)."""
    lib().or_set_num_threads(int(n))


def subset_views(nviews: int, M: int, m: int) -> np.ndarray:
    """Interleaved subset m of M: views v with v mod M == m (ascending)."""
    buf = np.zeros(nviews, dtype=np.int32)
    n = lib().or_subset_views(nviews, M, m, buf.ctypes.data_as(_I))
    return buf[:n].copy()


def _views(g, views):
    if views is None:
        views = np.arange(g.nviews, dtype=np.int32)
    return np.ascontiguousarray(np.asarray(views, dtype=np.int32))


def forward(g, x, views=None) -> np.ndarray:
    """A x for the listed views (default all): ``[len(views)][nb]``."""
    v = _views(g, views)
    x = _f64(x).reshape(g.ny, g.nx)
    p = np.zeros((len(v), g.nb))
    G = _geom(g)
    lib().or_forward(ctypes.byref(G), v.ctypes.data_as(_I), len(v), _dp(x), _dp(p))
    return p


def back(g, r, views=None) -> np.ndarray:
    """A' r for the listed views (default all): ``[ny][nx]``."""
    v = _views(g, views)
    r = _f64(r).reshape(len(v), g.nb)
    x = np.zeros((g.ny, g.nx))
    G = _geom(g)
    lib().or_back(ctypes.byref(G), v.ctypes.data_as(_I), len(v), _dp(r), _dp(x))
    return x


def view_scale(g, v: int):
    s = np.zeros(g.nb)
    rs = ctypes.c_int(0)
    G = _geom(g)
    lib().or_view_scale(ctypes.byref(G), v, _dp(s), ctypes.byref(rs))
    return s, bool(rs.value)


def line_boundaries(g, v: int, l: int) -> np.ndarray:
    b = np.zeros(g.nb + 1)
    G = _geom(g)
    lib().or_line_boundaries(ctypes.byref(G), v, l, _dp(b))
    return b


def row_sweep(g, v: int) -> bool:
    G = _geom(g)
    return bool(lib().or_row_sweep(ctypes.byref(G), v))


POTENTIALS = {"hyperbola": 0, "fair": 1, "qggmrf": 2}


def reg_cost(x, potential="hyperbola", delta=1e-4, beta=1024.0) -> float:
    x = _f64(x)
    ny, nx = x.shape
    return lib().or_reg_cost(nx, ny, _dp(x), POTENTIALS[potential], delta, beta)


def reg_grad(x, potential="hyperbola", delta=1e-4, beta=1024.0, huber=True):
    """(grad R(x), D_R(x)) with Huber curvature (or maximum curvature when huber=False)."""
    x = _f64(x)
    ny, nx = x.shape
    gr = np.zeros_like(x)
    dr = np.zeros_like(x)
    lib().or_reg_grad(nx, ny, _dp(x), POTENTIALS[potential], delta, beta, int(huber), _dp(gr), _dp(dr))
    return gr, dr


def cost(g, y, w, x, potential="hyperbola", delta=1e-4, beta=1024.0) -> float:
    G = _geom(g)
    return lib().or_cost(ctypes.byref(G), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(x).reshape(g.ny, g.nx)),
                         POTENTIALS[potential], delta, beta)


def dl(g, w) -> np.ndarray:
    """D_L = A' (w .* A 1) over all views."""
    out = np.zeros((g.ny, g.nx))
    G = _geom(g)
    lib().or_dl(ctypes.byref(G), _dp(_f64(w)), _dp(out))
    return out


def data_grad(g, y, w, x) -> np.ndarray:
    out = np.zeros((g.ny, g.nx))
    G = _geom(g)
    lib().or_data_grad(ctypes.byref(G), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(x).reshape(g.ny, g.nx)), _dp(out))
    return out


def rho(k: int, alpha: float) -> float:
    return lib().or_rho(k, alpha)


ORDERS = {"sequential": 0, "bitrev": 1}


def params(alpha=1.999, niters=20, nsubsets=10, rho_mode="continuation", rho_fixed=0.05, potential="hyperbola",
           delta=1e-4, beta=1024.0, huber=True, algorithm=1, init_full=False, dl_scale=1.0,
           subset_order="sequential", kappa=False) -> _Params:
    return _Params(alpha, niters, nsubsets, {"continuation": 0, "fixed": 1}[rho_mode], rho_fixed,
                   POTENTIALS[potential], delta, beta, int(huber), algorithm, int(init_full), dl_scale,
                   ORDERS[subset_order], int(kappa))


def subset_order(M: int, kind="sequential") -> np.ndarray:
    out = np.zeros(M, dtype=np.int32)
    lib().or_subset_order(M, ORDERS[kind], out.ctypes.data_as(_I))
    return out


def kappa(g, w) -> np.ndarray:
    """Certainty weights sqrt(A'w / A'1) over all views."""
    out = np.zeros((g.ny, g.nx))
    G = _geom(g)
    lib().or_kappa(ctypes.byref(G), _dp(_f64(w)), _dp(out))
    return out


def reg_grad_kappa(x, kap, potential="hyperbola", delta=1e-4, beta=1024.0, huber=True):
    x = _f64(x)
    ny, nx = x.shape
    gr = np.zeros_like(x)
    dr = np.zeros_like(x)
    lib().or_reg_grad_k(nx, ny, _dp(x), POTENTIALS[potential], delta, beta, int(huber), _dp(_f64(kap)), _dp(gr),
                        _dp(dr))
    return gr, dr


def reg_cost_kappa(x, kap, potential="hyperbola", delta=1e-4, beta=1024.0) -> float:
    x = _f64(x)
    ny, nx = x.shape
    return lib().or_reg_cost_k(nx, ny, _dp(x), POTENTIALS[potential], delta, beta, _dp(_f64(kap)))


def rlalm_init(g, p: _Params, y, w, dlv, x0):
    x = _f64(x0).reshape(g.ny, g.nx).copy()
    gv = np.zeros_like(x)
    h = np.zeros_like(x)
    G = _geom(g)
    lib().or_rlalm_init(ctypes.byref(G), ctypes.byref(p), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(dlv)), _dp(x),
                        _dp(gv), _dp(h))
    return x, gv, h


def rlalm_iterate(g, p: _Params, y, w, dlv, x, gv, h, t0: int, nsub: int, kap=None):
    """Advance the state in place by nsub subiterations starting at subiteration index t0."""
    G = _geom(g)
    kp = _dp(_f64(kap)) if kap is not None else None
    lib().or_rlalm_iterate(ctypes.byref(G), ctypes.byref(p), _dp(_f64(y)), _dp(_f64(w)), _dp(_f64(dlv)), kp, _dp(x),
                           _dp(gv), _dp(h), t0, nsub)


def rlalm_solve(g, p: _Params, y, w, x0, xref=None, mask=None, mu_w=0.02):
    """Run Algorithm 1 (or 2): returns (x^(K), D_L, rmsd_hu trace or None)."""
    x = _f64(x0).reshape(g.ny, g.nx).copy()
    dlv = np.zeros_like(x)
    trace = None
    G = _geom(g)
    args = [ctypes.byref(G), ctypes.byref(p), _dp(_f64(y)), _dp(_f64(w)), _dp(x), _dp(dlv)]
    if xref is not None:
        xr = _f64(xref).reshape(g.ny, g.nx)
        mk = np.ascontiguousarray(np.ones_like(x, dtype=np.uint8) if mask is None else mask.astype(np.uint8))
        trace = np.zeros(p.niters)
        args += [_dp(xr), mk.ctypes.data_as(_U8), mu_w, _dp(trace)]
    else:
        args += [None, None, mu_w, None]
    lib().or_rlalm_solve(*args)
    return x, dlv, trace


def xstar(g, y, w, x0, potential="hyperbola", delta=1e-4, beta=1024.0, maxit=5000, step_tol=2e-7,
          kkt_tol=1e-8):
    """Converged PWLS solution by preconditioned projected FGM with adaptive restart.

    Returns (x*, iterations, kkt residual)."""
    x = _f64(x0).reshape(g.ny, g.nx).copy()
    kkt = ctypes.c_double(0.0)
    G = _geom(g)
    n = lib().or_xstar(ctypes.byref(G), _dp(_f64(y)), _dp(_f64(w)), POTENTIALS[potential], delta, beta, _dp(x),
                       maxit, step_tol, kkt_tol, ctypes.byref(kkt))
    return x, n, kkt.value


def fbp(g, y) -> np.ndarray:
    x = np.zeros((g.ny, g.nx))
    G = _geom(g)
    lib().or_fbp(ctypes.byref(G), _dp(_f64(y)), _dp(x))
    return x


def fov_mask(g, radius: float) -> np.ndarray:
    """Pixels whose centres lie within ``radius`` mm of the isocentre."""
    xs = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.dx
    ys = (np.arange(g.ny) - (g.ny - 1) / 2.0) * g.dy
    X, Y = np.meshgrid(xs, ys)
    return (X * X + Y * Y) <= radius * radius


def rmsd_hu(x, xref, mask=None, mu_w=0.02) -> float:
    d = np.asarray(x, dtype=np.float64) - np.asarray(xref, dtype=np.float64)
    if mask is not None:
        d = d[mask]
    return float(1000.0 / mu_w * np.sqrt(np.mean(d * d)))
