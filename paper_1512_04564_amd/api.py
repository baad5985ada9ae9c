"""Python front end of libctrlalm: geometry handles, projections and the relaxed OS-LALM solver.

Same names as the C ABI (include/ct.h) minus the ``ct_`` prefix. Images are float32 CUDA tensors
``[ny][nx]``; sinograms are CUDA tensors ``[views][nb]``: float32 for the projection operators, and the
geometry's storage dtype (float32, float16 or bfloat16) for the solver's y and w. Work is enqueued on
torch's current stream (or the stream passed in). Nothing here computes: it checks shapes and forwards
pointers.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import CtError, GeomDesc, RlalmParams, TraceRow, check

__all__ = ["Geometry", "Params", "forward", "forward_noalloc", "back", "fbp", "cost", "rlalm_solve", "rlalm_status",
           "rlalm_solve_batched", "rlalm_prepare", "rlalm_init", "rlalm_iterate", "kernel_times", "Helix",
           "helix_forward", "helix_back", "helix_solve", "CtError"]


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: torch.Tensor, *, shape=None, name="tensor", dtype=torch.float32) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


STORAGE = {"f32": (0, torch.float32), "f16": (1, torch.float16), "bf16": (2, torch.bfloat16)}


class Geometry:
    """Owning wrapper of a ``ct_geom`` handle (device tables + solver workspace).

    ``storage``: "f32", "f16" or "bf16" -- the dtype of the solver's sinogram inputs y and w, and of its
    internal residual block and projector image copies (ct_geom_desc.storage)."""

    def __init__(self, geom, storage: str = "f32"):
        self.desc_py = geom
        self.storage = storage
        storage, self.sino_dtype = STORAGE[storage]
        det = {"flat": 0, "arc": 1}[geom.det] if isinstance(geom.det, str) else int(geom.det)
        d = GeomDesc(geom.nx, geom.ny, geom.dx, geom.dy, geom.nb, geom.du, geom.u_offset, det, geom.nviews,
                     geom.beta0, geom.span, geom.dso, geom.dsd, geom.nsubsets, storage)
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        check(self._lib.ct_geom_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.nx, self.ny, self.nb, self.nviews, self.nsubsets = geom.nx, geom.ny, geom.nb, geom.nviews, geom.nsubsets

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self._lib.ct_geom_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def views_in(self, subset: int) -> int:
        return self.nviews if subset == -1 else self.nviews // self.nsubsets

    @property
    def img_shape(self):
        return (self.ny, self.nx)


@dataclasses.dataclass
class Params:
    alpha: float = 1.999
    niters: int = 20
    rho_mode: str = "continuation"   # or "fixed"
    rho_fixed: float = 0.05
    potential: str = "hyperbola"     # or "fair", "qggmrf"
    delta: float = 1e-4
    beta: float = 1024.0
    huber: bool = True
    algorithm: int = 1
    subset_order: str = "sequential"  # or "bitrev"
    kappa: bool = False
    start: str = "given"             # or "zero", "fbp", "learned" (needs unet)
    init_full: bool = False
    dl_scale: float = 1.0
    mu_water: float = 0.02
    fov_radius: float = 0.0
    use_graph: bool = True
    time_kernels: bool = False
    unet: object = None              # unet.UNet for start="learned"
    forward_split: int = -1          # -1: when the launch underfills the device, 0: never, 1: always
    diverge_factor: float = 2.0      # traced solves: cost above this factor times its lowest traced value ...
    diverge_window: int = 3          # ... for this many rows in a row is CT_ERR_DIVERGED (0: never)

    def to_c(self, x_ref: torch.Tensor | None = None) -> RlalmParams:
        p = RlalmParams()
        _lib.load().ct_rlalm_params_default(ctypes.byref(p))
        p.alpha = self.alpha
        p.niters = self.niters
        p.rho_mode = {"continuation": 0, "fixed": 1}[self.rho_mode]
        p.rho_fixed = self.rho_fixed
        p.potential = {"hyperbola": 0, "fair": 1, "qggmrf": 2}[self.potential]
        p.delta = self.delta
        p.beta = self.beta
        p.huber = int(self.huber)
        p.algorithm = self.algorithm
        p.subset_order = {"sequential": 0, "bitrev": 1}[self.subset_order]
        p.kappa = int(self.kappa)
        p.start = {"given": 0, "zero": 1, "fbp": 2, "learned": 3}[self.start]
        p.unet = self.unet.handle.value if self.unet is not None else None
        p.init_full = int(self.init_full)
        p.forward_split = self.forward_split
        p.dl_scale = self.dl_scale
        p.x_ref = x_ref.data_ptr() if x_ref is not None else None
        p.mu_water = self.mu_water
        p.fov_radius = self.fov_radius
        p.use_graph = int(self.use_graph)
        p.time_kernels = int(self.time_kernels)
        p.diverge_factor = self.diverge_factor
        p.diverge_window = self.diverge_window
        return p


def forward(g: Geometry, x: torch.Tensor, subset: int = -1, out: torch.Tensor | None = None, stream=None):
    """A_m x (subset m) or A x (subset -1): ``[views][nb]`` float32."""
    nv = g.views_in(subset)
    if out is None:
        out = torch.empty((nv, g.nb), dtype=torch.float32, device=x.device)
    check(g._lib.ct_forward(g.handle, subset, _ptr(x, shape=g.img_shape, name="x"),
                            _ptr(out, shape=(nv, g.nb), name="out"), _stream_handle(stream)))
    return out


def forward_noalloc(g: Geometry, x: torch.Tensor, out: torch.Tensor, subset: int = -1, stream=None):
    """ct_forward_noalloc: A_m x into the caller's ``out`` with no device allocation in the library."""
    nv = g.views_in(subset)
    check(g._lib.ct_forward_noalloc(g.handle, subset, _ptr(x, shape=g.img_shape, name="x"),
                                    _ptr(out, shape=(nv, g.nb), name="out"), _stream_handle(stream)))
    return out


def back(g: Geometry, r: torch.Tensor, subset: int = -1, out: torch.Tensor | None = None, stream=None):
    """A_m' r (subset m) or A' r (subset -1): ``[ny][nx]`` float32."""
    nv = g.views_in(subset)
    if out is None:
        out = torch.empty(g.img_shape, dtype=torch.float32, device=r.device)
    check(g._lib.ct_back(g.handle, subset, _ptr(r, shape=(nv, g.nb), name="r"),
                         _ptr(out, shape=g.img_shape, name="out"), _stream_handle(stream)))
    return out


def fbp(g: Geometry, y: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """FBP-like start image of the sinogram y: ``[ny][nx]`` float32."""
    if out is None:
        out = torch.empty(g.img_shape, dtype=torch.float32, device=y.device)
    check(g._lib.ct_fbp(g.handle, _ptr(y, shape=(g.nviews, g.nb), name="y", dtype=g.sino_dtype),
                        _ptr(out, shape=g.img_shape, name="out"), _stream_handle(stream)))
    return out


def cost(g: Geometry, p: Params, y: torch.Tensor, w: torch.Tensor, x: torch.Tensor,
         kappa: torch.Tensor | None = None, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """PWLS cost of x (ct_cost): float64 CUDA tensor [Psi, data term, R(x)], computed on the device."""
    sino = (g.nviews, g.nb)
    sd = g.sino_dtype
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=x.device)
    cp = p.to_c()
    check(g._lib.ct_cost(g.handle, ctypes.byref(cp), _ptr(y, shape=sino, name="y", dtype=sd),
                         _ptr(w, shape=sino, name="w", dtype=sd), _ptr(x, shape=g.img_shape, name="x"),
                         _ptr(kappa, shape=g.img_shape, name="kappa") if kappa is not None else None,
                         _ptr(out, shape=(3,), name="out", dtype=torch.float64), _stream_handle(stream)))
    return out


def _rows(rows, n):
    return [dict(iter=r.iter, seconds=r.seconds, rmsd_hu=r.rmsd_hu, rmsd_hu_all=r.rmsd_hu_all, cost=r.cost,
                 rho=r.rho, finite=bool(r.finite)) for r in rows[:n] if r.iter > 0]


def rlalm_solve(g: Geometry, p: Params, y: torch.Tensor, w: torch.Tensor, x: torch.Tensor, *,
                x_ref: torch.Tensor | None = None, trace: bool = False, wait: bool = True, stream=None):
    """Run the whole solve in place on ``x``. Returns the trace rows (list of dicts) when ``trace``.

    Untraced solves are asynchronous in the library; with ``wait`` (the default) this waits for the solve
    and raises CtError(CT_ERR_DIVERGED) when it ended non-finite (``rlalm_status``). A traced solve that
    stops on divergence raises CtError with the rows taken so far in its ``rows`` attribute."""
    sino = (g.nviews, g.nb)
    cp = p.to_c(x_ref)
    if x_ref is not None:
        _ptr(x_ref, shape=g.img_shape, name="x_ref")
    rows = (TraceRow * max(p.niters, 1))() if trace else None
    sd = g.sino_dtype
    st = g._lib.ct_rlalm_solve(g.handle, ctypes.byref(cp), _ptr(y, shape=sino, name="y", dtype=sd),
                               _ptr(w, shape=sino, name="w", dtype=sd), _ptr(x, shape=g.img_shape, name="x"),
                               rows, _stream_handle(stream))
    if trace:
        try:
            check(st)
        except CtError as e:
            e.rows = _rows(rows, p.niters)
            raise
        return _rows(rows, p.niters)
    check(st)
    if wait:
        rlalm_status(g)
    return None


def rlalm_status(g: Geometry) -> None:
    """Wait for the last untraced solve on ``g``; raise CtError(CT_ERR_DIVERGED) if it ended non-finite."""
    check(g._lib.ct_rlalm_status(g.handle))


def rlalm_solve_batched(geoms, p: Params, ys, ws, xs, *, autotune=False, stream=None) -> dict:
    """Solve len(geoms) independent slices in place on each ``xs[i]`` (ct_rlalm_solve_batched).
    ``autotune``: False / 0 lockstep default shape, True / 1 tuned (lockstep or persistent), 2 or
    "persistent" the single persistent launch at its fastest shape on this batch. Returns the launch
    shape used:
    ``{"fp_waves", "largest_first", "ms_subiteration", "persistent", "blocks_per_cu", "forward_split"}``."""
    autotune = 2 if autotune == "persistent" else int(autotune)
    n = len(geoms)
    if not (len(ys) == len(ws) == len(xs) == n) or n == 0:
        raise ValueError("geoms, ys, ws and xs must be non-empty and of equal length")
    cp = p.to_c()
    VP = ctypes.c_void_p * n
    hs = VP(*[g.handle.value for g in geoms])
    yp = VP(*[_ptr(y, shape=(g.nviews, g.nb), name="y", dtype=g.sino_dtype) for g, y in zip(geoms, ys)])
    wp = VP(*[_ptr(w, shape=(g.nviews, g.nb), name="w", dtype=g.sino_dtype) for g, w in zip(geoms, ws)])
    xp = VP(*[_ptr(x, shape=g.img_shape, name="x") for g, x in zip(geoms, xs)])
    cfg = _lib.BatchConfig()
    check(geoms[0]._lib.ct_rlalm_solve_batched(hs, n, ctypes.byref(cp), yp, wp, xp, autotune, ctypes.byref(cfg),
                                               _stream_handle(stream)))
    return dict(fp_waves=cfg.fp_waves, largest_first=bool(cfg.largest_first), ms_subiteration=cfg.ms_subiteration,
                persistent=bool(cfg.persistent), blocks_per_cu=cfg.blocks_per_cu, forward_split=cfg.forward_split)


def rlalm_prepare(g: Geometry, p: Params, w: torch.Tensor, dl: torch.Tensor, kappa: torch.Tensor | None = None,
                  stream=None):
    cp = p.to_c()
    check(g._lib.ct_rlalm_prepare(g.handle, ctypes.byref(cp),
                                  _ptr(w, shape=(g.nviews, g.nb), name="w", dtype=g.sino_dtype),
                                  _ptr(dl, shape=g.img_shape, name="dl"),
                                  _ptr(kappa, shape=g.img_shape, name="kappa") if kappa is not None else None,
                                  _stream_handle(stream)))


def rlalm_init(g: Geometry, p: Params, y, w, dl, x, gv, h, stream=None):
    cp = p.to_c()
    sino = (g.nviews, g.nb)
    sd = g.sino_dtype
    check(g._lib.ct_rlalm_init(g.handle, ctypes.byref(cp), _ptr(y, shape=sino, name="y", dtype=sd),
                               _ptr(w, shape=sino, name="w", dtype=sd), _ptr(dl, shape=g.img_shape, name="dl"),
                               _ptr(x, shape=g.img_shape, name="x"), _ptr(gv, shape=g.img_shape, name="g"),
                               _ptr(h, shape=g.img_shape, name="h"), _stream_handle(stream)))


def rlalm_iterate(g: Geometry, p: Params, y, w, dl, x, gv, h, t0: int, nsub: int, kappa=None, stream=None):
    cp = p.to_c()
    sino = (g.nviews, g.nb)
    sd = g.sino_dtype
    check(g._lib.ct_rlalm_iterate(g.handle, ctypes.byref(cp), _ptr(y, shape=sino, name="y", dtype=sd),
                                  _ptr(w, shape=sino, name="w", dtype=sd), _ptr(dl, shape=g.img_shape, name="dl"),
                                  _ptr(kappa, shape=g.img_shape, name="kappa") if kappa is not None else None,
                                  _ptr(x, shape=g.img_shape, name="x"), _ptr(gv, shape=g.img_shape, name="g"),
                                  _ptr(h, shape=g.img_shape, name="h"), int(t0), int(nsub), _stream_handle(stream)))


def kernel_times(g: Geometry) -> dict:
    """Event-measured kernel totals of the last solve / iterate made with ``time_kernels=True``."""
    kt = _lib.KernelTimes()
    check(g._lib.ct_rlalm_kernel_times(g.handle, ctypes.byref(kt)))
    return dict(n_forward=kt.n_forward, n_update=kt.n_update, ms_forward=kt.ms_forward, ms_update=kt.ms_update)


class Helix:
    """Owning wrapper of a ``ct_helix`` handle: a 3-D helical cone-beam scan (include/ct_helix.h).

    ``geom``: any object with the ``synth.HelicalGeometry`` fields. Volumes are float32 CUDA tensors
    ``[nz][ny][nx]``, sinograms ``[views][rows][bins]``."""

    def __init__(self, geom):
        self.desc_py = geom
        d = _lib.HelixDesc(geom.nx, geom.ny, geom.nz, geom.dx, geom.dy, geom.dz, geom.zc, geom.nb, geom.du,
                           geom.u_offset, geom.nr, geom.dw, geom.w_offset, geom.nviews, geom.views_per_turn,
                           geom.beta0, geom.z0, geom.feed, geom.dso, geom.dsd, geom.nsubsets)
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        check(self._lib.ct_helix_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.nx, self.ny, self.nz = geom.nx, geom.ny, geom.nz
        self.nb, self.nr, self.nviews, self.nsubsets = geom.nb, geom.nr, geom.nviews, geom.nsubsets

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self._lib.ct_helix_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def views_in(self, subset: int) -> int:
        return self.nviews if subset == -1 else self.nviews // self.nsubsets

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)


def helix_forward(h: Helix, x: torch.Tensor, subset: int = -1, out: torch.Tensor | None = None, stream=None):
    """A_m x (subset m) or A x (subset -1) of a volume: ``[views][rows][bins]`` float32."""
    shape = (h.views_in(subset), h.nr, h.nb)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=x.device)
    check(h._lib.ct_helix_forward(h.handle, subset, _ptr(x, shape=h.vol_shape, name="x"),
                                  _ptr(out, shape=shape, name="out"), _stream_handle(stream)))
    return out


def helix_back(h: Helix, r: torch.Tensor, subset: int = -1, out: torch.Tensor | None = None, stream=None):
    """A_m' r (subset m) or A' r (subset -1): ``[nz][ny][nx]`` float32."""
    shape = (h.views_in(subset), h.nr, h.nb)
    if out is None:
        out = torch.empty(h.vol_shape, dtype=torch.float32, device=r.device)
    check(h._lib.ct_helix_back(h.handle, subset, _ptr(r, shape=shape, name="r"),
                               _ptr(out, shape=h.vol_shape, name="out"), _stream_handle(stream)))
    return out


def helix_solve(h: Helix, p: Params, y: torch.Tensor, w: torch.Tensor, x: torch.Tensor, stream=None) -> None:
    """3-D relaxed OS-LALM solve in place on the volume ``x`` (waits for the device; raises CtError)."""
    sino = (h.nviews, h.nr, h.nb)
    cp = p.to_c()
    check(h._lib.ct_helix_solve(h.handle, ctypes.byref(cp), _ptr(y, shape=sino, name="y"),
                                _ptr(w, shape=sino, name="w"), _ptr(x, shape=h.vol_shape, name="x"),
                                _stream_handle(stream)))
