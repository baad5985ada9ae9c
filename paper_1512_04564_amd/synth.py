"""Seeded synthetic fan-beam CT scans: random-ellipse phantoms, analytic sinograms, noise and weights.

This module is the only code shared by the HIP path's callers and the CPU oracle's tests. It simulates
the *scanner*, not the reconstruction method: it holds no projector, regularizer or update arithmetic.
Its sinograms are exact line integrals through ellipses (averaged over sub-rays per detector bin), so
they carry no discretisation of the reconstruction grid ("no inverse crime").

Geometry conventions (shared by every consumer; the reconstruction grid only matters for `truth`):

* Image ``[ny][nx]`` row-major; pixel ``(i, j)`` is centred at
  ``x_j = (j - (nx-1)/2) dx``, ``y_i = (i - (ny-1)/2) dy`` (mm).
* View ``v`` has angle ``beta_v = beta0 + span * v / nviews``; central direction ``d = (cos b, sin b)``,
  detector axis ``e = (-sin b, cos b)``; the source sits at ``S = -dso d``.
* Detector bin boundaries ``u_k = (k - nb/2 + u_offset) du`` for ``k = 0..nb``. Flat detector: the point
  at coordinate ``u`` is ``(dsd - dso) d + u e``. Arc detector: angle ``u/dsd`` about the source at radius
  ``dsd``.

The workload recipe follows the paper's XCAT acquisition (888 channels, 984 views, 541/949 mm source
distances, 1e5 incident photons; Section "XCAT phantom") reduced to a 2-D fan beam, with seeded ellipses
standing in for the XCAT phantom and the clinical scans, which are not available.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "ScanGeometry", "CFG1", "CFG2", "BATCH_CLASSES", "fov_radius", "random_ellipses", "phantom_image",
    "ray_points", "analytic_sinogram", "noisy_scan", "Scan", "MU_WATER", "UNET_SHAPES", "unet_params",
    "HelicalGeometry", "helical_geometry", "CFG3", "HELICAL_SMALL", "random_ellipsoids", "phantom_volume",
    "helical_ray_points", "analytic_helical_sinogram", "noisy_helical_scan", "HelicalScan",
]

MU_WATER = 0.02  # mm^-1; 1000 HU.  The HU scale puts air at 0.


@dataclasses.dataclass(frozen=True)
class ScanGeometry:
    nx: int
    ny: int
    dx: float
    dy: float
    nb: int
    du: float
    u_offset: float
    det: str            # "flat" or "arc"
    nviews: int
    beta0: float
    span: float
    dso: float
    dsd: float
    nsubsets: int

    def replace(self, **kw) -> "ScanGeometry":
        return dataclasses.replace(self, **kw)


#: 128x128 at 1 mm, flat 256 x 1 mm detector, 220 views over 360 deg, 10 subsets.
CFG1 = ScanGeometry(128, 128, 1.0, 1.0, 256, 1.0, 0.0, "flat", 220, 0.0, 2 * math.pi, 541.0, 949.0, 10)
#: 512x512 at 0.98 mm, flat 888 x 1.0239 mm detector, 984 views over 360 deg, 41 subsets.
CFG2 = ScanGeometry(512, 512, 0.98, 0.98, 888, 1.0239, 0.0, "flat", 984, 0.0, 2 * math.pi, 541.0, 949.0, 41)


def _batch_class(n: int, nv: int, nb: int) -> ScanGeometry:
    # Constant ~500 mm field: pixel and bin sizes scale from the 512^2 / 0.98 mm / 888-bin class.
    scale = 512.0 / n
    return ScanGeometry(n, n, 0.98 * scale, 0.98 * scale, nb, 1.0239 * 888.0 / nb, 0.0, "flat", nv, 0.0,
                        2 * math.pi, 541.0, 949.0, 41)


#: The three slice classes of the uneven batch: 256^2/492 views/444 bins, 384^2/738/666, 512^2/984/888.
BATCH_CLASSES = (_batch_class(256, 492, 444), _batch_class(384, 738, 666), _batch_class(512, 984, 888))


def fov_radius(g: ScanGeometry) -> float:
    """Radius (mm) of the disk seen by every view: the fan's half-angle seen from the source."""
    half = 0.5 * g.nb * g.du
    gam = math.atan(half / g.dsd) if g.det == "flat" else half / g.dsd
    return g.dso * math.sin(gam)


def _view_frame(g: ScanGeometry, v):
    beta = g.beta0 + g.span * np.asarray(v, dtype=np.float64) / g.nviews
    c, s = np.cos(beta), np.sin(beta)
    return c, s


def ray_points(g: ScanGeometry, v, u):
    """Source point and detector point (both ``[..., 2]``, mm) for views ``v`` and detector coords ``u``.

    ``v`` and ``u`` broadcast against each other.
    """
    c, s = _view_frame(g, v)
    u = np.asarray(u, dtype=np.float64)
    c, s, u = np.broadcast_arrays(c, s, u)
    src = np.stack([-g.dso * c, -g.dso * s], axis=-1)
    if g.det == "flat":
        off = g.dsd - g.dso
        det = np.stack([off * c - u * s, off * s + u * c], axis=-1)
    elif g.det == "arc":
        gam = u / g.dsd
        dirx = np.cos(gam) * c - np.sin(gam) * s
        diry = np.cos(gam) * s + np.sin(gam) * c
        det = src + g.dsd * np.stack([dirx, diry], axis=-1)
    else:
        raise ValueError(f"unknown detector shape {g.det!r}")
    return src, det


@dataclasses.dataclass
class Ellipse:
    cx: float
    cy: float
    a: float
    b: float
    phi: float
    mu: float       # additive value (mm^-1)


def random_ellipses(g: ScanGeometry, seed: int, n: int = 8, *, rng: np.random.Generator | None = None):
    """Body ellipse plus ``n-1`` disjoint inserts, all inside the field of view.

    Every object pixel ends up in [0.01, 0.04] mm^-1 (inserts are stored as contrast to the body).
    """
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
    rf = fov_radius(g)
    ell = []
    cx, cy = rng.uniform(-0.05, 0.05, 2) * rf
    a, b = rng.uniform(0.55, 0.80, 2) * rf
    phi = rng.uniform(0.0, math.pi)
    mu_body = rng.uniform(0.015, 0.025)
    body = Ellipse(cx, cy, a, b, phi, mu_body)
    ell.append(body)
    shrink = 2.0 * max(g.dx, g.dy)
    circles = []
    tries = 0
    while len(ell) < n:
        tries += 1
        if tries > 20000:
            raise RuntimeError("could not place ellipses")
        ea, eb = rng.uniform(0.04, 0.20, 2) * rf
        ephi = rng.uniform(0.0, math.pi)
        mu = rng.uniform(0.01, 0.04)
        # candidate centre uniformly inside the body's bounding box
        ecx = cx + rng.uniform(-1, 1) * max(a, b)
        ecy = cy + rng.uniform(-1, 1) * max(a, b)
        rad = max(ea, eb)
        t = np.linspace(0, 2 * math.pi, 72, endpoint=False)
        px, py = ecx + rad * np.cos(t), ecy + rad * np.sin(t)
        if not np.all(_inside(px, py, cx, cy, a - shrink, b - shrink, phi)):
            continue
        if any(math.hypot(ecx - ox, ecy - oy) < rad + orad for ox, oy, orad in circles):
            continue
        circles.append((ecx, ecy, rad))
        ell.append(Ellipse(ecx, ecy, ea, eb, ephi, mu - mu_body))
    return ell


def _inside(px, py, cx, cy, a, b, phi):
    c, s = math.cos(phi), math.sin(phi)
    dx, dy = px - cx, py - cy
    xr = c * dx + s * dy
    yr = -s * dx + c * dy
    return (xr / a) ** 2 + (yr / b) ** 2 <= 1.0


def phantom_image(g: ScanGeometry, ellipses, supersample: int = 4) -> np.ndarray:
    """Pixel-averaged phantom on the reconstruction grid (``[ny][nx]`` float64, mm^-1)."""
    ss = supersample
    off = (np.arange(ss) + 0.5) / ss - 0.5
    xs = ((np.arange(g.nx) - (g.nx - 1) / 2.0)[:, None] * g.dx + off[None, :] * g.dx).reshape(-1)
    ys = ((np.arange(g.ny) - (g.ny - 1) / 2.0)[:, None] * g.dy + off[None, :] * g.dy).reshape(-1)
    X, Y = np.meshgrid(xs, ys)
    img = np.zeros_like(X)
    for e in ellipses:
        img += e.mu * _inside(X, Y, e.cx, e.cy, e.a, e.b, e.phi)
    return img.reshape(g.ny, ss, g.nx, ss).mean(axis=(1, 3))


def _chords(src, det, ellipses):
    """Sum over ellipses of mu * (length of the line src->det inside the ellipse)."""
    d = det - src
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    total = np.zeros(src.shape[:-1])
    for e in ellipses:
        c, s = math.cos(e.phi), math.sin(e.phi)
        px, py = src[..., 0] - e.cx, src[..., 1] - e.cy
        qx = (c * px + s * py) / e.a
        qy = (-s * px + c * py) / e.b
        rx = (c * d[..., 0] + s * d[..., 1]) / e.a
        ry = (-s * d[..., 0] + c * d[..., 1]) / e.b
        A = rx * rx + ry * ry
        B = 2.0 * (qx * rx + qy * ry)
        C = qx * qx + qy * qy - 1.0
        disc = B * B - 4.0 * A * C
        total += e.mu * np.sqrt(np.maximum(disc, 0.0)) / A
    return total


def analytic_sinogram(g: ScanGeometry, ellipses, subrays: int = 4, views=None) -> np.ndarray:
    """Exact ellipse line integrals, averaged over ``subrays`` equally spaced rays per bin.

    Returns ``[nviews][nb]`` float64 (dimensionless) for all views, or for the listed ``views``.
    """
    v = np.arange(g.nviews) if views is None else np.asarray(views)
    k = np.arange(g.nb)
    sub = (np.arange(subrays) + 0.5) / subrays
    u = ((k[:, None] + sub[None, :]) - g.nb / 2.0 + g.u_offset) * g.du      # [nb][subrays]
    out = np.empty((len(v), g.nb))
    for a in range(0, len(v), 64):
        vv = v[a:a + 64]
        src, det = ray_points(g, vv[:, None, None], u[None, :, :])
        out[a:a + 64] = _chords(src, det, ellipses).mean(axis=-1)
    return out


@dataclasses.dataclass
class Scan:
    geom: ScanGeometry
    seed: int
    y: np.ndarray        # [nviews][nb] float32 post-log sinogram
    w: np.ndarray        # [nviews][nb] float32 statistical weights
    truth: np.ndarray    # [ny][nx] float64 supersampled phantom (mm^-1)
    line_integrals: np.ndarray  # [nviews][nb] float64 noise-free sinogram
    ellipses: list


def noisy_scan(g: ScanGeometry, seed: int, *, i0: float = 1e5, sigma: float = 5.0, n_ellipses: int = 8,
               truth: bool = True, weights: str = "counts") -> Scan:
    """One seeded scan: Poisson(I0 e^-l) + N(0, sigma^2) counts, clamped at 1, log, weights Y^2/(Y+25)
    (``weights="counts"``) or exp(-y) = Y/I0 (``weights="exp"``, the statistical weights of the paper's
    simulated scan; a scale of about 1/I0 against the default, so beta scales with them).

    ``y`` and ``w`` are rounded to float32; every consumer (GPU path and oracle) reads the same values.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ell = random_ellipses(g, seed, n_ellipses, rng=rng)
    li = analytic_sinogram(g, ell)
    counts = rng.poisson(i0 * np.exp(-li)).astype(np.float64) + rng.normal(0.0, sigma, li.shape)
    counts = np.maximum(counts, 1.0)
    y = np.log(i0 / counts).astype(np.float32)
    if weights == "exp":
        w = np.exp(-y.astype(np.float64)).astype(np.float32)
    else:
        w = (counts * counts / (counts + sigma * sigma)).astype(np.float32)
    img = phantom_image(g, ell) if truth else None
    return Scan(g, seed, y, w, img, li, ell)


# ---- warm-start network: seeded initial weights (shapes only; the network itself lives elsewhere) -----

#: Convolution shapes (c_in, c_out, kernel) of the warm-start U-Net in its canonical parameter order:
#: encoder levels 1-3 (two 3x3 convolutions each), the 256-channel bottleneck, decoder levels 3-1 (their
#: first convolution reads the upsampled lower level concatenated with the skip), and the 1x1 output.
UNET_SHAPES = (
    (1, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3), (64, 128, 3), (128, 128, 3), (128, 256, 3), (256, 256, 3),
    (384, 128, 3), (128, 128, 3), (192, 64, 3), (64, 64, 3), (96, 32, 3), (32, 32, 3), (32, 1, 1),
)


def unet_params(seed: int, out_std: float = 1e-3) -> np.ndarray:
    """Seeded initial weights, float32, flat in canonical order: per layer the weight [c_out][c_in][k][k]
    (He-normal, std sqrt(2 / (c_in k^2))) then the bias [c_out] (zero). The 1x1 output layer is drawn with
    std ``out_std`` so that the untrained network starts close to its residual identity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i, (ci, co, k) in enumerate(UNET_SHAPES):
        std = out_std if i == len(UNET_SHAPES) - 1 else math.sqrt(2.0 / (ci * k * k))
        parts.append(rng.normal(0.0, std, co * ci * k * k))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


# ---- 3-D helical cone-beam scans ---------------------------------------------------------------------
#
# Conventions: volume [nz][ny][nx], voxel (kz, i, j) centred at ((j - (nx-1)/2) dx, (i - (ny-1)/2) dy,
# zc + (kz - (nz-1)/2) dz). View v of a helix with V views per turn: angle b = beta0 + 2 pi v / V, source
# S = (-dso cos b, -dso sin b, z0 + feed v / V). A flat detector panel moves with the source, at distance
# dsd along d = (cos b, sin b, 0): the point at detector coordinates (u, w) is S + dsd d + u e + w z_hat,
# e = (-sin b, cos b, 0), with bin boundaries u_k = (k - nb/2 + u_offset) du and row boundaries
# w_l = (l - nr/2 + w_offset) dw. Sinograms are [view][row][bin].


@dataclasses.dataclass(frozen=True)
class HelicalGeometry:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    zc: float
    nb: int
    du: float
    u_offset: float
    nr: int
    dw: float
    w_offset: float
    nviews: int
    views_per_turn: int
    beta0: float
    z0: float
    feed: float
    dso: float
    dsd: float
    nsubsets: int

    def replace(self, **kw) -> "HelicalGeometry":
        return dataclasses.replace(self, **kw)


def helical_geometry(n: int, nz: int, dxy: float, dz: float, nb: int, du: float, nr: int, views_per_turn: int,
                     turns: int, pitch: float, nsubsets: int, dso: float = 541.0, dsd: float = 949.0):
    """Helix centred on the volume: a detector row is dz high at the isocentre (dw = dz dsd / dso) and the
    table moves pitch * nr * dz per turn."""
    feed = pitch * nr * dz
    return HelicalGeometry(n, n, nz, dxy, dxy, dz, 0.0, nb, du, 0.0, nr, dz * dsd / dso, 0.0,
                           views_per_turn * turns, views_per_turn, 0.0, -0.5 * turns * feed, feed, dso, dsd,
                           nsubsets)


#: 512x512x64 at 0.69 x 0.69 x 0.625 mm; flat 888 x 1.0239 mm channels x 32 rows; 984 views per turn,
#: 3 turns, pitch 1.0 (20 mm per turn); 12 subsets of 246 views.
CFG3 = helical_geometry(512, 64, 0.69, 0.625, 888, 1.0239, 32, 984, 3, 1.0, 12)
#: The same scan at a quarter of the sampling in every direction: 128x128x16 at 2.76 x 2.76 x 2.5 mm,
#: 222 channels x 8 rows, 220 views per turn, 3 turns, pitch 1.0; 12 subsets of 55 views.
HELICAL_SMALL = helical_geometry(128, 16, 2.76, 2.5, 222, 4.0956, 8, 220, 3, 1.0, 12)


def _helical_fov(g) -> float:
    return g.dso * math.sin(math.atan(0.5 * g.nb * g.du / g.dsd))


@dataclasses.dataclass
class Ellipsoid:
    cx: float
    cy: float
    cz: float
    a: float
    b: float
    c: float
    phi: float      # rotation about z
    mu: float       # additive value (mm^-1)


def random_ellipsoids(g: HelicalGeometry, seed: int, n: int = 8, *, rng: np.random.Generator | None = None):
    """Body ellipsoid plus ``n-1`` inserts with disjoint bounding cylinders, all inside the transaxial field of
    view and inside the volume's z extent (so that the data hold nothing the volume cannot represent). Every
    object voxel ends up in [0.01, 0.04] mm^-1."""
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
    rf = _helical_fov(g)
    zh = 0.5 * g.nz * g.dz
    cx, cy = rng.uniform(-0.05, 0.05, 2) * rf
    cz = g.zc + rng.uniform(-0.05, 0.05) * zh
    a, b = rng.uniform(0.55, 0.80, 2) * rf
    c = rng.uniform(0.60, 0.85) * zh
    phi = rng.uniform(0.0, math.pi)
    mu_body = rng.uniform(0.015, 0.025)
    out = [Ellipsoid(cx, cy, cz, a, b, c, phi, mu_body)]
    margin = max(g.dx, g.dz)
    placed = []   # bounding cylinders (x, y, z, radius, half height)
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > 20000:
            raise RuntimeError("could not place ellipsoids")
        ea, eb = rng.uniform(0.04, 0.15, 2) * rf
        ec = rng.uniform(0.15, 0.45) * zh
        ephi = rng.uniform(0.0, math.pi)
        mu = rng.uniform(0.01, 0.04)
        ex = cx + rng.uniform(-1, 1) * max(a, b)
        ey = cy + rng.uniform(-1, 1) * max(a, b)
        ez = cz + rng.uniform(-1, 1) * c
        rad = max(ea, eb)
        # the insert's bounding cylinder must lie inside the body shrunk by the margin
        p = np.linspace(0, 2 * math.pi, 24, endpoint=False)
        px = np.concatenate([ex + rad * np.cos(p)] * 2)
        py = np.concatenate([ey + rad * np.sin(p)] * 2)
        pz = np.concatenate([np.full(24, ez - ec), np.full(24, ez + ec)])
        if not np.all(_inside3(px, py, pz, out[0], a - margin, b - margin, c - margin)):
            continue
        if any(math.hypot(ex - ox, ey - oy) < rad + orad and abs(ez - oz) < ec + oc
               for ox, oy, oz, orad, oc in placed):
            continue
        placed.append((ex, ey, ez, rad, ec))
        out.append(Ellipsoid(ex, ey, ez, ea, eb, ec, ephi, mu - mu_body))
    return out


def _inside3(px, py, pz, e: Ellipsoid, a=None, b=None, c=None):
    a = e.a if a is None else a
    b = e.b if b is None else b
    c = e.c if c is None else c
    co, si = math.cos(e.phi), math.sin(e.phi)
    dx, dy, dz = px - e.cx, py - e.cy, pz - e.cz
    xr = co * dx + si * dy
    yr = -si * dx + co * dy
    return (xr / a) ** 2 + (yr / b) ** 2 + (dz / c) ** 2 <= 1.0


def phantom_volume(g: HelicalGeometry, ellipsoids, supersample: int = 2) -> np.ndarray:
    """Voxel-averaged phantom ``[nz][ny][nx]`` float64 (mm^-1), slice by slice."""
    ss = supersample
    off = (np.arange(ss) + 0.5) / ss - 0.5
    xs = ((np.arange(g.nx) - (g.nx - 1) / 2.0)[:, None] * g.dx + off[None, :] * g.dx).reshape(-1)
    ys = ((np.arange(g.ny) - (g.ny - 1) / 2.0)[:, None] * g.dy + off[None, :] * g.dy).reshape(-1)
    X, Y = np.meshgrid(xs, ys)
    vol = np.zeros((g.nz, g.ny, g.nx))
    for kz in range(g.nz):
        acc = np.zeros((g.ny, g.nx))
        for o in off:
            z = g.zc + (kz - (g.nz - 1) / 2.0 + o) * g.dz
            img = np.zeros_like(X)
            for e in ellipsoids:
                img += e.mu * _inside3(X, Y, z, e)
            acc += img.reshape(g.ny, ss, g.nx, ss).mean(axis=(1, 3))
        vol[kz] = acc / ss
    return vol


def helical_ray_points(g: HelicalGeometry, v, u, w):
    """Source and detector points (``[..., 3]``, mm) for views ``v`` and detector coordinates ``(u, w)``
    (broadcast against each other)."""
    v, u, w = np.broadcast_arrays(np.asarray(v, np.float64), np.asarray(u, np.float64), np.asarray(w, np.float64))
    beta = g.beta0 + 2.0 * math.pi * v / g.views_per_turn
    c, s = np.cos(beta), np.sin(beta)
    src = np.stack([-g.dso * c, -g.dso * s, g.z0 + g.feed * v / g.views_per_turn], axis=-1)
    det = src + np.stack([g.dsd * c - u * s, g.dsd * s + u * c, w], axis=-1)
    return src, det


def _chords3(src, det, ellipsoids):
    d = det - src
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    total = np.zeros(src.shape[:-1])
    for e in ellipsoids:
        co, si = math.cos(e.phi), math.sin(e.phi)
        px, py, pz = src[..., 0] - e.cx, src[..., 1] - e.cy, src[..., 2] - e.cz
        qx = (co * px + si * py) / e.a
        qy = (-si * px + co * py) / e.b
        qz = pz / e.c
        rx = (co * d[..., 0] + si * d[..., 1]) / e.a
        ry = (-si * d[..., 0] + co * d[..., 1]) / e.b
        rz = d[..., 2] / e.c
        A = rx * rx + ry * ry + rz * rz
        B = 2.0 * (qx * rx + qy * ry + qz * rz)
        C = qx * qx + qy * qy + qz * qz - 1.0
        total += e.mu * np.sqrt(np.maximum(B * B - 4.0 * A * C, 0.0)) / A
    return total


def _helical_chunk(a):
    g, ell, subrays, views = a
    return analytic_helical_sinogram(g, ell, subrays=subrays, views=views)


def analytic_helical_sinogram(g: HelicalGeometry, ellipsoids, subrays: int = 2, views=None,
                              workers: int = 1) -> np.ndarray:
    """Exact ellipsoid line integrals averaged over subrays x subrays rays per detector cell:
    ``[views][nr][nb]`` float64. ``workers`` > 1 splits the views over forked processes (call it before the
    calling process has initialised a GPU)."""
    v = np.arange(g.nviews) if views is None else np.asarray(views)
    if workers > 1 and len(v) > workers:
        import multiprocessing as mp
        parts = np.array_split(v, workers * 4)
        with mp.get_context("fork").Pool(workers) as pool:
            return np.concatenate(pool.map(_helical_chunk, [(g, ellipsoids, subrays, pv) for pv in parts]))
    sub = (np.arange(subrays) + 0.5) / subrays
    u = ((np.arange(g.nb)[:, None] + sub[None, :]) - g.nb / 2.0 + g.u_offset) * g.du     # [nb][s]
    w = ((np.arange(g.nr)[:, None] + sub[None, :]) - g.nr / 2.0 + g.w_offset) * g.dw     # [nr][s]
    out = np.empty((len(v), g.nr, g.nb))
    chunk = max(1, 2 ** 22 // (g.nr * g.nb * subrays * subrays))
    for a in range(0, len(v), chunk):
        vv = v[a:a + chunk]
        src, det = helical_ray_points(g, vv[:, None, None, None, None], u[None, None, :, None, :],
                                      w[None, :, None, :, None])
        out[a:a + chunk] = _chords3(src, det, ellipsoids).mean(axis=(-2, -1))
    return out


@dataclasses.dataclass
class HelicalScan:
    geom: HelicalGeometry
    seed: int
    y: np.ndarray        # [nviews][nr][nb] float32 post-log sinogram
    w: np.ndarray        # [nviews][nr][nb] float32 statistical weights
    truth: np.ndarray    # [nz][ny][nx] float64 voxel-averaged phantom (or None)
    ellipsoids: list


def noisy_helical_scan(g: HelicalGeometry, seed: int, *, i0: float = 1e5, sigma: float = 5.0, subrays: int = 2,
                       truth: bool = True, workers: int = 1) -> HelicalScan:
    """One seeded helical scan: Poisson(I0 e^-l) + N(0, sigma^2) counts clamped at 1, y = log(I0 / Y),
    w = Y^2 / (Y + sigma^2); y and w rounded to float32. ``workers``: processes for the line integrals."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ell = random_ellipsoids(g, seed, rng=rng)
    li = analytic_helical_sinogram(g, ell, subrays=subrays, workers=workers)
    counts = rng.poisson(i0 * np.exp(-li)).astype(np.float64) + rng.normal(0.0, sigma, li.shape)
    counts = np.maximum(counts, 1.0)
    y = np.log(i0 / counts).astype(np.float32)
    w = (counts * counts / (counts + sigma * sigma)).astype(np.float32)
    vol = phantom_volume(g, ell) if truth else None
    return HelicalScan(g, seed, y, w, vol, ell)
