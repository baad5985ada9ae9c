"""CPU emulation of the 3-D helical kernels against the FP64 oracle, with every device read bounds-checked.

The per-thread bodies that the HIP kernels run (csrc/ct_helix_body.hpp) are compiled for the host with g++
and driven over the kernels' own grids (tests/emu/helix_emu.cpp); each table, volume and residual read
goes through a checked accessor. This pins, before any GPU run, the index arithmetic of the forward
projector, the gather back-projector and the 26-neighbour stencil, and their FP32 results against the
oracle (1e-5 relative, norm-wise and as the largest element difference over the largest element).
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import helical as H
from paper_1512_04564_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1512_04564_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dz", ctypes.c_double), ("zc", ctypes.c_double), ("nb", ctypes.c_int),
                ("du", ctypes.c_double), ("u_offset", ctypes.c_double), ("nr", ctypes.c_int), ("dw", ctypes.c_double),
                ("w_offset", ctypes.c_double), ("nviews", ctypes.c_int), ("views_per_turn", ctypes.c_int),
                ("beta0", ctypes.c_double), ("z0", ctypes.c_double), ("feed", ctypes.c_double),
                ("dso", ctypes.c_double), ("dsd", ctypes.c_double), ("nsubsets", ctypes.c_int)]


def desc(g):
    return Desc(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.zc, g.nb, g.du, g.u_offset, g.nr, g.dw, g.w_offset, g.nviews,
                g.views_per_turn, g.beta0, g.z0, g.feed, g.dso, g.dsd, g.nsubsets)


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("emu") / "libhelixemu.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
                    os.path.join(ROOT, "tests", "emu", "helix_emu.cpp"), os.path.join(CSRC, "ct_helix_tables.cpp"),
                    os.path.join(CSRC, "ct_geom.cpp"), "-o", out, f"-L{ROCM}/lib", "-lamdhip64"], check=True)
    L = ctypes.CDLL(out)
    fp = ctypes.POINTER(ctypes.c_float)
    ll = ctypes.POINTER(ctypes.c_longlong)
    L.hemu_forward.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, fp, ll]
    L.hemu_back.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, fp, ll]
    L.hemu_reg.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, ctypes.c_int, ctypes.c_double,
                           ctypes.c_double, ctypes.c_int, fp, fp, ll]
    L.hemu_error.restype = ctypes.c_char_p
    return L


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def run_forward(L, g, x, views):
    vs, vst, nv = views
    p = np.zeros((nv, g.nr, g.nb), dtype=np.float32)
    first = ctypes.c_longlong(0)
    n = L.hemu_forward(ctypes.byref(desc(g)), vs, vst, nv, fptr(f32(x)), fptr(p), ctypes.byref(first))
    assert n >= 0, L.hemu_error()
    assert n == 0, f"{n} out-of-range reads, first index {first.value}"
    return p


def run_back(L, g, r, views):
    vs, vst, nv = views
    x = np.zeros((g.nz, g.ny, g.nx), dtype=np.float32)
    first = ctypes.c_longlong(0)
    n = L.hemu_back(ctypes.byref(desc(g)), vs, vst, nv, fptr(f32(r)), fptr(x), ctypes.byref(first))
    assert n >= 0, L.hemu_error()
    assert n == 0, f"{n} out-of-range reads, first index {first.value}"
    return x


def check_close(a, b, tol=1e-5):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    elem = np.max(np.abs(a - b)) / np.max(np.abs(b))
    assert rel <= tol and elem <= tol, (rel, elem)
    return rel, elem


GEOMS = {
    "tiny_ties": synth.HelicalGeometry(5, 4, 3, 1.3, 0.9, 1.1, 0.2, 7, 2.0, 0.3, 4, 1.7, -0.2, 12, 8, 0.0, -2.0, 3.0,
                                       20.0, 40.0, 3),
    # ragged sizes: not multiples of the 64-bin block, the 8-row block, the 8 x 8 tile or the 32-voxel z span
    "ragged": synth.HelicalGeometry(37, 29, 70, 1.1, 0.9, 0.6, 0.4, 97, 1.7, -0.3, 11, 1.2, 0.25, 40, 16, 0.1, -9.0,
                                    6.0, 300.0, 560.0, 4),
    # channels four times finer than the voxels: columns meet 5 to 9 bins, more than the back-projector keeps in
    # registers, and rows thinner than the voxels (the fallback paths of both loops)
    "fine_detector": synth.HelicalGeometry(11, 9, 6, 2.0, 2.0, 1.5, 0.0, 61, 0.9, 0.2, 9, 0.7, 0.1, 24, 12, 0.3,
                                           -4.0, 4.0, 60.0, 110.0, 2),
    # a quarter of the 512^2 x 64 helical scan's sampling in each direction: 128^2 x 16, 222 x 8, 3 x 220 views
    "helical_small": synth.HELICAL_SMALL,
}


@pytest.mark.parametrize("name", list(GEOMS))
def test_forward_emulation_matches_oracle(emu, name):
    g = GEOMS[name]
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 0.03, (g.nz, g.ny, g.nx))
    views = (0, 1, g.nviews) if name != "helical_small" else (5, g.nsubsets, g.nviews // g.nsubsets)
    p = run_forward(emu, g, x, views)
    vs, vst, nv = views
    po = H.forward(g, f32(x).astype(np.float64), views=np.arange(vs, vs + vst * nv, vst))
    check_close(p, po)


@pytest.mark.parametrize("name", list(GEOMS))
def test_back_emulation_matches_oracle(emu, name):
    g = GEOMS[name]
    rng = np.random.default_rng(2)
    views = (0, 1, g.nviews) if name != "helical_small" else (7, g.nsubsets, g.nviews // g.nsubsets)
    vs, vst, nv = views
    r = rng.standard_normal((nv, g.nr, g.nb))
    x = run_back(emu, g, r, views)
    xo = H.back(g, f32(r).astype(np.float64), views=np.arange(vs, vs + vst * nv, vst))
    check_close(x, xo)


def test_emulated_pair_is_adjoint(emu):
    g = GEOMS["ragged"]
    rng = np.random.default_rng(3)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.nviews, g.nr, g.nb))
    views = (0, 1, g.nviews)
    lhs = float(np.vdot(run_forward(emu, g, x, views).astype(np.float64), f32(r)))
    rhs = float(np.vdot(f32(x), run_back(emu, g, r, views).astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_ones_volume_emulation(emu):
    """The all-ones volume (the D_L pass) through the same body."""
    g = GEOMS["ragged"]
    p = run_forward(emu, g, np.ones((g.nz, g.ny, g.nx)), (0, 1, g.nviews))
    check_close(p, H.forward(g, np.ones((g.nz, g.ny, g.nx))))


@pytest.mark.parametrize("pot,huber", [("hyperbola", 1), ("fair", 1), ("qggmrf", 1), ("hyperbola", 0)])
def test_stencil_emulation_matches_oracle(emu, pot, huber):
    g = GEOMS["ragged"]
    rng = np.random.default_rng(4)
    x = f32(rng.uniform(0.0, 4e-4, (g.nz, g.ny, g.nx)))
    gr = np.zeros_like(x)
    dr = np.zeros_like(x)
    first = ctypes.c_longlong(0)
    n = emu.hemu_reg(g.nx, g.ny, g.nz, fptr(x), H.POTENTIALS[pot], 1e-4, 1024.0, huber, fptr(gr), fptr(dr),
                     ctypes.byref(first))
    assert n == 0, first.value
    gro, dro = H.reg_grad(g, x.astype(np.float64), potential=pot, huber=bool(huber))
    check_close(gr, gro, 2e-5)
    check_close(dr, dro, 2e-5)


def test_full_size_emulation_on_three_views(emu):
    """The 512^2 x 64 / 888 x 32 / 2952-view scan: subset 123 of 984 (views 123, 1107, 2091; view 123 sits at
    45 degrees) through the emulated kernels, without an out-of-range read, against the oracle."""
    g = synth.CFG3
    views = (123, 984, 3)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 0.03, (g.nz, g.ny, g.nx))
    p = run_forward(emu, g, x, views)
    check_close(p, H.forward(g, f32(x).astype(np.float64), views=[123, 1107, 2091]))
    r = rng.standard_normal((3, g.nr, g.nb))
    b = run_back(emu, g, r, views)
    check_close(b, H.back(g, f32(r).astype(np.float64), views=[123, 1107, 2091]))
