"""The C ABI library loads on any host and exports every entry point that the headers under include/
declare. No GPU compute calls are made here."""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ct_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ct_geom_create", "ct_forward", "ct_back", "ct_rlalm_solve"):
        assert required in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_1512_04564_amd import _lib
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (ct_[a-z_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_params_default_and_struct_layout():
    import ctypes
    from paper_1512_04564_amd import _lib
    p = _lib.RlalmParams()
    _lib.load().ct_rlalm_params_default(ctypes.byref(p))
    assert p.alpha == pytest.approx(1.999)
    assert p.niters == 20 and p.algorithm == 1 and p.huber == 1 and p.use_graph == 1
    assert p.delta == pytest.approx(1e-4) and p.beta == pytest.approx(1024.0)
    assert p.mu_water == pytest.approx(0.02)
    assert p.forward_split == -1
    assert p.diverge_factor == pytest.approx(2.0) and p.diverge_window == 3


def test_invalid_descriptor_is_rejected_without_touching_the_gpu():
    import ctypes
    from paper_1512_04564_amd import _lib
    L = _lib.load()
    d = _lib.GeomDesc(128, 128, 1.0, 1.0, 256, 1.0, 0.0, 0, 220, 0.0, 6.283, 541.0, 949.0, 7, 0)  # 220 % 7 != 0
    h = ctypes.c_void_p()
    assert L.ct_geom_create(ctypes.byref(d), ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG
    assert b"nsubsets" in L.ct_last_error()
    d.nsubsets = 10
    d.dsd = 400.0   # dsd < dso
    assert L.ct_geom_create(ctypes.byref(d), ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG
    assert L.ct_geom_create(None, ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG


def test_network_parameter_count_is_host_only_and_matches_the_reference():
    from oracle import unet
    from paper_1512_04564_amd import _lib
    assert _lib.load().ct_unet_num_params() == unet.n_params() == 1946305


def test_helical_descriptor_limits_are_checked_on_the_host():
    """The 3-D projectors index the padded cumulative volume and the residual block in 32 bits; a
    descriptor beyond those limits is rejected before any GPU call, as is an inconsistent one."""
    import ctypes
    from paper_1512_04564_amd import _lib, synth
    L = _lib.load()
    g = synth.HELICAL_SMALL

    def desc(**kw):
        f = dict(nx=g.nx, ny=g.ny, nz=g.nz, dx=g.dx, dy=g.dy, dz=g.dz, zc=g.zc, nb=g.nb, du=g.du,
                 u_offset=g.u_offset, nr=g.nr, dw=g.dw, w_offset=g.w_offset, nviews=g.nviews,
                 views_per_turn=g.views_per_turn, beta0=g.beta0, z0=g.z0, feed=g.feed, dso=g.dso, dsd=g.dsd,
                 nsubsets=g.nsubsets)
        f.update(kw)
        return _lib.HelixDesc(*[f[n] for n, _ in _lib.HelixDesc._fields_])

    h = ctypes.c_void_p()
    # a plane of 4096 x 4096 voxels (2^24) exceeds the 24-bit plane multiply (pixel size keeps the volume
    # inside the source circle, so the limit is what rejects it)
    big = desc(nx=4096, ny=4096, dx=0.05, dy=0.05)
    assert L.ct_helix_create(ctypes.byref(big), ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG
    assert b"volume too large" in L.ct_last_error()
    # nviews * nr * nb at 2^31 or more
    many = desc(nviews=2 ** 17, views_per_turn=2 ** 15, nr=128, nb=256, nsubsets=1, dw=g.dw / 16)
    assert L.ct_helix_create(ctypes.byref(many), ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG
    assert b"sinogram too large" in L.ct_last_error()
    bad = desc(nsubsets=7)   # 660 views, not a multiple of 7
    assert L.ct_helix_create(ctypes.byref(bad), ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG
    assert L.ct_helix_create(None, ctypes.byref(h)) == _lib.CT_ERR_INVALID_ARG
