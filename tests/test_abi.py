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
