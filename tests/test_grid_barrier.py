"""CPU check of the bounded grid barrier that the persistent batched solve uses between its phases.

The barrier's algorithm (csrc/ct_grid_barrier.hpp) runs with one host thread per workgroup: every read
after a barrier sees every workgroup's write before it, over hundreds of phases; and when one workgroup
starts far later than the spin limit allows (a grid that is not fully resident), the waiting workgroups
raise the error flag and every workgroup returns -- none waits forever.
"""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("barrier") / "libbarrier.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-D__HIP_PLATFORM_AMD__",
                    f"-I{ROCM}/include", os.path.join(ROOT, "tests", "emu", "barrier_emu.cpp"), "-o", out],
                   check=True)
    L = ctypes.CDLL(out)
    ip = ctypes.POINTER(ctypes.c_int)
    L.barrier_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_int, ctypes.c_int, ip, ip, ip]
    return L


def run(L, nblocks, phases, spin, late=-1, late_ms=0):
    e, c, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    stale = L.barrier_run(nblocks, phases, spin, late, late_ms, ctypes.byref(e), ctypes.byref(c), ctypes.byref(x))
    return stale, e.value, c.value, x.value


@pytest.mark.parametrize("nblocks", [1, 2, 7, 16])
def test_every_read_after_the_barrier_sees_every_write(lib, nblocks):
    stale, err, done, out = run(lib, nblocks, 300, 1 << 30)
    assert (stale, err, done, out) == (0, 0, nblocks, nblocks)


def test_a_late_workgroup_raises_the_error_and_everyone_returns(lib):
    stale, err, done, out = run(lib, 8, 50, 2000, late=3, late_ms=300)
    assert err == 1 and out == 8 and done < 8
