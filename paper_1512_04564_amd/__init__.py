"""MI355X-native relaxed OS-LALM (OS-RLALM) for 2-D fan-beam PWLS X-ray CT.

The compute path is the HIP library ``libctrlalm.so`` (C ABI in ``include/ct.h``); this package holds
its Python binding (``api``), the in-tree build (``build``) and the seeded synthetic-scan generator
(``synth``).
"""
from . import synth  # noqa: F401

__all__ = ["synth", "api"]


def __getattr__(name):
    # The binding imports torch; load it lazily so that synth alone stays light.
    if name == "api":
        import importlib
        return importlib.import_module(__name__ + ".api")
    raise AttributeError(name)
