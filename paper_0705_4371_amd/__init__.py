"""MI355X-native Ehrenfests'-step regularised lattice Boltzmann library.

The compute path is the gfx950 C-ABI library ``liblbm.so`` (HIP kernels in
``csrc/``, interface in ``include/lbm.h``); ``lbm`` is its ctypes binding.
"""
from . import _build  # noqa: F401

__all__ = ["lbm", "_build"]


def __getattr__(name):
    if name == "lbm":
        from . import lbm as m
        return m
    raise AttributeError(name)
