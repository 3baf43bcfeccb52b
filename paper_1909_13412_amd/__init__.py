"""MI355X-native lattice-Boltzmann fluid two-way coupled to Brownian point
particles (Yoshida, Kinjo & Washizu, arXiv:1909.13412).

The compute path is the HIP C-ABI library ``liblbmbp.so`` (declared in
``include/lbmbp.h``); ``Lattice`` is a thin ctypes handle over it, with torch
providing device memory and the stream.  Importing the package does not load
the library; the first ``Lattice`` does, and fails loudly if it is missing.
"""
from ._abi import EXPORTS, LIB_PATH, LbmError  # noqa: F401


def __getattr__(name):
    if name in ("Lattice", "Ensemble"):
        from . import sim

        return getattr(sim, name)
    raise AttributeError(name)
