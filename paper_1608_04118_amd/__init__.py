"""MI355X-native LTNE MRT lattice Boltzmann step (Liu & He, arXiv:1608.04118).

* ``binding``  -- ctypes binding of the HIP library ``liblbm_ltne.so`` (C ABI in
  ``include/lbm_ltne.h``); the library is loaded on first use and a call fails
  loudly if it has not been built.
* ``inputs``   -- seeded synthetic workloads (parameter sets and fields).
* ``build``    -- hipcc build of the library for gfx950.
"""
from . import binding, inputs  # noqa: F401
from .binding import Lattice, LtneError, nusselt_loss  # noqa: F401
