"""MI355X (gfx950) phonon lattice Boltzmann library: Python binding.

The compute path is the HIP library ``libphonon_lbm.so`` behind the C ABI of
``include/phonon_lbm.h``; this package only marshals arguments to it.
"""
from .lbm import *  # noqa: F401,F403
from .lbm import Lattice, LBMError, library, make_instance, instance_from_case  # noqa: F401

__all__ = [n for n in dir() if n.startswith("lbm_") or n.startswith("LBM_")] + [
    "Lattice", "LBMError", "library", "make_instance", "instance_from_case"]
