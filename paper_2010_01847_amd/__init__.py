"""MI355X (gfx950) phonon lattice Boltzmann library: Python binding.

The compute path is the HIP library ``libphonon_lbm.so`` behind the C ABIs of
``include/phonon_lbm.h`` (D2Q8) and ``include/phonon_d3q14.h`` (D3Q14, module
``d3q14``); this package only marshals arguments to it.
"""
from . import d3q14  # noqa: F401
from .lbm import *  # noqa: F401,F403
from .lbm import Lattice, LBMError, library, make_instance, instance_from_case  # noqa: F401

__all__ = [n for n in dir() if n.startswith("lbm_") or n.startswith("LBM_")] + [
    "Lattice", "LBMError", "library", "make_instance", "instance_from_case"]
