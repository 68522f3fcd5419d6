"""MI355X-native D3Q19 pseudo-potential (Shan-Chen) lattice Boltzmann step.

The method is that of arXiv:1905.09554 (Sec. 2): a D3Q19 lattice Boltzmann
step with the single-belt Shan-Chen force, Guo-like or velocity-shift
forcing and BGK or MRT collision, on a periodic box holding a liquid
ligament.  The step lives in liblbsc.so (HIP for gfx950) behind the C ABI of
include/lbsc.h; ``lbsc`` is its ctypes binding.
"""
from . import lbsc  # noqa: F401
from .lbsc import Simulation, lattice, make_params, state_bytes  # noqa: F401
