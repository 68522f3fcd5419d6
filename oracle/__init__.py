"""Oracle: a plain, slow, float64 CPU implementation of the pseudo-potential
(Shan-Chen) D3Q19 lattice Boltzmann step of Chiappini, Xue, Falcucci and
Sbragaglia, "Hydrodynamic behavior of the Pseudo-Potential lattice Boltzmann
method for interfacial flows" (arXiv:1905.09554).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check in
``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The GPU library under ``paper_1905_09554_amd`` never calls it and
shares no code with it (no tables, no helpers, no constants).

Every function works on whole arrays of torch float64 tensors laid out as
``[nz, ny, nx]`` (x fastest) and ``[19, nz, ny, nx]`` for populations; the
periodic neighbour access is ``torch.roll``.  Autograd through these functions
gives the float64 reference gradient.

Modules
-------
lattice      D3Q19 velocities, weights, the d'Humieres MRT basis (Sec. 2).
lbm          moments, psi, Shan-Chen force, equilibrium, Guo source, BGK and
             MRT collision, velocity-shift SRT, streaming, one step (Sec. 2).
diagnostics  pressure (Eq. EOS_SC), mass, momentum, ligament radius profile
             and minimum radius (Sec. 4, Fig. 5 discussion).
coexistence  the psi-specific equal-area rule and the flat-interface run
             (Sec. 3, the flat-interface simulations feeding Tables 1-2).
physics      Laplace test, capillary time and Ohnesorge number
             (Eq. Oh_Tcap), viscous Rayleigh-Plateau dispersion relation.
adjoint      reference gradients by torch autograd with checkpointing.

Pinning status of each function is listed in its module docstring.
"""
