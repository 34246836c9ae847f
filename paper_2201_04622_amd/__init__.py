"""MI355X-native nonequilibrium free-energy switching for EAM solids.

Frenkel--Ladd (Hamiltonian blending, Sec. "Free-energy difference between two
systems: Frenkel--Ladd path", Eqs. interp/einstein) and Reversible Scaling
(Eq. H_rs) Langevin MD with the irreversible work accumulated as the left-point
sum of Eq. w_irr.  The compute path is a C-ABI shared library of hand-written
HIP kernels for gfx950 (``csrc/``, declared in ``include/eamfe.h``); the Python
side only marshals arguments.

Submodules are imported explicitly (``from paper_2201_04622_amd import api``);
importing the package itself loads nothing, so the seeded input generators in
``inputs`` can be used without the native library.
"""
