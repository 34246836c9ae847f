"""MI355X-native nonequilibrium free-energy switching for EAM solids.

Frenkel--Ladd (Hamiltonian blending, Sec. "Free-energy difference between two
systems: Frenkel--Ladd path", Eqs. interp/einstein) and Reversible Scaling
(Eq. H_rs) Langevin MD with the irreversible work accumulated as the left-point
sum of Eq. w_irr.  The compute path is a C-ABI shared library of hand-written
HIP kernels for gfx950 (``csrc/``, declared in ``include/eamfe.h``); the Python
side only marshals arguments.

Submodules are imported explicitly (``import paper_2201_04622_amd.eamfe as E``
for the binding, ``from paper_2201_04622_amd import inputs`` for the seeded
input generators); importing the package itself loads nothing, so ``inputs``
can be used without the native library.
"""
