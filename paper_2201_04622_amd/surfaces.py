"""Surface excess free energy by Frenkel--Ladd switching.

The defect extension of the summary section: a system of N atoms of the
crystal with a free surface of total area A has the free energy
F_surf = F_bulk + gamma A, where F_bulk is that of N atoms of the perfect
bulk crystal, so gamma = (F_surf - F_bulk) / A.  Both free energies come
from the FL path of the bulk section (Eq. W12 in Eq. fl, with the fixed
centre-of-mass term Eq. cm); the same N, T, k and mass enter both, so the
Einstein reference cancels except through the centre-of-mass term, whose
volume is each system's own box.

A slab is the bulk supercell with empty space added to the box along z
(``inputs.Replica.vacuum``): x and y stay periodic, and along z the periodic
images of the crystal are separated by the vacuum, so the crystal has two
free faces normal to z (the (001) faces of the cubic cells, the basal faces
of hcp), A = 2 Lx Ly.  With a vacuum wider than the cutoff no atom interacts
across it.  The kernels are unchanged: a slab is a replica whose box has an
empty region.

Every step runs through the library (run_switching for the dynamics, the
C-ABI estimators for the arithmetic); this module only sequences the runs.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

from . import fl as FL


def slab(replica, vacuum: float):
    """The same crystal as ``replica`` with ``vacuum`` A of empty space along z."""
    if not vacuum > 0.0:
        raise ValueError("slab: the vacuum must be positive")
    return dataclasses.replace(replica, vacuum=float(vacuum))


def surface_area(replica) -> float:
    """Total free-surface area of a slab replica, 2 Lx Ly (A^2)."""
    L = np.asarray(replica.box, dtype=np.float64)
    return 2.0 * float(L[0] * L[1])


@dataclass
class SurfaceFreeEnergy:
    gamma: float          # eV/A^2
    gamma_err: float      # standard error from the realizations of both systems
    F_bulk: float         # eV, whole system of N atoms
    F_bulk_err: float
    F_slab: float         # eV, whole system of N atoms
    F_slab_err: float
    area: float           # A^2, both faces
    E_diss_bulk: float    # eV (Eq. Ediss)
    E_diss_slab: float


def _system_key(r):
    return (r.kind, r.dims, r.a, r.T, r.k, r.mass)


def surface_free_energy(ctx, replicas, x0, n_bulk, t_s, n_eq, n_hold, dt=0.001, damp=0.1, skin=0.3,
                        function=2) -> SurfaceFreeEnergy:
    """gamma from one batched FL run.

    ``ctx`` is set up with ``replicas``: first ``n_bulk`` realizations of the
    bulk crystal (no vacuum), then realizations of its slab (the same crystal,
    T, k and mass, one positive vacuum), and ``x0`` holds their lattice sites
    (device SoA).  Each system's F0 is the FL estimate over its realizations;
    gamma_err combines the two standard errors."""
    bulk, slabs = list(replicas[:n_bulk]), list(replicas[n_bulk:])
    if not bulk or not slabs:
        raise ValueError("surface_free_energy: need realizations of both the bulk and the slab")
    b0, s0 = bulk[0], slabs[0]
    if any(_system_key(r) != _system_key(b0) or r.vacuum != 0.0 for r in bulk):
        raise ValueError("surface_free_energy: the bulk replicas must be realizations of one periodic crystal")
    if any(_system_key(r) != _system_key(b0) or r.vacuum != s0.vacuum for r in slabs) or not s0.vacuum > 0.0:
        raise ValueError("surface_free_energy: the slab replicas must be the bulk crystal with one positive vacuum")

    p, Wf, Wb = FL.run(ctx, x0, t_s, n_eq, n_hold, dt=dt, damp=damp, skin=skin, function=function)
    Fb, Edb, eb = FL.system_free_energy(p, Wf[:n_bulk], Wb[:n_bulk], b0)
    Fs, Eds, es = FL.system_free_energy(p, Wf[n_bulk:], Wb[n_bulk:], s0)
    A = surface_area(s0)
    return SurfaceFreeEnergy((Fs - Fb) / A, float(np.hypot(es, eb)) / A, Fb, eb, Fs, es, A, Edb, Eds)
