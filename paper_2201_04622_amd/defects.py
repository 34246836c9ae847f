"""Vacancy formation free energy by Frenkel--Ladd switching.

The point-defect side of the summary section's defect extension: the
free energy of the crystal with one site empty, F_vac(N - 1), against the
perfect crystal's, F(N), both in the perfect crystal's box, gives the
formation free energy at fixed volume
    G_f = F_vac(N - 1) - (N - 1) / N F(N),
each F from the FL path of the bulk section (Eq. W12 in Eq. fl, with Eq.
cm).  A vacancy is a replica whose ``inputs.Replica.vacancies`` names the
empty site; the kernels are unchanged.

Every step runs through the library (run_switching for the dynamics, the
C-ABI estimators for the arithmetic); this module only sequences the runs.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

from . import fl as FL


def with_vacancy(replica, site=0):
    """The same crystal with lattice site ``site`` left empty."""
    return dataclasses.replace(replica, vacancies=(int(site),))


@dataclass
class VacancyFormation:
    G_f: float            # eV
    G_f_err: float        # standard error from the realizations of both systems
    F_perfect: float      # eV, N atoms
    F_perfect_err: float
    F_vacancy: float      # eV, N - 1 atoms
    F_vacancy_err: float
    E_diss_perfect: float
    E_diss_vacancy: float


def _key(r):
    return (r.kind, r.dims, r.a, r.T, r.k, r.mass, r.vacuum)


def vacancy_formation_free_energy(ctx, replicas, x0, n_perfect, t_s, n_eq, n_hold, dt=0.001, damp=0.1, skin=0.3,
                                  function=2) -> VacancyFormation:
    """G_f from one batched FL run.  ``ctx`` is set up with ``replicas``:
    first ``n_perfect`` realizations of the perfect crystal, then
    realizations of the same crystal with one vacancy (the same site in
    each), and ``x0`` holds their lattice sites (device SoA)."""
    perfect, vac = list(replicas[:n_perfect]), list(replicas[n_perfect:])
    if not perfect or not vac:
        raise ValueError("vacancy_formation_free_energy: need realizations of both crystals")
    p0, v0 = perfect[0], vac[0]
    if any(_key(r) != _key(p0) or r.vacancies for r in perfect):
        raise ValueError("vacancy_formation_free_energy: the perfect replicas must be realizations of one crystal")
    if any(_key(r) != _key(p0) or r.vacancies != v0.vacancies for r in vac) or len(set(v0.vacancies)) != 1:
        raise ValueError("vacancy_formation_free_energy: the defect replicas must be the crystal with one vacancy")

    p, Wf, Wb = FL.run(ctx, x0, t_s, n_eq, n_hold, dt=dt, damp=damp, skin=skin, function=function)
    V = float(np.prod(p0.box))   # both systems in the perfect crystal's box
    Fp, Edp, ep = FL.system_free_energy(p, Wf[:n_perfect], Wb[:n_perfect], p0, V)
    Fv, Edv, ev = FL.system_free_energy(p, Wf[n_perfect:], Wb[n_perfect:], v0, V)
    N = p0.natoms
    G = Fv - (N - 1) / N * Fp
    return VacancyFormation(G, float(np.hypot(ev, (N - 1) / N * ep)), Fp, ep, Fv, ev, Edp, Edv)
