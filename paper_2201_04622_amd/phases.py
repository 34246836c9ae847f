"""Free energies of the crystal structures of a potential, automated.

The summary section's use of the method for potential development and
benchmarking: for each structure (bcc, fcc, hcp), find its zero-pressure
lattice parameter at T (batched fixed-volume runs, lattice.py), choose the
Einstein spring constant from its mean-squared displacement (Eq. msd,
springs.py), and run FL on a batch of realizations (Eq. W12 in Eq. fl with
Eq. cm).  The free energies per atom at zero pressure then rank the phases,
as the paper's bcc/fcc/hcp comparisons do.  hcp relaxes both cell lengths
(lattice.zero_stress_hcp).

Every step runs through the library; this module only sequences the runs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import eamfe as E
from . import fl as FL
from . import inputs as I
from . import lattice as LT
from . import springs as SP

CELLS = {"bcc": (6, 6, 6), "fcc": (5, 5, 5), "hcp": (7, 4, 5)}   # every edge above 2 (r_cut + skin)
A_GUESS = {"bcc": I.A_BCC_STABLE, "fcc": I.A_FCC_STABLE, "hcp": I.A_FCC_STABLE / np.sqrt(2.0)}


@dataclass
class Phase:
    kind: str
    a: float              # zero-pressure lattice parameter at T (A)
    k: float              # spring constant from the MSD (eV/A^2)
    F_per_atom: float     # eV
    F_err: float
    E_diss_per_atom: float
    c_over_a: float = None   # hcp: relaxed c/a at T


def phase_free_energy(kind, T, cells=None, realizations=4, t_s=8000, n_eq=1000, n_hold=1000, precision=E.FP32,
                      skin=0.3, seed=0) -> Phase:
    """F per atom of ``kind`` at T and zero pressure."""
    import torch

    cells = CELLS[kind] if cells is None else cells
    if kind == "hcp":   # both cell lengths free
        zs = LT.zero_stress_hcp(cells, T, A_GUESS[kind], rel_span=0.004, n_steps=4000, discard=1000, seed=seed,
                                precision=precision, skin=skin, iterations=5)
        a0, q0 = zs.a, zs.c_over_a
    else:
        a0 = LT.zero_pressure_lattice(kind, cells, T, A_GUESS[kind], rel_span=0.004, n_trials=8, n_steps=4000,
                                      discard=1000, iterations=2, seed=seed, precision=precision, skin=skin).a0
        q0 = None
    reps = [I.Replica(kind, 0, a0, T, 1.0, seed + 10 + s, cells=cells, c_over_a=q0) for s in range(realizations)]

    def context(rs):
        ctx = E.Context(0, precision)
        ctx.eam_setup(I.synthetic_eam_knots())
        x = E.to_soa(I.batch_arrays(rs)["x0"])
        ctx.system_setup(rs, x)
        return ctx, x

    ctx, x = context(reps)
    try:
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, skin, 0)
        k, _, _ = SP.spring_constants(ctx, reps, x, v, 4000, 100, skin=skin, discard=1000)
    finally:
        ctx.close()
    import dataclasses
    reps = [dataclasses.replace(r, k=float(np.mean(k))) for r in reps]
    ctx, x0 = context(reps)
    try:
        p, Wf, Wb = FL.run(ctx, x0, t_s, n_eq, n_hold, skin=skin)
    finally:
        ctx.close()
    F0, Ed, err = FL.system_free_energy(p, Wf, Wb, reps[0])
    N = reps[0].natoms
    return Phase(kind, a0, reps[0].k, F0 / N, err / N, Ed / N, q0)


def rank_phases(T, kinds=("bcc", "fcc", "hcp"), **kw):
    """{kind: Phase} at T, and the kinds ordered from the lowest free energy."""
    out = {kd: phase_free_energy(kd, T, **kw) for kd in kinds}
    return out, sorted(kinds, key=lambda kd: out[kd].F_per_atom)
