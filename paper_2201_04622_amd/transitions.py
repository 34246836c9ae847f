"""Gibbs energy curves at zero pressure and the temperature where two
structures exchange stability.

The route of the paper's phase-stability results (Figs. bcc_fcc and
fcc_hcp): for each structure, FL at T0 in the box of its zero-pressure
lattice parameter gives G(T0) (at p = 0, G = F up to terms of order kB T per
system); reversible scaling under the barostat from T0 to T_f then gives
G(T) on a 1 K grid (Eq. rs in its fixed-centre-of-mass form, with G for F).
Where G_a(T) - G_b(T) changes sign the stable structure changes.  hcp starts
from its cell relaxed at T0 (a and c/a); the isotropic barostat keeps its c/a.

Every step runs through the library; this module only sequences the runs.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

from . import barostat as B
from . import eamfe as E
from . import fl as FL
from . import inputs as I
from . import lattice as LT
from . import springs as SP
from .phases import A_GUESS, CELLS


@dataclass
class GibbsCurve:
    kind: str
    a0: float                 # zero-pressure lattice parameter at T0 (A)
    k: float                  # FL spring constant (eV/A^2)
    T: np.ndarray             # K
    G: np.ndarray             # eV/atom, mean over realizations
    G_err: np.ndarray         # standard error (RS spread and the FL start, scaled by T/T0)
    G0: float                 # FL value at T0, eV/atom
    G0_err: float


def _context(reps, precision):
    ctx = E.Context(0, precision)
    ctx.eam_setup(I.synthetic_eam_knots())
    x = E.to_soa(I.batch_arrays(reps)["x0"])
    ctx.system_setup(reps, x)
    return ctx, x


def gibbs_curve(kind, T0, Tf, cells=None, realizations=4, fl_steps=(1000, 16000, 1000),
                rs_steps=(2000, 20000, 2000), every=10, tau_p=0.2, beta_T=0.3, precision=E.FP32, skin=0.3,
                seed=0) -> GibbsCurve:
    import torch

    cells = CELLS[kind] if cells is None else cells
    if kind == "hcp":   # the cell relaxed at T0; the isotropic barostat then keeps its c/a
        zs = LT.zero_stress_hcp(cells, T0, A_GUESS[kind], rel_span=0.004, n_steps=4000, discard=1000, seed=seed,
                                precision=precision, skin=skin, iterations=5)
        a0, q0 = zs.a, zs.c_over_a
    else:
        a0 = LT.zero_pressure_lattice(kind, cells, T0, A_GUESS[kind], rel_span=0.004, n_trials=8, n_steps=4000,
                                      discard=1000, iterations=2, seed=seed, precision=precision, skin=skin).a0
        q0 = None
    reps = [I.Replica(kind, 0, a0, T0, 1.0, seed + 10 + s, cells=cells, c_over_a=q0) for s in range(realizations)]
    ctx, x = _context(reps, precision)
    try:
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, skin, 0)
        k, _, _ = SP.spring_constants(ctx, reps, x, v, 4000, 100, skin=skin, discard=1000)
    finally:
        ctx.close()
    k = float(np.mean(k))
    reps = [dataclasses.replace(r, k=k) for r in reps]
    ctx, x0 = _context(reps, precision)
    try:
        p, Wf, Wb = FL.run(ctx, x0, fl_steps[1], fl_steps[0], fl_steps[2], skin=skin)
    finally:
        ctx.close()
    N = reps[0].natoms
    per = np.array([FL.system_free_energy(p, Wf[q:q + 1], Wb[q:q + 1], reps[0])[0] for q in range(len(reps))])
    G0, G0_err = per.mean(), per.std(ddof=1) / np.sqrt(len(per))

    rs_reps = [I.Replica(kind, 0, a0, T0, 0.0, seed + 50 + s, cells=cells, c_over_a=q0) for s in range(realizations)]
    ctx, x = _context(rs_reps, precision)
    try:
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, skin, 0)
        n_eq, n_sw, n_hold = rs_steps
        pr = E.protocol("rs", n_eq, n_sw, n_hold, 0, lambda_f=T0 / Tf, skin=skin)
        S = n_eq + 2 * n_sw + n_hold
        W = torch.zeros(len(rs_reps), S, dtype=torch.float64, device="cuda")
        B.run_npt(ctx, pr, x, v, 0, S, every, B.barostat(0.0, tau_p, beta_T, pr.dt, every), W_out=W)
    finally:
        ctx.close()
    W = W.cpu().numpy()
    grid = np.arange(T0, Tf + 0.5, 1.0)
    V0 = float(np.prod(rs_reps[0].box))
    G = np.array([E.rs_free_energy_cm(pr, W[q], G0, T0, N, V0, rs_reps[0].mass, grid) for q in range(len(rs_reps))]) / N
    err = np.hypot(G.std(axis=0, ddof=1) / np.sqrt(len(G)), G0_err / N * grid / T0)
    return GibbsCurve(kind, a0, k, grid, G.mean(axis=0), err, G0 / N, G0_err / N)


def transition_temperature(a: GibbsCurve, b: GibbsCurve):
    """The temperature where G_a - G_b changes sign on the common grid
    (linear between grid points), or None if it keeps one sign."""
    if not np.array_equal(a.T, b.T):
        raise ValueError("transition_temperature: the curves need the same temperature grid")
    d = a.G - b.G
    s = np.nonzero(np.signbit(d[:-1]) != np.signbit(d[1:]))[0]
    if len(s) == 0:
        return None
    i = int(s[0])
    return float(a.T[i] + (a.T[i + 1] - a.T[i]) * d[i] / (d[i] - d[i + 1]))
