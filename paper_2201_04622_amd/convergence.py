"""Convergence of Frenkel--Ladd switching with the switching time.

For a set of switching times t_s, runs the FL protocol (equilibration at
lambda = 0, forward switch to the Einstein crystal, hold, backward switch;
Sec. p_fl) on a batch of independent realizations of one system, and reports
per t_s the estimators the paper compares in its convergence study (Fig.
fl_convergence, Sec. p_fl):

* F0 from the two directions combined (Eq. W12 inserted in Eq. fl, with the
  fixed centre-of-mass term Eq. cm) and its standard error over realizations;
* the dissipation (Eq. Ediss), which vanishes as t_s grows;
* the one-way estimates of F0 from Jarzynski's equality (Eq. jarz) applied to
  the forward leg alone (F0 = F_E - dF_{0->E}) and to the backward leg alone
  (F0 = F_E + dF_{E->0}), with their errors;
* the plain one-way means F_E - mean W_fwd and F_E + mean W_bwd, whose bias is
  the dissipation of each leg.

Every step runs through the library (run_switching for the dynamics, the C-ABI
estimators for the arithmetic); this module only sequences the runs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import eamfe as E


@dataclass
class SweepPoint:
    t_s: int                 # switching steps of each leg
    F0_w12: float            # eV, whole system (Eq. fl, both directions)
    F0_w12_err: float
    E_diss: float            # eV (Eq. Ediss)
    F0_jarz_fwd: float       # eV, Jarzynski on the forward leg
    F0_jarz_fwd_err: float
    F0_jarz_bwd: float       # eV, Jarzynski on the backward leg
    F0_jarz_bwd_err: float
    F0_mean_fwd: float       # eV, F_E - mean W_fwd
    F0_mean_bwd: float       # eV, F_E + mean W_bwd
    W_fwd: np.ndarray        # per realization
    W_bwd: np.ndarray


def fl_sweep(ctx, replicas, x0, t_s_list, n_eq, n_hold, dt=0.001, damp=0.1, skin=0.3, function=2):
    """Run the FL protocol once per t_s on every replica of ``ctx`` (already
    set up with ``replicas``, realizations of one system: same lattice, size,
    box, T, k and mass, different seeds) from the lattice sites ``x0``
    (device SoA), and return one SweepPoint per t_s."""
    import torch

    r0 = replicas[0]
    for r in replicas[1:]:
        if (r.kind, r.dims, r.a, r.T, r.k, r.mass) != (r0.kind, r0.dims, r0.a, r0.T, r0.k, r0.mass):
            raise ValueError("fl_sweep: the replicas must be realizations of one system")
    N = int(x0.shape[1]) // len(replicas)
    L = np.asarray(r0.box, dtype=np.float64)
    V = float(np.prod(L))
    mass = float(getattr(r0, "mass", 55.845))
    out = []
    for t_s in t_s_list:
        p = E.protocol("fl", n_eq, int(t_s), n_hold, 0, function=function, dt=dt, damp=damp, skin=skin)
        S = n_eq + 2 * int(t_s) + n_hold
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, bool(p.fix_com))
        ctx.neigh_build(x, skin, 0)
        W = torch.zeros(len(replicas), S, dtype=torch.float64, device=x.device)
        ctx.run_switching(p, x, v, 0, S, W_out=W)
        Wf, Wb = E.switch_works(p, W.cpu().numpy())
        n_eff = N   # Eq. fl: all N oscillators; the held centre of mass enters through Eq. cm
        FE = E.einstein_free_energy(n_eff, r0.T, r0.k, mass)
        cm = E.fixed_cm_correction(N, V, r0.T, r0.k) if p.fix_com else 0.0
        F0, Ed, err = E.fl_free_energy(Wf, Wb, n_eff, r0.T, r0.k, mass, N if p.fix_com else None,
                                       V if p.fix_com else None)
        jf, jfe = E.jarzynski(Wf, r0.T)      # F_E - F0
        jb, jbe = E.jarzynski(Wb, r0.T)      # F0 - F_E
        out.append(SweepPoint(int(t_s), F0, err, Ed, FE + cm - jf, jfe, FE + cm + jb, jbe,
                              FE + cm - float(Wf.mean()), FE + cm + float(Wb.mean()), Wf, Wb))
    return out
