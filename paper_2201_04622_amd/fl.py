"""One batched Frenkel--Ladd run and the free energy of each system in it.

The pieces the defect and workload tools share: run the FL protocol (Sec.
p_fl) on every replica of a context from their lattice sites, split the work
traces into forward and backward legs, and estimate F0 (Eq. W12 in Eq. fl,
with Eq. cm when the centre of mass is fixed) for a group of realizations of
one system.  Every step runs through the library; this module only sequences
the calls.
"""
from __future__ import annotations

import numpy as np

from . import eamfe as E


def run(ctx, x0, t_s, n_eq, n_hold, dt=0.001, damp=0.1, skin=0.3, function=2):
    """The FL protocol [n_eq at lambda = 0][t_s forward][n_hold][t_s backward]
    on every replica of ``ctx`` from positions ``x0`` (device SoA, not
    modified); returns (protocol, W_fwd[n_rep], W_bwd[n_rep])."""
    import torch

    p = E.protocol("fl", n_eq, int(t_s), n_hold, 0, function=function, dt=dt, damp=damp, skin=skin)
    S = n_eq + 2 * int(t_s) + n_hold
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, bool(p.fix_com))
    ctx.neigh_build(x, skin, 0)
    W = torch.zeros(ctx.n_rep, S, dtype=torch.float64, device=x.device)
    ctx.run_switching(p, x, v, 0, S, W_out=W)
    Wf, Wb = E.switch_works(p, W.cpu().numpy())
    return p, Wf, Wb


def system_free_energy(p, W_fwd, W_bwd, rep, V=None):
    """(F0, E_diss, standard error) in eV for realizations of the system of
    replica ``rep`` (inputs.Replica) with works W_fwd, W_bwd; ``V`` is the
    volume in Eq. cm (default: the replica's box)."""
    N = rep.natoms
    n_eff = N   # Eq. fl: all N oscillators; the held centre of mass enters through Eq. cm
    V = float(np.prod(rep.box)) if V is None else float(V)
    return E.fl_free_energy(np.asarray(W_fwd), np.asarray(W_bwd), n_eff, rep.T, rep.k, rep.mass,
                            N if p.fix_com else None, V if p.fix_com else None)
