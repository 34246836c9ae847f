"""Constant-pressure runs: fixed-volume stretches of the switching dynamics
alternating with stochastic cell-rescaling moves (Bernetti and Bussi, J.
Chem. Phys. 153, 114107, 2020; ``eamfe_barostat_step``), isotropic or with
each box edge on its own (orthorhombic, for hcp's c/a).

The paper holds the pressure at zero with a barostat in its reversible-
scaling runs (Sec. p_rs) and while it fixes the lattice parameter of its
Frenkel--Ladd runs (Sec. p_fl).  Here a move follows every ``every`` steps of
``run_switching`` in the reversible-scaling mode (with lambda_f = 1 that is
plain dynamics of U_EAM).  It reads the internal pressure of the Hamiltonian
at the step boundary, lambda U_EAM. With p0 = 0 the scaled system at T0 then
stays at the zero pressure of the real system at T0 / lambda, and the RS work
gives the Gibbs energy G(T) at zero pressure (Eq. rs with F replaced by G).

Every step runs through the library; this module only sequences the calls.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import eamfe as E


@dataclass
class NptTrace:
    steps: np.ndarray     # [moves] step boundary of each move
    boxes: np.ndarray     # [moves + 1, n_rep, 3] box edges before the first move and after each
    mu: np.ndarray        # [moves, n_rep, 3] per-axis scale factors
    pressure: np.ndarray  # [moves, n_rep, 3] diagonal internal pressures the moves used, eV/A^3


def barostat(p0=0.0, tau_p=1.0, beta_T=1.0, dt=0.001, every=10, aniso=False) -> E.Barostat:
    """Parameters of the move made every ``every`` steps of length ``dt`` ps
    (the coupling interval is every * dt); ``aniso`` moves each box edge on
    its own."""
    return E.Barostat(float(p0), float(tau_p), float(beta_T), float(dt) * int(every), int(bool(aniso)), 0)


def run_npt(ctx, p: E.Protocol, x, v, step_begin, step_end, every, b: E.Barostat, dHdl_out=None,
            W_out=None) -> NptTrace:
    """Advance steps [step_begin, step_end) of protocol ``p`` with a barostat
    move at every multiple of ``every`` past step_begin (and none at
    step_end).  Traces as in run_switching."""
    if every <= 0:
        raise ValueError("run_npt: every must be positive")
    if p.mode != E.MODES["rs"]:
        raise ValueError("run_npt: constant pressure is for reversible scaling (lambda_f = 1 for plain dynamics); "
                         "the spring anchors of the other paths do not follow the box")
    lam = E.lambda_schedule(p)
    steps, boxes, mus, Ps = [], [ctx.boxes()], [], []
    s = int(step_begin)
    while s < step_end:
        e = min(int(step_end), s + int(every))
        ctx.run_switching(p, x, v, s, e, None, dHdl_out, W_out)
        if e < step_end:
            mu, P = ctx.barostat_step(b, e, lam[e], x, v)
            steps.append(e)
            mus.append(mu)
            Ps.append(P)
            boxes.append(ctx.boxes())
        s = e
    n = len(steps)
    return NptTrace(np.asarray(steps, dtype=np.int64), np.asarray(boxes),
                    np.asarray(mus).reshape(n, -1, 3), np.asarray(Ps).reshape(n, -1, 3))
