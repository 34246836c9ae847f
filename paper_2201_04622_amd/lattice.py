"""Lattice parameter at zero pressure (the volume at which the paper runs its
Frenkel--Ladd switching, Sec. p_fl, found there with a barostat).

Here the root is found without barostat dynamics: a batch of replicas of one
crystal at trial lattice parameters runs fixed-volume Langevin MD of the EAM
Hamiltonian (the lambda = 0 end of the FL path) at temperature T, each
replica's mean hydrostatic pressure p = tr P / 3 is sampled with
eamfe_pressure, and the root of a straight-line fit of p(a) near the guess is
the lattice parameter.  The dynamics and the pressure sums run in the library;
this module only sequences the runs and fits the line.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import eamfe as E
from . import inputs as I

EV_PER_A3_IN_GPA = 160.21766208


@dataclass
class ZeroPressure:
    a0: float                  # lattice parameter at p = 0 (A)
    slope: float               # dp/da at the root (eV/A^4)
    a_trials: np.ndarray
    p_mean: np.ndarray         # mean hydrostatic pressure per trial (eV/A^3)
    p_err: np.ndarray          # standard error of each mean
    samples: int


def zero_pressure_lattice(kind, cells, T, a_guess, rel_span=0.01, n_trials=8, n_steps=4000, discard=1000,
                          every=20, k=5.0, seed=0, precision=E.FP32, skin=0.3, lanes=2, block=256, iterations=1):
    """Batched fixed-volume runs of ``n_trials`` replicas of the ``kind``
    crystal (``cells``: n or (nx, ny, nz)) at lattice parameters spread over
    a_guess (1 +- rel_span), sampling each replica's pressure every ``every``
    steps after ``discard``; returns the root of the fitted p(a).  With
    ``iterations`` > 1 each further batch is centred on the last root with a
    third of the span, so the curvature of p(a) no longer moves the root."""
    out = None
    for it in range(iterations):
        out = _batch_root(kind, cells, T, a_guess if out is None else out.a0, rel_span / 3 ** it, n_trials, n_steps,
                          discard, every, k, seed + 1000 * it, precision, skin, lanes, block)
    return out


def _batch_root(kind, cells, T, a_guess, rel_span, n_trials, n_steps, discard, every, k, seed, precision, skin,
                lanes, block):
    import torch

    a = a_guess * (1.0 + rel_span * np.linspace(-1.0, 1.0, n_trials))
    dims = I.cell_counts(cells)
    reps = [I.Replica(kind, dims[0], float(ak), float(T), float(k), seed + q, cells=dims) for q, ak in enumerate(a)]
    arrs = I.batch_arrays(reps)
    ctx = E.Context(0, precision)
    try:
        ctx.set_launch(lanes, block)
        ctx.eam_setup(I.synthetic_eam_knots())
        x = E.to_soa(arrs["x0"])
        ctx.system_setup(reps, x)
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, skin, 0)
        p = E.protocol("fl", n_steps, 1, 0, 0, skin=skin)   # lambda = 0 throughout: the EAM crystal
        obs = []
        for s in range(0, n_steps - n_steps % every, every):
            ctx.run_switching(p, x, v, s, s + every)
            if s + every > discard:
                obs.append(ctx.pressure(x, v).mean(axis=1))
    finally:
        ctx.close()
    obs = np.array(obs)                                   # [samples, n_trials]
    pm = obs.mean(axis=0)
    # successive samples are correlated: the error of each mean from ten
    # contiguous block means
    nb = min(10, len(obs))
    if nb > 1:
        blocks = np.array([b.mean(axis=0) for b in np.array_split(obs, nb)])
        pe = blocks.std(axis=0, ddof=1) / np.sqrt(nb)
    else:
        pe = np.full(n_trials, np.nan)
    slope, icpt = np.polyfit(a, pm, 1)
    return ZeroPressure(float(-icpt / slope), float(slope), a, pm, pe, len(obs))


@dataclass
class ZeroStressHcp:
    a: float                   # A
    c_over_a: float
    P: np.ndarray              # [trials, 3] mean diagonal pressure of each trial (eV/A^3)
    trials: np.ndarray         # [trials, 2] (a, c/a) of each trial


def zero_stress_hcp(cells, T, a_guess, q_guess=np.sqrt(8.0 / 3.0), rel_span=0.004, n_steps=4000, discard=1000,
                    every=20, k=5.0, seed=0, precision=E.FP32, skin=0.3, lanes=2, block=256, iterations=2):
    """hcp with both cell lengths free: a 3 x 3 batch of fixed-volume runs over
    (a, c/a) around the guess, a plane fitted to the in-plane pressure
    (P_xx + P_yy) / 2 and one to P_zz, and the point where both vanish.  Each
    further iteration centres a new batch on the last solution (a Newton
    step); the last one spans a third as much."""
    import torch

    a0, q0 = float(a_guess), float(q_guess)
    out = None
    for it in range(iterations):
        span = rel_span if it < iterations - 1 else rel_span / 3.0
        grid = [(a0 * (1.0 + span * da), q0 * (1.0 + span * dq)) for da in (-1, 0, 1) for dq in (-1, 0, 1)]
        dims = I.cell_counts(cells)
        reps = [I.Replica("hcp", dims[0], ak, float(T), float(k), seed + 1000 * it + j, cells=dims, c_over_a=qk)
                for j, (ak, qk) in enumerate(grid)]
        ctx = E.Context(0, precision)
        try:
            ctx.set_launch(lanes, block)
            ctx.eam_setup(I.synthetic_eam_knots())
            x = E.to_soa(I.batch_arrays(reps)["x0"])
            ctx.system_setup(reps, x)
            v = torch.zeros_like(x)
            ctx.init_velocities(v, True)
            ctx.neigh_build(x, skin, 0)
            p = E.protocol("fl", n_steps, 1, 0, 0, skin=skin)   # lambda = 0 throughout: the EAM crystal
            obs = []
            for s in range(0, n_steps - n_steps % every, every):
                ctx.run_switching(p, x, v, s, s + every)
                if s + every > discard:
                    obs.append(ctx.pressure(x, v))
        finally:
            ctx.close()
        P = np.mean(obs, axis=0)                                   # [9, 3]
        g = np.array(grid)
        A = np.c_[np.ones(len(g)), g[:, 0] - a0, g[:, 1] - q0]
        c_in, *_ = np.linalg.lstsq(A, 0.5 * (P[:, 0] + P[:, 1]), rcond=None)
        c_z, *_ = np.linalg.lstsq(A, P[:, 2], rcond=None)
        M = np.array([[c_in[1], c_in[2]], [c_z[1], c_z[2]]])
        da, dq = np.linalg.solve(M, -np.array([c_in[0], c_z[0]]))
        a0, q0 = a0 + da, q0 + dq
        out = ZeroStressHcp(float(a0), float(q0), P, g)
    return out
