"""Constant-pressure dynamics with the FP64 oracle: fixed-volume stretches of
the oracle's step loop alternating with isotropic stochastic cell-rescaling
moves (Bernetti and Bussi, J. Chem. Phys. 153, 114107, 2020).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; never by the product
package.  One move, for a replica at temperature T in a box L with internal
pressure P of the Hamiltonian w U_EAM,
  P = (sum_i m v_i^2 + w W) / (3 V),  W the trace of the pair virial,
changes eps = ln V by
  d eps = -(beta_T / tau_p) (p0 - P - kB T / V) dt + sqrt(2 kB T beta_T dt / (V tau_p)) z,
with z the first Box--Muller deviate of Philox stream 3 at counter (atom 0,
step) under the replica's seed; positions and box edges are scaled by
exp(d eps / 3) and velocities by its inverse.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

KB = 8.617333262e-5        # eV/K
MVV2E = 1.0364269e-4       # eV per amu A^2/ps^2


def move(pot, x, v, L, T, mass, seed, step, w_eam, p0, tau_p, beta_T, dt):
    """One rescaling move in place on x, v (AoS [N, 3]); returns (L_new, mu, P)."""
    L = np.asarray(L, dtype=np.float64)
    V = float(np.prod(L))
    Pc = pot.pressure(x, L)                      # virial part only, per axis
    W = float(np.sum(Pc)) * V
    K = mass * MVV2E * float(np.sum(v * v))
    P = (K + w_eam * W) / (3.0 * V)
    kT = KB * T
    z = O.gauss3(seed, 0, step, 3)[0]
    deps = -(beta_T / tau_p) * (p0 - P - kT / V) * dt + np.sqrt(2.0 * kT * beta_T * dt / (V * tau_p)) * z
    mu = float(np.exp(deps / 3.0))
    x *= mu
    v /= mu
    return L * mu, mu, P


def run_npt(pot, params, x0, L, x, v, lam, every, p0, tau_p, beta_T):
    """Steps 0 .. len(lam) - 2 of the schedule ``lam`` (reversible-scaling
    mode: the Hamiltonian lam[s] U_EAM) with a move at every multiple of
    ``every`` before the end.  x, v advance in place; returns the box edges
    after each move, the factors, the pressures and the work trace."""
    S = len(lam) - 1
    boxes, mus, Ps = [np.array(L, dtype=np.float64)], [], []
    W = np.zeros(S)
    L = np.array(L, dtype=np.float64)
    w0 = 0.0
    for s in range(0, S, every):
        e = min(S, s + every)
        _, Wc, _, _ = O.run(pot, params, x0, L, x, v, lam[s:e + 1], step0=s, W0=w0)
        W[s:e] = Wc
        w0 = float(Wc[-1])
        if e < S:
            L, mu, P = move(pot, x, v, L, params.T, params.mass, params.seed, e, lam[e], p0, tau_p, beta_T,
                            params.dt * every)
            boxes.append(L.copy())
            mus.append(mu)
            Ps.append(P)
    return np.asarray(boxes), np.asarray(mus), np.asarray(Ps), W
