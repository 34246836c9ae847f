"""Constant-pressure dynamics with the FP64 oracle: fixed-volume stretches of
the oracle's step loop alternating with isotropic stochastic cell-rescaling
moves (Bernetti and Bussi, J. Chem. Phys. 153, 114107, 2020).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; never by the product
package.  The orthorhombic form (each box edge on its own, ``aniso``) is
described at ``move``.  One isotropic move, for a replica at temperature T in a box L with internal
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


def move(pot, x, v, L, T, mass, seed, step, w_eam, p0, tau_p, beta_T, dt, aniso=False):
    """One rescaling move in place on x, v (AoS [N, 3]); returns (L_new, mu, P).

    Isotropic: mu and P are scalars (P the internal pressure above).
    Orthorhombic (aniso): each edge moves on its own, eps_a = ln L_a, with the
    diagonal pressure P_aa = (sum_i m v_ia^2 + w W_aa) / V of that axis,
      d eps_a = -(beta_T / (3 tau_p)) (p0 - P_aa - kB T / V) dt
                + sqrt(2 kB T beta_T dt / (3 V tau_p)) z_a,
    z_a the three deviates of the same Philox block; positions and edges along
    a scale by exp(d eps_a), velocities by its inverse.  Summed over the axes
    this is the isotropic move of ln V (the drifts add, and so do the
    variances), and it samples exp(-(U + p0 V) / kB T) V^N over the three
    edges (V^N from the scaled coordinates, the measure dL_x dL_y dL_z =
    V d eps_x d eps_y d eps_z giving the kB T / V term per axis); mu and P
    are then 3-vectors."""
    L = np.asarray(L, dtype=np.float64)
    V = float(np.prod(L))
    Pc = pot.pressure(x, L)                      # virial part only, per axis
    kT = KB * T
    z = O.gauss3(seed, 0, step, 3)
    if not aniso:
        W = float(np.sum(Pc)) * V
        K = mass * MVV2E * float(np.sum(v * v))
        P = (K + w_eam * W) / (3.0 * V)
        deps = -(beta_T / tau_p) * (p0 - P - kT / V) * dt + np.sqrt(2.0 * kT * beta_T * dt / (V * tau_p)) * z[0]
        mu = float(np.exp(deps / 3.0))
        x *= mu
        v /= mu
        return L * mu, mu, P
    Paa = (mass * MVV2E * np.sum(v * v, axis=0) + w_eam * Pc * V) / V
    deps = -(beta_T / (3.0 * tau_p)) * (p0 - Paa - kT / V) * dt + np.sqrt(2.0 * kT * beta_T * dt / (3.0 * V * tau_p)) * z
    mu = np.exp(deps)
    x *= mu[None, :]
    v /= mu[None, :]
    return L * mu, mu, Paa


def run_npt(pot, params, x0, L, x, v, lam, every, p0, tau_p, beta_T, aniso=False):
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
                            params.dt * every, aniso)
            boxes.append(L.copy())
            mus.append(mu)
            Ps.append(P)
    return np.asarray(boxes), np.asarray(mus), np.asarray(Ps), W
