"""Free-energy estimators of the oracle (plain numpy, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle.py``).  Each function states the
passage of arXiv 2201.04622 it follows.
"""
from __future__ import annotations

import numpy as np

KB = 8.617333262e-5      # eV/K
HBAR = 6.582119569e-4    # eV ps
MVV2E = 1.0364269e-4     # eV per amu A^2/ps^2


def einstein_free_energy(n_eff, T, k, mass):
    """F_E = 3 N kB T ln(hbar w / kB T), w = sqrt(k/m)  (Eq. einstein and the
    closed form below it), ``n_eff`` oscillators.  In Eq. fl the Einstein
    crystal has all N atoms: the fixed centre of mass enters through Eq. cm
    alone, so n_eff = N there."""
    omega = np.sqrt(k / (mass * MVV2E))          # 1/ps
    return 3.0 * n_eff * KB * T * np.log(HBAR * omega / (KB * T))


def fixed_cm_correction(N, V, T, k):
    """delta F_CM = kB T ln[(N/V) (2 pi kB T / (N m w^2))^(3/2)], m w^2 = k  (Eq. cm)."""
    return KB * T * np.log((N / V) * (2.0 * np.pi * KB * T / (N * k)) ** 1.5)


def msd_com_removed(x, x0):
    """<(dr)^2> over the atoms of one replica, dr = x - x0 minus the mean
    displacement (the centre of mass removed), as in the spring-constant
    choice of Eq. msd.  x, x0: [n, 3]."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(x0, dtype=np.float64)
    d = d - d.mean(axis=0)
    return float((d * d).sum(axis=1).mean())


def spring_constant(msd, T):
    """k = 3 kB T / <(dr)^2>  (Eq. msd)."""
    return 3.0 * KB * T / msd


def forward_backward(W_fwd, W_bwd):
    """Eq. W12 and Eq. Ediss: dF = (W12 - W21)/2 and E_diss = (W12 + W21)/2 over
    the replica means; returns (dF, E_diss, standard error of dF)."""
    W_fwd = np.asarray(W_fwd, dtype=np.float64)
    W_bwd = np.asarray(W_bwd, dtype=np.float64)
    d = 0.5 * (W_fwd - W_bwd)
    n = d.size
    err = d.std(ddof=1) / np.sqrt(n) if n > 1 else float("nan")
    return float(d.mean()), float(0.5 * (W_fwd.mean() + W_bwd.mean())), float(err)


def jarzynski(W, T):
    """exp(-beta dF) = mean exp(-beta W)  (Eq. jarz)."""
    b = 1.0 / (KB * T)
    W = np.asarray(W, dtype=np.float64)
    m = (-b * W).max()
    return float(-(m + np.log(np.mean(np.exp(-b * W - m)))) / b)


def frenkel_ladd(W_fwd, W_bwd, n_eff, T, k, mass, N=None, V=None):
    """F0 = F_E + (W_{E->0} - W_{0->E})/2 [+ delta F_CM]  (Eq. fl with the forward
    run taking H0 to H_E; the sign follows from Eq. W12 with 1 = H0, 2 = H_E).
    The fixed-CM term (Eq. cm) is added when N and V are given; F_E then has
    all n_eff = N oscillators, as Eq. fl writes it: the switching work is
    that of the two systems with the centre of mass held, and Eq. cm takes
    the Einstein crystal's value to the free crystal's."""
    dF, ediss, err = forward_backward(W_fwd, W_bwd)   # dF = F_E - F0
    F0 = einstein_free_energy(n_eff, T, k, mass) - dF
    if N is not None and V is not None:
        F0 += fixed_cm_correction(N, V, T, k)
    return float(F0), ediss, err


def rs_work_curves(W_trace, n_eq, n_sw, n_hold):
    """Split one RS work trace (cumulative, per step) into the forward work
    W_{1->lambda} after q forward steps and the backward work W_{lambda->1}
    from backward step q to the end, q = 0..n_sw."""
    W_trace = np.asarray(W_trace, dtype=np.float64)
    base = W_trace[n_eq - 1] if n_eq > 0 else 0.0
    fwd = np.concatenate([[0.0], W_trace[n_eq: n_eq + n_sw] - base])
    b0 = n_eq + n_sw + n_hold
    wb_start = W_trace[b0 - 1]
    bwd_cum = np.concatenate([[0.0], W_trace[b0: b0 + n_sw] - wb_start])   # after q backward steps
    return fwd, bwd_cum


def reversible_scaling(F0_T0, T0, lambda_f, n_eff, W_fwd_curve, W_bwd_cum, T_grid):
    """F0(T) = F0(T0)/l + (3/2) N kB T0 ln(l)/l + (W_{1->l} - W_{l->1})/(2 l),
    l = T0/T  (Eq. rs).  The forward run passes l at tau = (T-T0)/(T_f-T0),
    i.e. after tau*n_sw steps; the backward run passes it after (1-tau)*n_sw
    steps, so W_{l->1} is the backward work from there to the end.  Work
    values between steps are linearly interpolated."""
    n_sw = len(W_fwd_curve) - 1
    Tf = T0 / lambda_f
    T_grid = np.asarray(T_grid, dtype=np.float64)
    lam = T0 / T_grid
    tau = (T_grid - T0) / (Tf - T0)
    q = np.arange(n_sw + 1, dtype=np.float64)
    w1 = np.interp(tau * n_sw, q, W_fwd_curve)
    wb_total = W_bwd_cum[-1]
    w2 = wb_total - np.interp((1.0 - tau) * n_sw, q, W_bwd_cum)
    return F0_T0 / lam + 1.5 * n_eff * KB * T0 * np.log(lam) / lam + (w1 - w2) / (2.0 * lam)


def thermal_wavelength(T, mass):
    """de Broglie wavelength Lambda = sqrt(2 pi hbar^2 / (m kB T)) in A, the
    momentum integral per degree of freedom of the partition function (the
    Lambda of the partition-function expression in the reversible-scaling
    section)."""
    return np.sqrt(2.0 * np.pi * HBAR ** 2 / (mass * MVV2E * KB * T))


def free_minus_fixed_cm(N, V, T, mass):
    """c(T) = F(free crystal) - F(crystal with its centre of mass held):
    -kB T ln(V/N) + 3 kB T ln Lambda(T).  The held system has 3(N-1) momenta
    and a configurational integral constrained at one centre-of-mass
    position; the free crystal integrates that position over the V/N volume
    per lattice translation and has all 3N momenta.  This is the convention
    under which Eq. einstein with N oscillators plus Eq. cm is the free
    crystal's free energy (the Gaussian integrals of the held Einstein crystal
    give F_E(N) + Eq. cm = F_E(held) + c)."""
    kT = KB * T
    return -kT * np.log(V / N) + 3.0 * kT * np.log(thermal_wavelength(T, mass))


def reversible_scaling_fixed_cm(F0_T0, T0, lambda_f, N, V, mass, W_fwd_curve, W_bwd_cum, T_grid):
    """Eq. rs for a run with the centre of mass held (every run here): the run
    samples the held system, whose free energy Eq. rs maps from T0 to T
    exactly with its 3(N-1) momenta in the kinetic term; the free crystal's
    F0(T0) (Eq. fl + Eq. cm) is taken to the held system and back with c:
      F(T) = rs_{N-1}(F0(T0) - c(T0)) + c(T)."""
    T_grid = np.asarray(T_grid, dtype=np.float64)
    held = reversible_scaling(F0_T0 - free_minus_fixed_cm(N, V, T0, mass), T0, lambda_f, N - 1,
                              W_fwd_curve, W_bwd_cum, T_grid)
    return held + free_minus_fixed_cm(N, V, T_grid, mass)
