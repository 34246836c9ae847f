"""The free-energy assembly pinned on a crystal whose classical free energy is
known exactly: fcc with central nearest-neighbour springs, phi(r) =
(K/2)(r - r0)^2 on the nearest-neighbour shell and zero beyond (rho = F = 0,
so U_EAM is this pair sum).  It is translation invariant like an EAM solid,
harmonic to far better than the tolerances at the temperatures used, and its
3N - 3 nonzero normal modes give

  F(T) = -kB T ln[(V/N) N^(3/2) prod_m (2 pi kB T / l_m)^(1/2)] + 3 N kB T ln Lambda(T),

the free crystal in the convention of Eq. cm (the centre of mass ranges
over V/N; N^(3/2) is the Jacobian of the centre-of-mass constraint; l_m the
Hessian's nonzero eigenvalues).  The oracle's Frenkel--Ladd runs (centre of
mass held) assembled by Eq. fl with N oscillators plus Eq. cm must reach
F(T0), and its reversible-scaling runs assembled by Eq. rs for the held
system must reach F(T) over the scan.  The N - 1 convention misses by
3 kB T ln(hbar w / kB T) per system, many standard errors here."""
import numpy as np
import pytest

from oracle import estimators as OE
from paper_2201_04622_amd import inputs as I

K_BOND = 1.25        # eV/A^2, nearest-neighbour bond spring
R0 = 2.5             # A, nearest-neighbour distance (fcc a = R0 sqrt 2)
R_CUT, R_TAPER = 3.2, 2.9
N_KNOTS = 2000
MASS = 55.845
K_EIN = 4.0 * K_BOND   # the Einstein spring with the same mean square frequency
KB, HBAR, MVV2E = 8.617333262e-5, 6.582119569e-4, 1.0364269e-4


def _spring_potential(O):
    r = np.arange(N_KNOTS) * R_CUT / (N_KNOTS - 1)
    taper = np.where(r <= R_TAPER, 1.0, 0.5 * (1.0 + np.cos(np.pi * (r - R_TAPER) / (R_CUT - R_TAPER))))
    phi = 0.5 * K_BOND * (r - R0) ** 2 * taper
    zero = np.zeros(N_KNOTS)
    return O.Potential(phi, zero, zero, R_CUT, 1.0)


def _crystal(n=2):
    a = R0 * np.sqrt(2.0)
    x0 = I.lattice_sites("fcc", n, a)
    return x0, np.full(3, n * a)


def _hessian(x0, L):
    """Force-constant matrix of the bond springs at the lattice (phi'(r0) = 0,
    so each bond contributes K r^ r^T)."""
    N = len(x0)
    H = np.zeros((3 * N, 3 * N))
    for i in range(N):
        for j in range(i + 1, N):
            d = x0[i] - x0[j]
            d -= L * np.round(d / L)
            r = np.linalg.norm(d)
            if r < R_CUT:
                assert abs(r - R0) < 1e-9
                b = K_BOND * np.outer(d, d) / (r * r)
                H[3 * i:3 * i + 3, 3 * i:3 * i + 3] += b
                H[3 * j:3 * j + 3, 3 * j:3 * j + 3] += b
                H[3 * i:3 * i + 3, 3 * j:3 * j + 3] -= b
                H[3 * j:3 * j + 3, 3 * i:3 * i + 3] -= b
    return H


def _exact_free_energy(x0, L, T):
    N, V, kT = len(x0), float(np.prod(L)), KB * T
    ev = np.linalg.eigvalsh(_hessian(x0, L))
    assert np.all(np.abs(ev[:3]) < 1e-9) and ev[3] > 1e-3     # three translations, the rest stable
    lnZ = np.log(V / N) + 1.5 * np.log(N) + 0.5 * np.sum(np.log(2 * np.pi * kT / ev[3:]))
    lam_dB = np.sqrt(2 * np.pi * HBAR ** 2 / (MASS * MVV2E * kT))
    return -kT * lnZ + 3 * N * kT * np.log(lam_dB)


def test_held_einstein_crystal_identity():
    """Closed forms only: the Einstein crystal with its centre of mass held
    has Z = N^(3/2) (2 pi kT / k)^(3(N-1)/2) Lambda^(-3(N-1)); Eq. einstein with
    N oscillators plus Eq. cm equals that held value plus c(T)."""
    for N, V, T in ((32, 353.6, 10.0), (432, 7600.0, 300.0), (2000, 23270.0, 1400.0)):
        kT = KB * T
        held = -kT * (1.5 * np.log(N) + 1.5 * (N - 1) * np.log(2 * np.pi * kT / K_EIN)
                      - 3 * (N - 1) * np.log(OE.thermal_wavelength(T, MASS)))
        lhs = OE.einstein_free_energy(N, T, K_EIN, MASS) + OE.fixed_cm_correction(N, V, T, K_EIN)
        assert lhs == pytest.approx(held + OE.free_minus_fixed_cm(N, V, T, MASS), rel=0, abs=1e-10 * N)


def test_frenkel_ladd_reaches_the_exact_free_energy(oracle_lib):
    O = oracle_lib
    pot = _spring_potential(O)
    x0, L = _crystal()
    N, V, T = len(x0), float(np.prod(L)), 10.0
    n_eq, n_sw, n_hold = 2000, 10000, 1000
    lam = O.schedule("fl", n_eq, n_sw, n_hold, 0)
    b0 = n_eq + n_sw + n_hold
    Wf, Wb = [], []
    for seed in range(10):
        p = O.RunParams(mode="fl", T=T, k=K_EIN, seed=seed, fix_com=True)
        x, v = x0.copy(), O.init_velocities(p, N)
        _, W, _, _ = O.run(pot, p, x0, L, x, v, lam)
        Wf.append(W[n_eq + n_sw - 1] - W[n_eq - 1])
        Wb.append(W[b0 + n_sw - 1] - W[b0 - 1])
    exact = _exact_free_energy(x0, L, T)
    F0, ediss, err = OE.frenkel_ladd(Wf, Wb, N, T, K_EIN, MASS, N=N, V=V)
    print(f"FL: F0 {F0:.6f} exact {exact:.6f} eV, error {err:.2e}, dissipation {ediss:.2e}")
    assert abs(F0 - exact) < 4 * err + 2e-5, (F0, exact, err)
    wrong, _, _ = OE.frenkel_ladd(Wf, Wb, N - 1, T, K_EIN, MASS, N=N, V=V)
    assert abs(wrong - exact) > 10 * err     # the pin resolves the N - 1 convention


def test_reversible_scaling_reaches_the_exact_free_energy(oracle_lib):
    O = oracle_lib
    pot = _spring_potential(O)
    x0, L = _crystal()
    N, V = len(x0), float(np.prod(L))
    T0, Tf = 10.0, 40.0
    n_eq, n_sw, n_hold = 1000, 10000, 500
    lam = O.schedule("rs", n_eq, n_sw, n_hold, 0, lambda_f=T0 / Tf)
    grid = np.array([10.0, 15.0, 20.0, 30.0, 40.0])
    F0_T0 = _exact_free_energy(x0, L, T0)
    curves = []
    for seed in range(10):
        p = O.RunParams(mode="rs", T=T0, k=0.0, seed=seed, fix_com=True)
        x, v = x0.copy(), O.init_velocities(p, N)
        _, W, _, _ = O.run(pot, p, x0, L, x, v, lam)
        fwd, bwd = OE.rs_work_curves(W, n_eq, n_sw, n_hold)
        curves.append(OE.reversible_scaling_fixed_cm(F0_T0, T0, T0 / Tf, N, V, MASS, fwd, bwd, grid))
    curves = np.asarray(curves)
    F, err = curves.mean(0), curves.std(0, ddof=1) / np.sqrt(len(curves))
    exact = np.array([_exact_free_energy(x0, L, t) for t in grid])
    print("RS:", np.c_[grid, F, exact, err])
    assert np.all(np.abs(F - exact) < 4 * err + 2e-5), (F - exact, err)
    # Eq. cm in place of c (the form the free crystal's F0 would need if
    # Eq. cm were the held-to-free step) misses by 3 kB T ln(T/T0) per system
    wrong = F - OE.free_minus_fixed_cm(N, V, grid, MASS) + OE.fixed_cm_correction(N, V, grid, K_EIN) \
        - (OE.fixed_cm_correction(N, V, T0, K_EIN) - OE.free_minus_fixed_cm(N, V, T0, MASS)) * grid / T0
    assert np.abs(wrong - exact)[-1] > 5 * err[-1]
