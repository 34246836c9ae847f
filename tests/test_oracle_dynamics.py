"""Pins of the oracle's integrator, switching runs and estimators against
closed forms (arXiv 2201.04622 and textbook statistical mechanics):

* harmonic equipartition, exact for the BAOAB splitting at any time step,
  and its known kinetic bias 1 - (w dt / 2)^2;
* NVE (gamma = 0, velocity Verlet) energy conservation with second-order
  scaling in dt (the paper's time-step check, Sec. p_fl);
* harmonic -> harmonic switching, whose exact dF = (3 N_dof/2) kT ln(k2/k1)
  the forward/backward estimator (Eq. W12) must reach, with equal forward and
  backward dissipation (Eq. Ediss);
* the Frenkel--Ladd assembly (Eq. fl, sign read from Eq. W12) and the
  reversible-scaling assembly (Eq. rs) on Einstein crystals, where both
  reduce to the closed-form Einstein free energy;
* the fixed centre of mass (Sec. p_fl) and the Verlet candidate list."""
import numpy as np
import pytest
from scipy import integrate, stats

from oracle import estimators as E
from paper_2201_04622_amd import inputs as I

MVV2E = 1.0364269e-4
KB = 8.617333262e-5


def _einstein_run(O, N, k, T, dt, steps, seed, gamma=10.0):
    p = O.RunParams(mode="ein_rs", T=T, gamma=gamma, dt=dt, k=k, seed=seed, fix_com=False)
    x0 = np.zeros((N, 3)) + np.arange(N)[:, None] * 3.0
    L = np.full(3, 1000.0)
    x = x0.copy()
    v = O.init_velocities(p, N)
    lam = np.ones(steps + 1)
    dH, W, e, st = O.run(None, p, x0, L, x, v, lam, energies=True)
    return dH, e


def test_baoab_harmonic_sampling(oracle_lib):
    N, k, T, dt = 200, 5.0, 300.0, 0.02
    dH, e = _einstein_run(oracle_lib, N, k, T, dt, 12000, seed=1)
    kT = KB * T
    burn = 500
    upot = dH[burn:]                       # U_E(x_s) at lambda = 1
    ke = e[burn:-1] - dH[burn + 1:]        # KE after step s = E_s - U(x_{s+1})
    conf = upot.mean() / (1.5 * N * kT)
    kin = ke.mean() / (1.5 * N * kT)
    w = np.sqrt(k / (55.845 * MVV2E))
    assert conf == pytest.approx(1.0, abs=6e-3)
    assert kin == pytest.approx(1.0 - (w * dt / 2) ** 2, abs=6e-3)
    assert abs(kin - 1.0) > 0.05            # the bias is real at this w*dt


def _nve_spread(O, pot, dt, steps):
    x0 = I.lattice_sites("bcc", 6, I.A_BCC_STABLE)
    L = np.full(3, 6 * I.A_BCC_STABLE)
    p = O.RunParams(mode="fl", T=300.0, gamma=0.0, dt=dt, seed=4, fix_com=True, skin=0.5, nlist_cap=400)
    x = x0.copy()
    v = O.init_velocities(p, len(x0))
    lam = np.zeros(steps + 1)
    _, _, e, _ = O.run(pot, p, x0, L, x, v, lam, energies=True)
    return e / len(x0)


def test_nve_energy_conservation_second_order(oracle_lib, opot):
    e1 = _nve_spread(oracle_lib, opot, 0.001, 400)
    e2 = _nve_spread(oracle_lib, opot, 0.0005, 800)
    s1 = e1.max() - e1.min()
    s2 = e2.max() - e2.min()
    assert s1 < 2e-4                       # eV/atom over 0.4 ps at 300 K
    assert 2.5 < s1 / s2 < 6.0             # error ~ dt^2
    drift = abs(np.polyfit(np.arange(len(e1)), e1, 1)[0]) * len(e1)
    assert drift < 5e-5


def _hh(O, N, k1, k2, T, n_sw, reps, fix_com, n_eq=1500, scale=None):
    p = O.RunParams(mode="hh", T=T, k=k1, k2=k2, fix_com=fix_com)
    lam = O.schedule("hh", n_eq, n_sw, n_eq, 0, function=2)
    Wf, Wb = [], []
    for s in range(reps):
        p.seed = 1000 + s
        x0 = np.arange(N)[:, None] * np.array([2.0, 0.0, 0.0])
        x = x0.copy()
        v = O.init_velocities(p, N)
        _, W, _, _ = O.run(None, p, x0, np.full(3, 1000.0), x, v, lam, spring_scale=scale)
        wf = W[n_eq + n_sw - 1]
        Wf.append(wf)
        Wb.append(W[-1] - wf)
    return np.array(Wf), np.array(Wb)


@pytest.mark.parametrize("fix_com", [False, True])
def test_harmonic_to_harmonic_exact(oracle_lib, fix_com):
    N, k1, k2, T = 24, 2.0, 8.0, 300.0
    Wf, Wb = _hh(oracle_lib, N, k1, k2, T, n_sw=6000, reps=32, fix_com=fix_com)
    dF, ediss, err = E.forward_backward(Wf, Wb)
    ndof = N - 1 if fix_com else N
    exact = 1.5 * ndof * KB * T * np.log(k2 / k1)
    assert abs(dF - exact) < 4 * err
    # the estimate resolves the N vs N-1 degrees of freedom the CM constraint removes
    assert 1.5 * KB * T * np.log(k2 / k1) > 6 * err
    # dissipation of the two directions agrees (linear response), both >= 0 on average
    dfwd = Wf.mean() - exact
    dbwd = Wb.mean() + exact
    assert dfwd > -3 * Wf.std() / 4 and dbwd > -3 * Wb.std() / 4
    assert abs(dfwd - dbwd) < 4 * np.sqrt(Wf.var() + Wb.var()) / np.sqrt(len(Wf)) + 0.2 * abs(dfwd + dbwd)
    if not fix_com:
        # Frenkel--Ladd assembly: with H0 = springs k1 and H_E = springs k2,
        # F0 must come out as the Einstein free energy at k1.
        F0, _, _ = E.frenkel_ladd(Wf, Wb, N, T, k2, 55.845)
        assert F0 == pytest.approx(E.einstein_free_energy(N, T, k1, 55.845), abs=4 * err)


def test_reversible_scaling_on_einstein_crystal(oracle_lib):
    N, k, T0, lf = 24, 5.0, 100.0, 0.25
    p = oracle_lib.RunParams(mode="ein_rs", T=T0, k=k, fix_com=False)
    n_eq, n_sw, n_hold = 1000, 3000, 1000
    lam = oracle_lib.schedule("ein_rs", n_eq, n_sw, n_hold, 0, lambda_f=lf)
    T_grid = np.arange(100.0, 401.0, 1.0)
    curves = []
    for s in range(8):
        p.seed = 50 + s
        x0 = np.arange(N)[:, None] * np.array([0.0, 2.0, 0.0])
        x = x0.copy()
        v = oracle_lib.init_velocities(p, N)
        _, W, _, _ = oracle_lib.run(None, p, x0, np.full(3, 1000.0), x, v, lam)
        fw, bw = E.rs_work_curves(W, n_eq, n_sw, n_hold)
        F0 = E.einstein_free_energy(N, T0, k, 55.845)
        curves.append(E.reversible_scaling(F0, T0, lf, N, fw, bw, T_grid))
    curves = np.array(curves)
    ref = E.einstein_free_energy(N, T_grid, k, 55.845)
    mean = curves.mean(0)
    err = curves.std(0, ddof=1) / np.sqrt(len(curves)) + 1e-12
    assert np.all(np.abs(mean - ref) < 5 * err + 2e-4 * N)
    assert mean[0] == pytest.approx(ref[0], abs=1e-9)


def test_fixed_center_of_mass(oracle_lib, opot):
    x0 = I.lattice_sites("bcc", 4, 2.855)
    L = np.full(3, 4 * 2.855)
    p = oracle_lib.RunParams(mode="fl", T=100.0, k=5.0, seed=0, fix_com=True)
    x = x0.copy()
    v = oracle_lib.init_velocities(p, len(x0))
    assert np.abs(v.sum(0)).max() < 1e-12
    lam = oracle_lib.schedule("fl", 20, 60, 10, 10)
    oracle_lib.run(opot, p, x0, L, x, v, lam)
    vscale = np.sqrt((v ** 2).mean())
    assert np.abs(v.mean(0)).max() < 1e-9 * vscale
    assert np.abs((x - x0).mean(0)).max() < 1e-9
    p.fix_com = False
    x = x0.copy(); v = oracle_lib.init_velocities(p, len(x0))
    oracle_lib.run(opot, p, x0, L, x, v, lam)
    assert np.abs(v.mean(0)).max() > 1e-4 * vscale


def test_verlet_candidates_match_brute_force(oracle_lib, opot):
    x0 = I.lattice_sites("bcc", 4, 2.855)
    L = np.full(3, 4 * 2.855)
    lam = oracle_lib.schedule("fl", 30, 60, 10, 0)
    out = []
    for skin in (0.0, 0.3):
        p = oracle_lib.RunParams(mode="fl", T=100.0, k=5.0, seed=2, skin=skin)
        x = x0.copy(); v = oracle_lib.init_velocities(p, len(x0))
        dH, W, _, _ = oracle_lib.run(opot, p, x0, L, x, v, lam)
        out.append((x, v, dH, W))
    assert np.allclose(out[0][0], out[1][0], atol=1e-9)
    assert np.allclose(out[0][2], out[1][2], rtol=1e-10, atol=1e-9)


def test_einstein_free_energy_by_quadrature():
    """F_E = -kT ln Z with Z the phase-space integral / h^{3N} of Eq. Z for
    independent oscillators, integrated numerically."""
    T, k, m = 700.0, 3.0, 55.845
    beta = 1.0 / (KB * T)
    hplanck = 2 * np.pi * 6.582119569e-4 / MVV2E                 # amu A^2 / ps
    sx = 1 / np.sqrt(beta * k)
    sp = np.sqrt(m / (beta * MVV2E))
    zx = integrate.quad(lambda x: np.exp(-0.5 * beta * k * x * x), -12 * sx, 12 * sx)[0]
    zp = integrate.quad(lambda p: np.exp(-beta * p * p * MVV2E / (2 * m)), -12 * sp, 12 * sp)[0]
    F1 = -KB * T * np.log(zx * zp / hplanck)
    N = 11
    assert E.einstein_free_energy(N, T, k, m) == pytest.approx(3 * N * F1, rel=1e-10)


def test_fixed_cm_gaussian_part():
    """The Einstein-crystal part of Eq. cm: fixing the centre of mass of N
    independent oscillators multiplies Z by the density of x_cm at its mean."""
    N, T, k, V = 128, 100.0, 5.0, 1000.0
    cov = KB * T / (N * k) * np.eye(3)
    pdf0 = stats.multivariate_normal(mean=np.zeros(3), cov=cov).pdf(np.zeros(3))
    expect = KB * T * np.log(N / V) - KB * T * np.log(pdf0)
    assert E.fixed_cm_correction(N, V, T, k) == pytest.approx(expect, rel=1e-12)


def test_jarzynski_gaussian_work():
    rng = np.random.default_rng(0)
    T = 300.0
    kT = KB * T
    mu, sd = 0.3, 0.6 * kT
    W = rng.normal(mu, sd, 400000)
    assert E.jarzynski(W, T) == pytest.approx(mu - sd ** 2 / (2 * kT), abs=3e-4)


def test_msd_removes_the_centre_of_mass():
    """The oracle's MSD with the centre of mass removed against the pair
    identity mean_i |d_i - <d>|^2 = (1 / 2n^2) sum_ij |d_i - d_j|^2 (brute
    force over pairs), and a rigid translation, which has none."""
    rng = np.random.default_rng(5)
    x0 = rng.uniform(0.0, 10.0, (17, 3))
    d = 0.2 * rng.standard_normal((17, 3))
    pair = sum(float(((d[i] - d[j]) ** 2).sum()) for i in range(17) for j in range(17)) / (2 * 17 ** 2)
    assert E.msd_com_removed(x0 + d, x0) == pytest.approx(pair, rel=1e-13)
    assert E.msd_com_removed(x0 + np.array([0.3, -1.2, 2.0]), x0) == pytest.approx(0.0, abs=1e-24)
    assert E.spring_constant(E.msd_com_removed(x0 + d, x0), 300.0) == pytest.approx(3 * E.KB * 300.0 / pair)


def test_harmonic_to_harmonic_exact_with_per_atom_springs(oracle_lib):
    """Two species of springs (atom i's spring k s_i, s_i = 1 or 3): between
    Einstein crystals k1 s_i and k2 s_i the exact free-energy difference is
    (3/2) N kB T ln(k2/k1) whatever the s_i.  An s_i missing from either the
    spring force or the spring energy shifts <dH/dl> by the mean of 1/s_i
    (a third here) and fails this."""
    N, k1, k2, T = 24, 2.0, 8.0, 300.0
    scale = np.where(np.arange(N) % 2 == 0, 1.0, 3.0)
    Wf, Wb = _hh(oracle_lib, N, k1, k2, T, n_sw=6000, reps=32, fix_com=False, scale=scale)
    dF, ediss, err = E.forward_backward(Wf, Wb)
    exact = 1.5 * N * KB * T * np.log(k2 / k1)
    assert abs(dF - exact) < 4 * err, (dF, exact, err)
    assert exact * (1.0 - np.mean(1.0 / scale)) > 10 * err   # the test can see a missing s_i


def test_energy_conserved_with_per_atom_springs(oracle_lib):
    """Without friction the total energy KE + sum_i k s_i |x_i - x0_i|^2 / 2
    of an Einstein crystal with per-atom springs is conserved by velocity
    Verlet (to O(dt^2)): the spring force and energy use the same s_i."""
    O = oracle_lib
    N = 16
    p = O.RunParams(mode="ein_rs", T=600.0, gamma=0.0, dt=0.0005, k=4.0, seed=9, fix_com=False)
    x0 = np.zeros((N, 3)) + np.arange(N)[:, None] * 3.0
    x = x0.copy()
    v = O.init_velocities(p, N)
    scale = 1.0 + 2.0 * (np.arange(N) % 3)
    _, _, e, _ = O.run(None, p, x0, np.full(3, 1000.0), x, v, np.ones(4001), energies=True, spring_scale=scale)
    assert np.ptp(e) < 2e-3 * np.abs(e).mean(), (np.ptp(e), e.mean())


# Metal-unit constants rebuilt from SI values (CODATA 2018 exact and
# recommended), independently of the literals the oracle carries.
_EV_J = 1.602176634e-19
_AMU_KG = 1.66053906660e-27
_MVV2E_SI = _AMU_KG * 1e-20 / 1e-24 / _EV_J      # 1 amu A^2 / ps^2 in eV
_KB_SI = 1.380649e-23 / _EV_J                     # eV / K


@pytest.mark.parametrize("fix_com", [False, True])
def test_initial_velocities_have_the_maxwell_boltzmann_amplitude(oracle_lib, fix_com):
    """Initial velocities (Sec. p_fl, thermal start at T): each Cartesian
    component is Gaussian with variance kB T / m, so sum m v^2 / (N_dof kB T)
    = 1 with N_dof = 3N, or 3(N - 1) once the mean velocity is removed; the
    ratio of the sum of N_dof independent squared deviates has relative
    standard deviation sqrt(2 / N_dof).  A wrong factor in the amplitude
    (sqrt 2, a missing unit conversion, T for kB T) fails by many sigma."""
    N, T, mass = 100000, 300.0, 55.845
    p = oracle_lib.RunParams(mode="fl", T=T, mass=mass, seed=11, fix_com=fix_com)
    v = oracle_lib.init_velocities(p, N)
    dof = 3 * (N - 1) if fix_com else 3 * N
    ratio = mass * _MVV2E_SI * float(np.sum(v * v)) / (dof * _KB_SI * T)
    assert abs(ratio - 1.0) < 4.0 * np.sqrt(2.0 / dof), ratio
    sig = np.sqrt(_KB_SI * T / (mass * _MVV2E_SI))
    for c in range(3):   # each component alone, and its shape
        rc = float(np.sum(v[:, c] ** 2)) / (N * sig * sig)
        assert abs(rc - 1.0) < 4.0 * np.sqrt(2.0 / N), (c, rc)
        assert stats.kstest(v[:, c] / sig, "norm").pvalue > 1e-4
    # a second temperature scales the amplitude as sqrt(T)
    p2 = oracle_lib.RunParams(mode="fl", T=4 * T, mass=mass, seed=11, fix_com=fix_com)
    assert np.allclose(oracle_lib.init_velocities(p2, N), 2.0 * v, rtol=1e-13, atol=1e-13)
