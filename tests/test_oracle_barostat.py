"""The oracle's constant-pressure dynamics (isotropic stochastic cell
rescaling between fixed-volume stretches), pinned by the zero-coupling limit
and by the 0 K zero-pressure lattice parameter found from the static
pressure alone."""
import numpy as np
import pytest

from paper_2201_04622_amd import inputs as I


def _zero_pressure_a(opot, kind, cells, lo, hi):
    """Bisection on the static pressure of the perfect lattice: P(a) = 0."""
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        r = I.Replica(kind, 0, mid, 1.0, 0.0, 0, cells=cells)
        if np.mean(opot.pressure(r.sites(), r.box)) > 0.0:   # compressed: the root is larger
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_no_coupling_is_the_fixed_volume_run(oracle_lib, opot):
    """beta_T = 0 makes every move the identity: the chunked run with moves
    reproduces one uninterrupted fixed-volume run."""
    from oracle import barostat as OB
    rep = I.Replica("bcc", 0, I.A_BCC_STABLE * 1.01, 300.0, 0.0, 7, cells=(6, 6, 6))
    p = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed)
    lam = oracle_lib.schedule("rs", 5, 40, 5, 0, lambda_f=0.6)
    v0 = oracle_lib.init_velocities(p, rep.natoms)
    x1, v1 = rep.sites(), v0.copy()
    boxes, mus, Ps, W1 = OB.run_npt(opot, p, rep.sites(), rep.box, x1, v1, lam, 10, 0.0, 0.5, 0.0)
    x2, v2 = rep.sites(), v0.copy()
    _, W2, _, _ = oracle_lib.run(opot, p, rep.sites(), rep.box, x2, v2, lam)
    assert len(mus) == (len(lam) - 2) // 10 and np.all(mus == 1.0)
    assert np.all(boxes == rep.box)
    assert np.abs(x1 - x2).max() < 1e-12 and np.abs(v1 - v2).max() < 1e-11
    assert np.abs(W1 - W2).max() < 1e-9


def test_relaxes_to_the_zero_pressure_lattice_at_low_temperature(oracle_lib, opot):
    """At 1 K and p0 = 0 the box relaxes from 1.5 % too large to the lattice
    parameter at which the static pressure of the perfect crystal vanishes
    (thermal expansion at 1 K is far below the 2e-4 bar); a move's pressure
    is the static one plus the small kinetic part."""
    from oracle import barostat as OB
    cells = (6, 6, 6)
    a0 = _zero_pressure_a(opot, "bcc", cells, 1.9, 2.05)
    assert abs(a0 - I.A_BCC_STABLE) < 1e-3
    rep = I.Replica("bcc", 0, a0 * 1.015, 1.0, 0.0, 3, cells=cells)
    p = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed)
    lam = np.ones(3001)   # plain dynamics of U_EAM
    x, v = rep.sites(), oracle_lib.init_velocities(p, rep.natoms)
    boxes, mus, Ps, _ = OB.run_npt(opot, p, rep.sites(), rep.box, x, v, lam, 10, 0.0, 0.2, 0.3)
    a = boxes[:, 0] / cells[0]
    assert np.allclose(boxes[:, 0], boxes[:, 1]) and np.allclose(boxes[:, 0], boxes[:, 2])   # isotropic
    late = a[len(a) // 2:]
    assert abs(late.mean() / a0 - 1.0) < 2e-4, (late.mean(), a0)
    assert Ps[0] < 0.0            # the expanded start is under tension
    assert abs(Ps[-20:].mean()) < 2e-3 * abs(Ps[0])


def _virial_trace_by_strain(opot, x, L, h=1e-5):
    """Trace of the pair virial, sum over pairs of r_ij . f_ij, from the energy
    alone: under a uniform dilation x -> s x, L -> s L the energy changes by
    dU/ds = -tr W at s = 1 (central difference)."""
    up = opot.eam(x * (1 + h), L * (1 + h))["U"]
    dn = opot.eam(x * (1 - h), L * (1 - h))["U"]
    return -(up - dn) / (2 * h)


def test_move_statistics_match_the_published_rescaling(oracle_lib, opot):
    """One stochastic cell-rescaling move (Bernetti and Bussi 2020) at a fixed
    configuration: d eps = ln(V'/V) has the drift
    -(beta_T/tau_p)(p0 - P - kB T/V) dt and the variance
    2 kB T beta_T dt / (V tau_p), with P = (sum m v^2 + tr W)/(3 V) the internal
    pressure.  P is rebuilt here from a strain derivative of the energy, and
    the constants from SI values.  Over many steps (each keys its own
    deviate) the sample mean and variance of d eps must match, and since the
    deviate is a known function of (seed, step), each move must equal drift +
    amplitude z to rounding, which resolves the kB T / V term as well."""
    from oracle import barostat as OB
    rep = I.Replica("bcc", 0, I.A_BCC_STABLE * 1.01, 600.0, 0.0, 5, cells=(6, 6, 6))
    p = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed)
    x0 = I.displaced(rep.sites(), 0.04, seed=9)
    v0 = oracle_lib.init_velocities(p, rep.natoms)
    L = np.asarray(rep.box, dtype=np.float64)
    V = float(np.prod(L))
    w_eam, tau_p, beta_T, dt = 0.8, 0.2, 0.3, 0.01
    mass = 55.845
    P = (mass * _MVV2E_SI * float(np.sum(v0 * v0)) + w_eam * _virial_trace_by_strain(opot, x0, L)) / (3 * V)
    kT = _KB_SI * rep.T
    amp = np.sqrt(2 * kT * beta_T * dt / (V * tau_p))
    for p0 in (P + 0.05, P + kT / V):    # a strong drift, then the stationary point
        drift = -(beta_T / tau_p) * (p0 - P - kT / V) * dt
        deps, zs = [], []
        for step in range(1, 801):
            x, v = x0.copy(), v0.copy()
            L1, mu, Pm = OB.move(opot, x, v, L, rep.T, mass, rep.seed, step, w_eam, p0, tau_p, beta_T, dt)
            assert Pm == pytest.approx(P, rel=1e-7)
            assert np.allclose(L1, L * mu) and np.allclose(x, x0 * mu) and np.allclose(v, v0 / mu)
            deps.append(3 * np.log(mu))
            zs.append(oracle_lib.gauss3(rep.seed, 0, step, 3)[0])
        deps, zs = np.asarray(deps), np.asarray(zs)
        n = len(deps)
        assert abs(deps.mean() - drift) < 4 * amp / np.sqrt(n), (deps.mean(), drift)
        assert abs(deps.var(ddof=1) / amp ** 2 - 1) < 4 * np.sqrt(2.0 / (n - 1))
        # move by move: d eps - amp z is the drift; the kB T / V part of it is
        # (beta_T / tau_p)(kB T / V) dt, far above this bound
        assert np.abs(deps - amp * zs - drift).max() < 1e-3 * (beta_T / tau_p) * (kT / V) * dt


# the oracle-independent metal-unit constants (SI, CODATA 2018)
_EV_J = 1.602176634e-19
_MVV2E_SI = 1.66053906660e-27 * 1e-20 / 1e-24 / _EV_J
_KB_SI = 1.380649e-23 / _EV_J


def _hcp_zero_stress(opot, cells):
    """(a, c/a) of the perfect hcp lattice at zero static stress: P_xx = 0 and
    P_zz = 0 from the oracle's pressure tensor (P_yy = P_xx by the basal
    plane's symmetry)."""
    from scipy.optimize import fsolve

    def P(a, q):
        r = I.Replica("hcp", 0, a, 1.0, 0.0, 0, cells=cells, c_over_a=q)
        return opot.pressure(r.sites(), r.box)
    a, q = fsolve(lambda t: [P(*t)[0], P(*t)[2]], [1.78, 1.56], xtol=1e-12)
    assert np.abs(P(a, q)).max() < 1e-10
    return a, q


def _virial_diag_by_strain(opot, x, L, h=1e-5):
    """Pair virial W_aa of each axis from the energy alone: under the
    uniaxial stretch x_a -> s x_a, L_a -> s L_a, dU/ds = -W_aa at s = 1."""
    out = np.zeros(3)
    for a in range(3):
        e = np.ones(3)
        e[a] = 1 + h
        up = opot.eam(x * e, L * e)["U"]
        e[a] = 1 - h
        dn = opot.eam(x * e, L * e)["U"]
        out[a] = -(up - dn) / (2 * h)
    return out


def test_orthorhombic_move_statistics(oracle_lib, opot):
    """The orthorhombic move (each edge on its own, eps_a = ln L_a) at a
    fixed configuration of a strained, displaced hcp cell: per axis, the
    drift -(beta_T/(3 tau_p))(p0 - P_aa - kB T/V) dt and the variance
    2 kB T beta_T dt / (3 V tau_p), with P_aa rebuilt from a uniaxial strain
    derivative of the energy; move by move d eps_a - amp z_a is the drift, and
    the sum over axes is the isotropic move's drift and variance."""
    from oracle import barostat as OB
    cells = (7, 4, 4)
    a0, q0 = _hcp_zero_stress(opot, cells)
    rep = I.Replica("hcp", 0, a0 * 1.01, 500.0, 0.0, 6, cells=cells, c_over_a=q0 * 0.98)
    p = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed)
    x0 = I.displaced(rep.sites(), 0.04, seed=12)
    v0 = oracle_lib.init_velocities(p, rep.natoms)
    L = np.asarray(rep.box, dtype=np.float64)
    V = float(np.prod(L))
    w_eam, tau_p, beta_T, dt, mass = 0.9, 0.2, 0.3, 0.01, 55.845
    Paa = (mass * _MVV2E_SI * np.sum(v0 * v0, axis=0) + w_eam * _virial_diag_by_strain(opot, x0, L)) / V
    assert np.ptp(Paa) > 1e-3     # the strained cell's axes differ
    kT = _KB_SI * rep.T
    amp = np.sqrt(2 * kT * beta_T * dt / (3 * V * tau_p))
    p0 = float(Paa.mean()) + 0.03
    drift = -(beta_T / (3 * tau_p)) * (p0 - Paa - kT / V) * dt
    deps, zs = [], []
    for step in range(1, 401):
        x, v = x0.copy(), v0.copy()
        L1, mu, Pm = OB.move(opot, x, v, L, rep.T, mass, rep.seed, step, w_eam, p0, tau_p, beta_T, dt, aniso=True)
        assert np.allclose(Pm, Paa, rtol=1e-7)
        assert np.allclose(L1, L * mu) and np.allclose(x, x0 * mu) and np.allclose(v, v0 / mu)
        deps.append(np.log(mu))
        zs.append(oracle_lib.gauss3(rep.seed, 0, step, 3))
    deps, zs = np.asarray(deps), np.asarray(zs)
    n = len(deps)
    assert np.all(np.abs(deps.mean(0) - drift) < 4 * amp / np.sqrt(n))
    assert np.all(np.abs(deps.var(0, ddof=1) / amp ** 2 - 1) < 4 * np.sqrt(2.0 / (n - 1)))
    assert np.abs(deps - amp * zs - drift).max() < 1e-3 * (beta_T / (3 * tau_p)) * (kT / V) * dt
    # the volume: the isotropic drift and variance of ln V
    dlnV = deps.sum(1)
    assert abs(dlnV.mean() - drift.sum()) < 4 * np.sqrt(3) * amp / np.sqrt(n)
    assert abs(dlnV.var(ddof=1) / (2 * kT * beta_T * dt / (V * tau_p)) - 1) < 4 * np.sqrt(2.0 / (n - 1))


def test_orthorhombic_relaxes_hcp_to_the_zero_stress_cell(oracle_lib, opot):
    """At 1 K and p0 = 0, hcp started at the ideal c/a = sqrt(8/3) and with
    a 0.5 % too large relaxes under the orthorhombic move to the cell where
    the static stress tensor of the perfect lattice vanishes (c/a = 1.560 for
    this potential), keeping the basal plane's ratio; the isotropic move
    cannot change c/a."""
    from oracle import barostat as OB
    cells = (7, 4, 4)
    a0, q0 = _hcp_zero_stress(opot, cells)
    rep = I.Replica("hcp", 0, a0 * 1.005, 1.0, 0.0, 3, cells=cells)
    p = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed)
    lam = np.ones(1501)
    x, v = rep.sites(), oracle_lib.init_velocities(p, rep.natoms)
    boxes, mus, Ps, _ = OB.run_npt(opot, p, rep.sites(), rep.box, x, v, lam, 10, 0.0, 0.1, 1.0, aniso=True)
    a = boxes[:, 0] / cells[0]
    q = boxes[:, 2] / cells[2] / a
    plane = boxes[:, 1] / (cells[1] * np.sqrt(3.0)) / a
    late = slice(len(a) // 2, None)
    assert abs(q[0] - np.sqrt(8.0 / 3.0)) < 1e-12 and abs(q0 - 1.56) < 1e-3
    assert abs(q[late].mean() / q0 - 1) < 2e-4, (q[late].mean(), q0)
    assert abs(a[late].mean() / a0 - 1) < 2e-4
    assert abs(plane[late].mean() - 1) < 5e-4
