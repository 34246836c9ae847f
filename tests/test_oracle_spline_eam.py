"""Pins of the oracle's tables and EAM sums against things other than itself:
scipy's natural cubic spline, closed-form lattice shell sums of the analytic
potential, a dimer closed form, central finite differences of the energy, and
symmetry invariants (translation, permutation, momentum)."""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from paper_2201_04622_amd import inputs as I


def test_spline_matches_scipy_natural(oracle_lib, knots):
    rng = np.random.default_rng(1)
    for y, top in ((knots.phi, knots.r_cut), (knots.rho, knots.r_cut), (knots.embed, knots.rho_max)):
        n = len(y)
        h = top / (n - 1)
        grid = np.arange(n) * h
        ref = CubicSpline(grid, y, bc_type="natural")
        coef = oracle_lib.spline_coefficients(y, h)
        xs = rng.uniform(0.0, top, 2000)
        for xq in xs:
            v, d = oracle_lib.spline_eval(coef, h, xq)
            scale = max(1.0, abs(float(ref(xq))))
            assert abs(v - float(ref(xq))) <= 1e-11 * scale
            assert abs(d - float(ref(xq, 1))) <= 1e-8 * max(1.0, abs(float(ref(xq, 1))))


def test_spline_random_data_and_linear_exactness(oracle_lib):
    rng = np.random.default_rng(2)
    y = rng.standard_normal(37)
    h = 0.37
    ref = CubicSpline(np.arange(37) * h, y, bc_type="natural")
    coef = oracle_lib.spline_coefficients(y, h)
    for xq in rng.uniform(0, 36 * h, 300):
        v, d = oracle_lib.spline_eval(coef, h, xq)
        assert v == pytest.approx(float(ref(xq)), abs=1e-12)
        assert d == pytest.approx(float(ref(xq, 1)), abs=1e-10)
    # a natural spline reproduces straight lines exactly
    lin = 2.5 - 0.75 * np.arange(11) * 0.2
    c = oracle_lib.spline_coefficients(lin, 0.2)
    for xq in np.linspace(0, 2.0, 41):
        v, d = oracle_lib.spline_eval(c, 0.2, xq)
        assert v == pytest.approx(2.5 - 0.75 * xq, abs=1e-13)
        assert d == pytest.approx(-0.75, abs=1e-12)


def _shells(kind, a, rc):
    """Distances and multiplicities of an infinite lattice around one site,
    enumerated directly from lattice vectors (no periodic box, no pair list)."""
    basis = I.BASIS[kind]
    m = int(np.ceil(rc / a)) + 1
    r = np.arange(-m, m + 1)
    cells = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    pts = (cells[:, None, :] + basis[None]).reshape(-1, 3) * a
    d = np.linalg.norm(pts, axis=1)
    d = d[(d > 1e-9) & (d < rc)]
    return d


@pytest.mark.parametrize("kind,a,n", [("bcc", 2.855, 4), ("fcc", 3.65, 3), ("bcc", 1.9646, 6), ("fcc", 2.5216, 5)])
def test_perfect_lattice_energy_equals_shell_sum(opot, kind, a, n):
    d = _shells(kind, a, I.R_CUT)
    rho = I.rho_analytic(d).sum()
    u_ref = I.embed_analytic(rho) + 0.5 * I.phi_analytic(d).sum()
    x = I.lattice_sites(kind, n, a)
    r = opot.eam(x, np.full(3, n * a))
    # spline vs analytic functions: value error below 2e-7 eV per evaluation
    assert np.allclose(r["rho"], rho, rtol=0, atol=1e-6 * len(d))
    assert r["U"] / len(x) == pytest.approx(u_ref, abs=2e-6 * len(d))
    assert np.abs(r["f"]).max() < 1e-10     # every site is a centre of inversion


def test_dimer_closed_form(opot, knots):
    """Two atoms: U = 2 F(rho(r)) + phi(r), |f| = phi'(r) + 2 F'(rho(r)) rho'(r)."""
    h = knots.r_cut / (knots.n - 1)
    grid = np.arange(knots.n) * h
    sphi = CubicSpline(grid, knots.phi, bc_type="natural")
    srho = CubicSpline(grid, knots.rho, bc_type="natural")
    sF = CubicSpline(np.arange(knots.n) * knots.rho_max / (knots.n - 1), knots.embed, bc_type="natural")
    L = np.full(3, 30.0)
    for r in (1.9, 2.48, 3.3, 4.95, 5.29):
        x = np.array([[10.0, 10.0, 10.0], [10.0 + r / np.sqrt(3), 10.0 + r / np.sqrt(3), 10.0 + r / np.sqrt(3)]])
        out = opot.eam(x, L)
        rr = float(srho(r))
        U = 2 * float(sF(rr)) + float(sphi(r))
        g = float(sphi(r, 1)) + 2 * float(sF(rr, 1)) * float(srho(r, 1))
        assert out["U"] == pytest.approx(U, rel=1e-12, abs=1e-12)
        u = (x[0] - x[1]) / r
        assert np.allclose(out["f"][0], -g * u, rtol=1e-9, atol=1e-11)
        assert np.allclose(out["f"][1], g * u, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("kind,a,n", [("bcc", 2.855, 4), ("fcc", 2.5216, 5)])
def test_forces_are_minus_energy_gradient(opot, kind, a, n):
    x0 = I.lattice_sites(kind, n, a)
    L = np.full(3, n * a)
    x = I.displaced(x0, 0.05, seed=7)
    r = opot.eam(x, L)
    rng = np.random.default_rng(3)
    h = 1e-5
    idx = rng.choice(len(x), 6, replace=False)
    for i in idx:
        for c in range(3):
            xp = x.copy(); xp[i, c] += h
            xm = x.copy(); xm[i, c] -= h
            fd = -(opot.eam(xp, L)["U"] - opot.eam(xm, L)["U"]) / (2 * h)
            assert fd == pytest.approx(r["f"][i, c], abs=2e-7 * max(1.0, np.abs(r["f"]).max()))


def test_invariances(opot):
    x0 = I.lattice_sites("bcc", 4, 2.855)
    L = np.full(3, 4 * 2.855)
    x = I.displaced(x0, 0.08, seed=11)
    r = opot.eam(x, L)
    assert np.abs(r["f"].sum(axis=0)).max() < 1e-11 * len(x)
    r2 = opot.eam(x + np.array([0.37, -1.3, 12.9]), L)       # translation (with unwrapped coordinates)
    assert r2["U"] == pytest.approx(r["U"], abs=1e-10)
    perm = np.random.default_rng(5).permutation(len(x))
    r3 = opot.eam(x[perm], L)
    assert r3["U"] == pytest.approx(r["U"], abs=1e-10)
    assert np.allclose(r3["f"], r["f"][perm], atol=1e-11)
    assert r["e_atom"].sum() == pytest.approx(r["U"], abs=1e-9)


def test_single_atom_query_matches_full_evaluation(opot):
    x0 = I.lattice_sites("fcc", 3, 3.65)
    L = np.full(3, 3 * 3.65)
    x = I.displaced(x0, 0.1, seed=2)
    r = opot.eam(x, L)
    for i in (0, 17, 107):
        a = opot.eam_atom(x, L, i)
        assert np.allclose(a["f"], r["f"][i], atol=1e-12)
        assert a["rho"] == pytest.approx(r["rho"][i], abs=1e-12)
        assert a["e_atom"] == pytest.approx(r["e_atom"][i], abs=1e-12)


def test_table_range_flag(oracle_lib, knots):
    # a tiny rho_max makes every density leave the table: flagged, still finite
    pot = oracle_lib.Potential(knots.phi, knots.rho, knots.embed, knots.r_cut, 5.0)
    x = I.lattice_sites("bcc", 4, 2.855)
    r = pot.eam(x, np.full(3, 4 * 2.855))
    assert r["status"] & oracle_lib.ETABLE
    assert np.isfinite(r["U"])


def test_small_box_rejected(opot):
    x = I.lattice_sites("bcc", 3, 2.855)   # L = 8.57 < 2 r_cut
    with pytest.raises(ValueError):
        opot.eam(x, np.full(3, 3 * 2.855))


@pytest.mark.parametrize("kind,n,a", [("bcc", 6, None), ("fcc", 5, None)])
def test_virial_is_minus_the_strain_derivative_of_the_energy(opot, kind, n, a):
    """The oracle's pair virial against finite differences of its energy
    under a homogeneous strain of one axis (positions and box edge scaled by
    1 + e): W_aa = -dU/de at e = 0, for displaced crystals, each axis."""
    a = a or (I.A_BCC_STABLE if kind == "bcc" else I.A_FCC_VERBATIM)
    x0 = I.lattice_sites(kind, n, a)
    L = np.full(3, n * a)
    rng = np.random.default_rng(2)
    x = x0 + 0.08 * rng.standard_normal(x0.shape)
    W = opot.pressure(x, L) * np.prod(L)   # no velocities: V P = W
    eps = 1e-5
    for c in range(3):
        s = np.ones(3)
        s[c] = 1 + eps
        up = opot.eam(x * s, L * s)["U"]
        s[c] = 1 - eps
        dn = opot.eam(x * s, L * s)["U"]
        assert W[c] == pytest.approx(-(up - dn) / (2 * eps), rel=1e-7, abs=1e-9)


def test_kinetic_pressure_term(opot):
    """The kinetic part of P_aa is sum m v_a^2 / V (metal units)."""
    x0 = I.lattice_sites("bcc", 6, I.A_BCC_STABLE)
    L = np.full(3, 6 * I.A_BCC_STABLE)
    v = np.random.default_rng(3).standard_normal(x0.shape)
    dP = opot.pressure(x0, L, v=v) - opot.pressure(x0, L)
    assert np.allclose(dP, 55.845 * 1.0364269e-4 * (v ** 2).sum(0) / np.prod(L), rtol=1e-12)
