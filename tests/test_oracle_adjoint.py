"""Pins of the oracle's dU/dtheta (theta = the 3 x n knot values of phi, rho, F)
against central finite differences of the energy (exact for the phi and F
knots, on which U is linear) and against exact identities that follow from
the form of the EAM energy:
  sum_k dU/dF_k = N            (a natural spline reproduces constants),
  phi . dU/dphi = U_pair,  F . dU/dF = U_embed   (U linear in those knots),
  rho . dU/drho = sum_i F'(rho_i) rho_i          (rho_i linear in the rho knots).
By Eq. dFdL with theta in the role of lambda, <dU/dtheta> is dF/dtheta."""
import numpy as np
import pytest

from paper_2201_04622_amd import inputs as I


@pytest.fixture(scope="module")
def system():
    x0 = I.lattice_sites("bcc", 4, 2.855)
    L = np.full(3, 4 * 2.855)
    return I.displaced(x0, 0.07, seed=21), L


@pytest.fixture(scope="module")
def grad(opot, system):
    x, L = system
    return opot.adjoint_theta(x, L)


def _energy(O, knots, x, L, which=None, k=None, h=0.0):
    phi, rho, F = knots.phi.copy(), knots.rho.copy(), knots.embed.copy()
    arr = {"phi": phi, "rho": rho, "F": F}
    if which:
        arr[which][k] += h
    pot = O.Potential(phi, rho, F, knots.r_cut, knots.rho_max)
    return pot.eam(x, L)["U"]


@pytest.mark.parametrize("which,row", [("phi", 0), ("rho", 1), ("F", 2)])
def test_knot_gradient_matches_finite_differences(oracle_lib, knots, system, grad, which, row):
    x, L = system
    rng = np.random.default_rng(row)
    if which == "F":
        r = oracle_lib.Potential.from_knots(knots).eam(x, L)["rho"]
        lo = int(r.min() / (knots.rho_max / (knots.n - 1))) - 2
        hi = int(r.max() / (knots.rho_max / (knots.n - 1))) + 3
    else:
        lo, hi = int(1.8 / (knots.r_cut / (knots.n - 1))), knots.n - 1
    ks = rng.integers(lo, hi, 5)
    h = 1e-3 if which != "rho" else 1e-5
    for k in ks:
        fd = (_energy(oracle_lib, knots, x, L, which, k, h) - _energy(oracle_lib, knots, x, L, which, k, -h)) / (2 * h)
        tol = 1e-8 * max(1.0, abs(fd)) + (1e-9 if which != "rho" else 1e-6 * max(1.0, abs(fd)))
        assert grad[row, k] == pytest.approx(fd, abs=tol)


def test_gradient_identities(opot, knots, system, grad):
    x, L = system
    r = opot.eam(x, L)
    N = len(x)
    coef_phi, coef_rho, coef_F = opot.coefficients()
    # U_embed recomputed from the oracle's own per-atom F values via the spline
    from oracle import oracle as O
    hF = knots.rho_max / (knots.n - 1)
    U_emb = sum(O.spline_eval(coef_F, hF, rho)[0] for rho in r["rho"])
    U_pair = r["U"] - U_emb
    assert grad[2].sum() == pytest.approx(N, rel=1e-11)
    assert knots.phi @ grad[0] == pytest.approx(U_pair, rel=1e-10)
    assert knots.embed @ grad[2] == pytest.approx(U_emb, rel=1e-10)
    assert knots.rho @ grad[1] == pytest.approx(float((r["Fp"] * r["rho"]).sum()), rel=1e-10)
    # knots far below every pair distance carry only the geometrically decaying
    # tail of the (non-local) natural-spline basis
    assert np.abs(grad[0][: int(1.0 / (knots.r_cut / (knots.n - 1)))]).max() < 1e-100
