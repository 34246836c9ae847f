"""The automated phase comparison: zero-pressure lattice parameter, spring
constant from the MSD and FL for bcc, fcc and hcp, end to end.  At 10 K the
free-energy differences are the static energy differences of the relaxed
perfect lattices (each at its own zero-pressure lattice parameter, found by
the oracle from the static energy alone) up to the vibrational part, a few
0.1 meV/atom."""
import numpy as np
import pytest

from gpu_common import say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu


def _static_minimum(opot, kind, cells, a_guess):
    """Golden-section minimum of the perfect lattice's energy per atom over a."""
    def e(a):
        r = I.Replica(kind, 0, a, 1.0, 1.0, 0, cells=cells)
        return opot.eam(r.sites(), r.box)["U"] / r.natoms
    lo, hi = 0.97 * a_guess, 1.03 * a_guess
    g = (np.sqrt(5.0) - 1.0) / 2.0
    for _ in range(60):
        m1, m2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if e(m1) < e(m2):
            hi = m2
        else:
            lo = m1
    a = 0.5 * (lo + hi)
    return a, e(a)


def _static_minimum_hcp(opot, cells, a_guess, q_guess):
    """Minimum of the perfect hcp lattice's energy per atom over a and c/a
    (Nelder-Mead on the oracle's energy; no virial involved)."""
    from scipy.optimize import minimize

    def e(z):
        r = I.Replica("hcp", 0, z[0], 1.0, 1.0, 0, cells=cells, c_over_a=z[1])
        return opot.eam(r.sites(), r.box)["U"] / r.natoms

    m = minimize(e, [a_guess, q_guess], method="Nelder-Mead",
                 options={"xatol": 1e-8, "fatol": 1e-13, "maxiter": 2000, "initial_simplex":
                          [[a_guess, q_guess], [1.02 * a_guess, q_guess], [a_guess, 0.96 * q_guess]]})
    assert m.success
    return m.x[0], m.fun, m.x[1]


def test_phase_ranking_at_low_temperature_follows_static_energies(opot):
    import paper_2201_04622_amd.phases as PH
    res, order = PH.rank_phases(10.0)
    static = {kd: _static_minimum(opot, kd, PH.CELLS[kd], PH.A_GUESS[kd]) for kd in ("bcc", "fcc")}
    static["hcp"] = _static_minimum_hcp(opot, PH.CELLS["hcp"], PH.A_GUESS["hcp"], np.sqrt(8.0 / 3.0))
    say(f"hcp static c/a {static['hcp'][2]:.5f}, at 10 K {res['hcp'].c_over_a:.5f}")
    assert res["hcp"].c_over_a == pytest.approx(static["hcp"][2], rel=1e-3)
    for kd, ph in res.items():
        say(f"{kd}: a {ph.a:.5f} (static {static[kd][0]:.5f}), k {ph.k:.2f}, F {ph.F_per_atom:.6f} +- {ph.F_err:.1e} "
            f"(static E {static[kd][1]:.6f}), dissipation {ph.E_diss_per_atom * 1e3:.4f} meV/atom")
        assert ph.a == pytest.approx(static[kd][0], rel=1e-3)
    assert order == sorted(static, key=lambda kd: static[kd][1])
    for a, b in (("bcc", "fcc"), ("fcc", "hcp")):
        d_fl = res[b].F_per_atom - res[a].F_per_atom
        d_st = static[b][1] - static[a][1]
        err = np.hypot(res[a].F_err, res[b].F_err)
        say(f"F_{b} - F_{a}: {d_fl * 1e3:+.4f} meV/atom, static {d_st * 1e3:+.4f}")
        assert abs(d_fl - d_st) < 5e-4 + 3.0 * err
