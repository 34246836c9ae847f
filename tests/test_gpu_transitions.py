"""Gibbs energy curves at zero pressure by reversible scaling under the
barostat (the route of the paper's phase-stability figures), for bcc and fcc
from 300 to 900 K, against FL at 900 K in the box of each structure's
zero-pressure lattice parameter there, within three combined standard
errors plus 0.2 meV/atom (observed: bcc +0.61 +- 0.34, fcc -0.14 +- 0.45
meV/atom; bcc at these lattice parameters settles into a slightly distorted
structure, which makes its curve the noisier).  fcc stays above bcc by
10.2 meV/atom at 300 K and 6.8 at 900 K, so no transition is found."""
import numpy as np
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu


def test_gibbs_curves_end_on_fl_at_the_end_temperature():
    import paper_2201_04622_amd.lattice as LT
    import paper_2201_04622_amd.phases as PH
    import paper_2201_04622_amd.transitions as TR
    T0, Tf = 300.0, 900.0
    curves = {kd: TR.gibbs_curve(kd, T0, Tf) for kd in ("bcc", "fcc")}
    Ts = TR.transition_temperature(curves["bcc"], curves["fcc"])
    fl = {}
    for kd in ("bcc", "fcc"):
        ph = PH.phase_free_energy(kd, Tf, realizations=4, t_s=16000, seed=700)
        fl[kd] = ph
        c = curves[kd]
        d = c.G[-1] - ph.F_per_atom
        say(f"{kd}: a0(300) {c.a0:.5f}, k {c.k:.2f}; G(900) RS {c.G[-1]:.6f} +- {c.G_err[-1]:.1e}, "
            f"FL {ph.F_per_atom:.6f} +- {ph.F_err:.1e} (a {ph.a:.5f}), diff {d * 1e3:+.4f} meV/atom")
        assert abs(d) < 2e-4 + 3.0 * np.hypot(c.G_err[-1], ph.F_err)
    dG = curves["fcc"].G - curves["bcc"].G
    say(f"G_fcc - G_bcc: {dG[0] * 1e3:+.3f} meV/atom at 300 K, {dG[-1] * 1e3:+.3f} at 900 K; transition {Ts}")
    assert (Ts is None) == (np.sign(dG[0]) == np.sign(dG[-1]))


def test_hcp_gibbs_curve_ends_on_fl_at_the_end_temperature():
    """The hcp curve starts from the cell relaxed at 300 K (a and c/a), and
    the isotropic barostat keeps that c/a. At zero stress F is stationary in
    c/a, so the c/a drift to 900 K costs only second order. G(900 K) agrees
    with FL in the cell relaxed at 900 K within three combined standard
    errors plus 0.2 meV/atom; hcp stays below bcc (measured 7.3 meV/atom at
    300 K)."""
    import paper_2201_04622_amd.phases as PH
    import paper_2201_04622_amd.transitions as TR
    c = TR.gibbs_curve("hcp", 300.0, 900.0)
    ph = PH.phase_free_energy("hcp", 900.0, realizations=4, t_s=16000, seed=700)
    d = c.G[-1] - ph.F_per_atom
    say(f"hcp: G(900) RS {c.G[-1]:.6f} +- {c.G_err[-1]:.1e}, FL {ph.F_per_atom:.6f} +- {ph.F_err:.1e} "
        f"(c/a {ph.c_over_a:.5f}), diff {d * 1e3:+.4f} meV/atom")
    assert abs(d) < 2e-4 + 3.0 * np.hypot(c.G_err[-1], ph.F_err)
