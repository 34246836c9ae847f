"""Pressure tensor (virial + kinetic) on the GPU against the oracle, and the
zero-pressure lattice parameter found from batched fixed-volume runs."""
import numpy as np
import pytest

from gpu_common import make_ctx, say, split
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_pressure_matches_oracle(opot, prec):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 1), I.Replica("fcc", 5, I.A_FCC_VERBATIM, 600.0, 5.0, 2),
            I.Replica("hcp", 0, I.A_FCC_VERBATIM / np.sqrt(2.0), 300.0, 5.0, 3, cells=(6, 4, 4))]
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    x = I.displaced(arrs["x0"], 0.08, seed=12)
    v = np.random.default_rng(4).standard_normal(x.shape) * 5.0
    P = ctx.pressure(E.to_soa(x), E.to_soa(v))
    P0 = ctx.pressure(E.to_soa(x))
    tol = 1e-11 if prec == 0 else 2e-5
    off = ctx.offsets
    for r, rep in enumerate(reps):
        o = opot.pressure(x[off[r]:off[r + 1]], rep.box, v=v[off[r]:off[r + 1]], mass=rep.mass)
        o0 = opot.pressure(x[off[r]:off[r + 1]], rep.box, mass=rep.mass)
        scale = np.abs(o0).max()
        say(f"{rep.kind}: P {P[r]} vs oracle {o} (configurational scale {scale:.3e} eV/A^3)")
        assert np.abs(P[r] - o).max() <= tol * max(scale, np.abs(o).max())
        assert np.abs(P0[r] - o0).max() <= tol * scale
    ctx.close()


def test_zero_pressure_lattice_parameter(opot):
    """At 1 K the zero-pressure lattice parameter is the static one, where the
    oracle's perfect-lattice energy per atom is smallest (a golden-section
    search, independent of the virial); at 300 K the lattice found gives a
    mean pressure within its errors of zero in an independent run."""
    import paper_2201_04622_amd.lattice as LT

    def e_static(a):
        x = I.lattice_sites("bcc", 6, a)
        return opot.eam(x, np.full(3, 6 * a))["U"] / len(x)

    lo, hi = 0.97 * I.A_BCC_STABLE, 1.03 * I.A_BCC_STABLE
    g = (np.sqrt(5) - 1) / 2
    for _ in range(60):
        m1, m2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if e_static(m1) < e_static(m2):
            hi = m2
        else:
            lo = m1
    a_static = 0.5 * (lo + hi)
    cold = LT.zero_pressure_lattice("bcc", 6, 1.0, a_static, rel_span=0.003, n_trials=8, n_steps=1500,
                                    discard=500, every=50, precision=0)
    say(f"static minimum {a_static:.6f} A, zero pressure at 1 K {cold.a0:.6f} A")
    assert cold.a0 == pytest.approx(a_static, rel=2e-4)
    hot = LT.zero_pressure_lattice("bcc", 6, 300.0, a_static, rel_span=0.01, n_trials=8, n_steps=6000, discard=1500,
                                   iterations=2)
    check = LT.zero_pressure_lattice("bcc", 6, 300.0, hot.a0, rel_span=1e-9, n_trials=4, n_steps=6000, discard=1500,
                                     seed=50)
    say(f"300 K: a0 {hot.a0:.6f} A (thermal expansion {hot.a0 / a_static - 1:.2e}); check p = {check.p_mean} "
        f"+- {check.p_err} eV/A^3")
    assert hot.a0 > a_static   # the crystal expands on heating
    # the check's mean from the spread of its independent replicas, the
    # root's uncertainty as a pressure from the trials' block errors
    err = check.p_mean.std(ddof=1) / np.sqrt(len(check.p_mean))
    err_root = np.sqrt((hot.p_err ** 2).mean() / len(hot.p_err))
    assert abs(check.p_mean.mean()) < 4 * np.hypot(err, err_root), (check.p_mean, err, err_root)
