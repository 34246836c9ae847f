"""The oracle's constant-pressure dynamics (isotropic stochastic cell
rescaling between fixed-volume stretches), pinned by the zero-coupling limit
and by the 0 K zero-pressure lattice parameter found from the static
pressure alone."""
import numpy as np

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
