"""Checks of the oracle's stored switching ensembles (tests/golden/ensembles.json,
written by tests/golden/make_ensembles.py from the oracle alone).

  - Eq. dFdL with the knots as the parameter: the oracle's adjoint average
    <dU/dtheta>_{lambda=0} along a smooth direction u matches the central
    difference of its own switching estimate of F0 (Eq. fl) at theta +- eps u.
    The two sides share nothing but the potential: one is a per-configuration
    derivative, the other a difference of nonequilibrium work averages.
  - Eq. Ediss: the dissipated work of the stable crystals is positive.
  - Per-replica values are finite and the ensembles have the sizes stated.
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _gold():
    with open(os.path.join(HERE, "golden", "ensembles.json")) as fh:
        return json.load(fh)


def _direction(knots):
    r = np.linspace(0.0, knots.r_cut, knots.n)
    q = np.linspace(0.0, knots.rho_max, knots.n)
    u = np.stack([np.exp(-((r - 2.0) / 0.3) ** 2),
                  0.3 * np.exp(-((r - 2.6) / 0.3) ** 2),
                  np.exp(-((q - 60.0) / 15.0) ** 2)])
    return u / np.linalg.norm(u)


def test_free_energy_differences_resolve_the_gradient():
    """Central differences of the oracle's F0 (Eq. fl) at theta +- eps u agree
    in sign and size with its adjoint average <dU/dtheta>_0 along u (Eq. dFdL):
    within 1 % here, where the 2000-step switching leaves a dissipation bias
    that depends on theta (the GPU test repeats the comparison with slow
    switching at the 0.5 meV/atom gate)."""
    g = _gold()
    fs = g["fl_stable"]
    N = fs["n_bcc"] ** 3 * 2
    eps = g["fl_stable_u"]["eps"]
    h = {s: np.array([-0.5 * (r["W_fwd"] - r["W_bwd"]) for r in g["runs"]["fl_stable_u"][s]])
         for s in ("plus", "minus")}
    fd = (h["plus"] - h["minus"]) / (2 * eps) / N
    adj = np.array([np.mean(np.array(r["grad_samples"])[:, 0]) for r in g["runs"]["fl_stable"]["bcc"]]) / N
    assert abs(fd.mean() - adj.mean()) <= 0.01 * abs(adj.mean()), (fd.mean(), adj.mean())
    # both resolved far above their scatter
    assert abs(adj.mean()) > 100 * adj.std(ddof=1) / np.sqrt(len(adj))
    assert abs(fd.mean()) > 100 * fd.std(ddof=1) / np.sqrt(len(fd))


def test_dissipation_is_positive():
    """Eq. Ediss: the mean dissipated work of both directions together is
    positive (second law); the switching is irreversible at this speed."""
    g = _gold()
    for kind in ("bcc", "fcc"):
        runs = g["runs"]["fl_stable"][kind]
        Wf = np.array([r["W_fwd"] for r in runs])
        Wb = np.array([r["W_bwd"] for r in runs])
        ed = 0.5 * (Wf + Wb)
        assert ed.mean() > 3 * ed.std(ddof=1) / np.sqrt(len(ed)), (kind, ed.mean())


def test_ensemble_shapes_and_values():
    from paper_2201_04622_amd import inputs as I
    g = _gold()
    knots = I.synthetic_eam_knots()
    assert _direction(knots).shape == (3, knots.n)
    fs = g["fl_stable"]
    for kind in ("bcc", "fcc"):
        runs = g["runs"]["fl_stable"][kind]
        assert len(runs) == fs["seeds"]
        for r in runs:
            s = np.array(r["grad_samples"])
            assert s.shape[1] == 1 + len(fs["knots"]) and np.isfinite(s).all()
            assert np.isfinite([r["W_fwd"], r["W_bwd"]]).all()
    assert len(g["runs"]["fl_verbatim"]["bcc"]) == g["fl_verbatim"]["seeds"]
    assert len(g["runs"]["rs_stable"]["bcc"]) == g["rs_stable"]["seeds"]
    for r in g["runs"]["rs_stable"]["bcc"]:
        assert len(r["F_minus_F0_over_l"]) == len(g["rs_stable"]["T_grid"])
