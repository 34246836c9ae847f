"""Statistical parity of the GPU switching ensembles with the FP64 oracle.

The oracle's ensembles are in tests/golden/ensembles.json, written by
tests/golden/make_ensembles.py, which calls only the oracle.  Here the same
replicas (same seeds, protocols and Philox noise) run batched on the GPU in
FP64 and in FP32, and the estimators are compared.  Each replica's GPU run
and oracle run consume the same noise, so they are compared as pairs: the
estimate of the difference is the mean over replicas of the per-replica
differences, with the standard error of that mean.  (Same-noise Langevin
trajectories separate only as fast as rounding differences grow; once they
have separated the pairs are independent and the paired error is the
combined one.)

Gates, per atom:
  - stable-crystal FL free energy F0 (Eq. fl with Eq. cm), dF(bcc -> fcc),
    and dF/dtheta = <dU/dtheta>_{lambda=0} (Eq. dFdL with theta = knots)
    projected on a smooth direction u and on 20 single knots:
    |GPU - oracle| <= 0.5 meV/atom and <= 3 standard errors;
  - the adjoint's dF/dtheta along u against central differences of F0 at
    theta +- eps u from slow switching runs (independent estimators): within
    3 combined standard errors and 0.5 meV/atom per unit of theta;
  - the verbatim 128-atom crystal (which disorders and dissipates ~3
    eV/atom, so its F0 scatters by tens of meV/atom) and the RS curve F(T) -
    F(T0)/lambda of Eq. rs (whose scatter grows with T): within 3 standard
    errors.
"""
import json
import os

import numpy as np
import pytest

from gpu_common import make_ctx, say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
GATE = 5e-4                       # eV/atom
NSIG = 3.0
# Pairs whose trajectories have not separated differ only by rounding, which
# in FP32 is a systematic offset of the work, not a random one (observed:
# ~2e-7 eV/atom on F0 of the stable crystals): allowed up to these floors.
FLOOR = {FP64: 1e-9, FP32: 2e-5}  # eV/atom
HERE = os.path.dirname(os.path.abspath(__file__))


def _gold():
    with open(os.path.join(HERE, "golden", "ensembles.json")) as fh:
        return json.load(fh)


def _direction(knots):
    # the smooth unit direction of the generator script, restated
    r = np.linspace(0.0, knots.r_cut, knots.n)
    q = np.linspace(0.0, knots.rho_max, knots.n)
    u = np.stack([np.exp(-((r - 2.0) / 0.3) ** 2),
                  0.3 * np.exp(-((r - 2.6) / 0.3) ** 2),
                  np.exp(-((q - 60.0) / 15.0) ** 2)])
    return u / np.linalg.norm(u)


def _paired(name, g, o, prec, gate=True):
    """g, o: per-replica values (per atom) of the same estimator's summand."""
    g, o = np.asarray(g, dtype=np.float64), np.asarray(o, dtype=np.float64)
    d = g - o
    n = d.size
    mean = d.mean()
    se = d.std(ddof=1) / np.sqrt(n)
    unpaired = np.hypot(g.std(ddof=1), o.std(ddof=1)) / np.sqrt(n)
    say(f"{name}: gpu {g.mean():.7f} oracle {o.mean():.7f} diff {mean * 1e3:+.5f} meV/atom, "
        f"paired se {se * 1e3:.5f}, unpaired se {unpaired * 1e3:.5f}")
    if gate:
        assert abs(mean) <= GATE, (name, mean)
    assert abs(mean) <= NSIG * se + FLOOR[prec], (name, mean, se)
    return mean, se


def _run_fl(prec, reps, prm, sample_every=0, sample_from=0):
    """One FL ensemble batched on the GPU: per-replica W_fwd, W_bwd and, with
    sampling, the per-replica mean dU/dtheta over the samples."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    ctx, x0, _ = make_ctx(reps, prec, 2, 256)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, 0.3, 0)
    p = E.protocol("fl", prm["n_eq"], prm["n_sw"], prm["n_hold"], prm["n_hold2"], function=2, skin=0.3)
    S = prm["n_eq"] + 2 * prm["n_sw"] + prm["n_hold"] + prm["n_hold2"]
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    acc = None
    s0 = 0
    if sample_every:
        # samples at x_s before step s, s = sample_from, sample_from + every, ... where lambda_s = 0
        assert sample_from < prm["n_eq"] and sample_from % sample_every == 0
        ctx.run_switching(p, x, v, 0, sample_from)
        s0 = sample_from
        acc = torch.zeros(len(reps), 3, I.N_KNOTS, dtype=torch.float64, device="cuda")
        ctx.set_adjoint_sampling(sample_every, acc)
    ctx.run_switching(p, x, v, s0, S, W_out=W)   # traces are indexed by the global step
    grads = None
    if sample_every:
        n = ctx.adjoint_samples()
        ctx.set_adjoint_sampling(0)
        grads = acc.cpu().numpy() / n
    ctx.close()
    W = W.cpu().numpy()
    e0, e1 = prm["n_eq"], prm["n_eq"] + prm["n_sw"]
    b0, b1 = e1 + prm["n_hold"], e1 + prm["n_hold"] + prm["n_sw"]
    W_fwd = W[:, e1 - 1] - (W[:, e0 - 1] if e0 > 0 else 0.0)
    W_bwd = W[:, b1 - 1] - W[:, b0 - 1]
    return W_fwd, W_bwd, grads


def _stable_reps(g, kind):
    fs = g["fl_stable"]
    n, a = (fs["n_bcc"], fs["a_bcc"]) if kind == "bcc" else (fs["n_fcc"], fs["a_fcc"])
    return [I.Replica(kind, n, a, fs["T"], fs["k"], s) for s in range(fs["seeds"])]


@pytest.fixture(scope="module")
def gold():
    return _gold()


@pytest.fixture(scope="module")
def stable_runs(gold):
    """GPU FL runs of the stable ensembles in both precisions (bcc and fcc in one batch)."""
    reps = _stable_reps(gold, "bcc") + _stable_reps(gold, "fcc")
    fs = gold["fl_stable"]
    out = {}
    for prec in (FP64, FP32):
        say(f"stable FL ensemble, precision {prec}, {len(reps)} replicas")
        out[prec] = _run_fl(prec, reps, fs, sample_every=fs["sample_every"], sample_from=fs["sample_from"])
    return reps, out


def _half_diff(Wf, Wb):
    # F0 = F_E + dF_CM - mean_r (W_fwd - W_bwd)/2: the replica summand of Eq. fl
    return -0.5 * (np.asarray(Wf) - np.asarray(Wb))


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_fl_free_energy_and_bcc_fcc_difference(gold, stable_runs, prec):
    import paper_2201_04622_amd.eamfe as E
    from oracle import estimators as OE
    reps, runs = stable_runs
    Wf, Wb, _ = runs[prec]
    nb = gold["fl_stable"]["seeds"]
    per = {}
    for kind, sl in (("bcc", slice(0, nb)), ("fcc", slice(nb, 2 * nb))):
        rep = reps[sl][0]
        N = rep.natoms
        orc = gold["runs"]["fl_stable"][kind]
        Wfo = np.array([r["W_fwd"] for r in orc])
        Wbo = np.array([r["W_bwd"] for r in orc])
        # the product's and the oracle's estimators: the same constant part (F_E + dF_CM)
        Fg, _, _ = E.fl_free_energy(Wf[sl], Wb[sl], N, rep.T, rep.k, rep.mass, N=N, V=float(np.prod(rep.box)))
        Fo, _, _ = OE.frenkel_ladd(Wfo, Wbo, N, rep.T, rep.k, rep.mass, N=N, V=float(np.prod(rep.box)))
        cg = Fg - _half_diff(Wf[sl], Wb[sl]).mean()
        co = Fo - _half_diff(Wfo, Wbo).mean()
        assert cg == pytest.approx(co, rel=1e-12, abs=1e-9)
        g = _half_diff(Wf[sl], Wb[sl]) / N
        o = _half_diff(Wfo, Wbo) / N
        _paired(f"F0/N {kind} prec={prec}", g, o, prec)
        per[kind] = (g, o)
    # dF(bcc -> fcc) per atom: replica r of each lattice has the same seed on both sides
    _paired(f"dF(bcc->fcc)/N prec={prec}", per["fcc"][0] - per["bcc"][0], per["fcc"][1] - per["bcc"][1], prec)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_fl_verbatim_small_crystal(gold, prec):
    fv = gold["fl_verbatim"]
    reps = [I.Replica("bcc", fv["n"], fv["a"], fv["T"], fv["k"], s) for s in range(fv["seeds"])]
    say(f"verbatim FL ensemble, precision {prec}")
    Wf, Wb, _ = _run_fl(prec, reps, fv)
    orc = gold["runs"]["fl_verbatim"]["bcc"]
    N = reps[0].natoms
    g = _half_diff(Wf, Wb) / N
    o = _half_diff([r["W_fwd"] for r in orc], [r["W_bwd"] for r in orc]) / N
    _paired(f"F0/N verbatim bcc4 prec={prec}", g, o, prec, gate=False)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_rs_free_energy_curve(gold, prec):
    import torch

    import paper_2201_04622_amd.eamfe as E
    rs = gold["rs_stable"]
    reps = [I.Replica("bcc", rs["n"], rs["a"], rs["T"], rs["k"], s) for s in range(rs["seeds"])]
    say(f"RS ensemble, precision {prec}")
    ctx, x0, _ = make_ctx(reps, prec, 2, 256)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, 0.3, 0)
    p = E.protocol("rs", rs["n_eq"], rs["n_sw"], rs["n_hold"], rs["n_hold2"], lambda_f=rs["lambda_f"], skin=0.3)
    S = rs["n_eq"] + 2 * rs["n_sw"] + rs["n_hold"] + rs["n_hold2"]
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, S, W_out=W)
    ctx.close()
    W = W.cpu().numpy()
    N = reps[0].natoms
    g = np.array([E.rs_free_energy(p, W[r], 0.0, rs["T"], N - 1, rs["T_grid"]) for r in range(len(reps))]) / N
    o = np.array([r["F_minus_F0_over_l"] for r in gold["runs"]["rs_stable"]["bcc"]]) / N
    for q, T in enumerate(rs["T_grid"]):
        _paired(f"RS F(T)-F(T0)/l at {T:.0f} K prec={prec}", g[:, q], o[:, q], prec, gate=False)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_dF_dtheta_matches_oracle(gold, stable_runs, prec):
    """Ensemble means of dU/dtheta at lambda = 0 (projected), GPU vs oracle."""
    reps, runs = stable_runs
    _, _, gr = runs[prec]
    knots = I.synthetic_eam_knots()
    u = _direction(knots)
    ks = [tuple(k) for k in gold["fl_stable"]["knots"]]
    nb = gold["fl_stable"]["seeds"]
    for kind, sl in (("bcc", slice(0, nb)), ("fcc", slice(nb, 2 * nb))):
        N = reps[sl][0].natoms
        proj_g = np.array([[np.sum(g * u)] + [g[f, k] for f, k in ks] for g in gr[sl]]) / N
        orc = gold["runs"]["fl_stable"][kind]
        proj_o = np.array([np.mean(np.array(r["grad_samples"]), axis=0) for r in orc]) / N
        for q in range(proj_g.shape[1]):
            name = "u" if q == 0 else f"knot {ks[q - 1]}"
            _paired(f"dF/dtheta {kind} {name} prec={prec}", proj_g[:, q], proj_o[:, q], prec)


def test_dF_dtheta_matches_free_energy_differences():
    """dF/dtheta along the smooth direction u from the adjoint (<dU/dtheta>_0,
    sampled in the lambda = 0 equilibration) against central differences of
    the FL free energy F0 at theta +- eps u, both from the FP64 GPU path
    (parity with the oracle is covered above).  The switching estimate of F0
    carries a dissipation bias that itself depends on theta; with the slow
    protocol used here (60k-step switching) that part of the difference is
    well below the gate (it is 0.86 meV/atom per unit theta at 2k steps and
    0.26 at 20k).  bcc 6^3 at the zero-pressure
    lattice constant, T = 100 K, 32 replicas with common random numbers."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    knots = I.synthetic_eam_knots()
    u = _direction(knots)
    th = knots.stacked()
    eps = 0.05
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 100.0, 5.0, s) for s in range(32)]
    N = reps[0].natoms
    prm = dict(n_eq=5000, n_sw=60000, n_hold=2000, n_hold2=0)
    h, adj = {}, []
    for sign in (1.0, -1.0):
        kn = I.PotentialKnots(knots.r_cut, knots.rho_max, *(th + sign * eps * u))
        say(f"FL at theta {'+' if sign > 0 else '-'} eps u, 32 replicas, {prm['n_eq'] + 2 * prm['n_sw'] + prm['n_hold']} steps")
        ctx, x0, _ = make_ctx(reps, FP64, 2, 256, knots=kn)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, 0.3, 0)
        p = E.protocol("fl", prm["n_eq"], prm["n_sw"], prm["n_hold"], prm["n_hold2"], function=2, skin=0.3)
        S = prm["n_eq"] + 2 * prm["n_sw"] + prm["n_hold"]
        W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
        ctx.run_switching(p, x, v, 0, 500)
        acc = torch.zeros(len(reps), 3, I.N_KNOTS, dtype=torch.float64, device="cuda")
        ctx.set_adjoint_sampling(100, acc)
        ctx.run_switching(p, x, v, 500, S, W_out=W)
        n = ctx.adjoint_samples()
        ctx.set_adjoint_sampling(0)
        ctx.close()
        W = W.cpu().numpy()
        e0, e1 = prm["n_eq"], prm["n_eq"] + prm["n_sw"]
        b0, b1 = e1 + prm["n_hold"], S
        h[sign] = _half_diff(W[:, e1 - 1] - W[:, e0 - 1], W[:, b1 - 1] - W[:, b0 - 1])
        g = acc.cpu().numpy() / n
        adj.append(np.array([np.sum(gr * u) for gr in g]))
    fd = (h[1.0] - h[-1.0]) / (2 * eps) / N           # paired over seeds
    ad = 0.5 * (adj[0] + adj[1]) / N                   # theta_0 up to O(eps^2)
    d = ad.mean() - fd.mean()
    se = np.hypot(ad.std(ddof=1), fd.std(ddof=1)) / np.sqrt(len(reps))
    say(f"dF/dtheta.u: adjoint {ad.mean():.6f} F0 differences {fd.mean():.6f} diff {d * 1e3:+.4f} meV/atom se {se * 1e3:.4f}")
    assert abs(d) <= GATE
    assert abs(d) <= NSIG * se
