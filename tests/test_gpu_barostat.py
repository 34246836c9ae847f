"""Constant-pressure runs on the GPU: the barostat moves between fixed-volume
stretches follow the oracle's step by step on the same noise, and the
sampled volume agrees with the zero-pressure lattice parameter from
fixed-volume runs and with the compressibility their pressures imply."""
import numpy as np
import pytest

from gpu_common import make_ctx, say, split
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
KB = 8.617333262e-5


def _reps():
    return [
        I.Replica("bcc", 0, I.A_BCC_STABLE * 1.01, 300.0, 0.0, 11, cells=(6, 6, 6)),
        I.Replica("fcc", 0, I.A_FCC_STABLE * 0.99, 600.0, 0.0, 12, cells=(5, 5, 5)),
    ]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_npt_trajectory_matches_oracle(oracle_lib, opot, prec):
    """Reversible scaling (lambda from 1 to 0.7 and back) with a move every
    10 steps: boxes, scale factors, pressures, positions, velocities and work
    agree with the oracle on the same thermostat and barostat noise."""
    import torch

    import paper_2201_04622_amd.barostat as B
    import paper_2201_04622_amd.eamfe as E
    from oracle import barostat as OB
    say(f"npt trajectory prec={prec}")
    reps = _reps()
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    n_eq, n_sw, n_hold = 10, 40, 10
    p = E.protocol("rs", n_eq, n_sw, n_hold, 0, lambda_f=0.7, skin=0.3)
    S = n_eq + 2 * n_sw + n_hold
    every, p0, tau_p, beta_T = 10, 0.0, 0.2, 0.3
    b = B.barostat(p0, tau_p, beta_T, 0.001, every)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    v_init = E.from_soa(v)
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    tr = B.run_npt(ctx, p, x, v, 0, S, every, b, W_out=W)
    ctx.close()
    lam = oracle_lib.schedule("rs", n_eq, n_sw, n_hold, 0, lambda_f=0.7)
    xg, vg, Wg = E.from_soa(x), E.from_soa(v), W.cpu().numpy()
    tol = 1e-9 if prec == FP64 else 2e-3
    for r, (rep, xr, vr, vi) in enumerate(zip(reps, split(xg, ctx.offsets), split(vg, ctx.offsets),
                                               split(v_init, ctx.offsets))):
        po = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed, mass=rep.mass)
        xo, vo = rep.sites(), vi.copy()
        boxes, mus, Ps, Wo = OB.run_npt(opot, po, rep.sites(), rep.box, xo, vo, lam, every, p0, tau_p, beta_T)
        say(f"replica {r}: box {tr.boxes[-1, r]} vs {boxes[-1]}, |dx| {np.abs(xr - xo).max():.1e}")
        assert len(mus) == len(tr.mu) == (S - 1) // every
        assert np.abs(tr.boxes[:, r] / boxes - 1).max() < (1e-12 if prec == FP64 else 1e-6)
        assert np.all(tr.mu[:, r, 0] == tr.mu[:, r, 1]) and np.all(tr.mu[:, r, 0] == tr.mu[:, r, 2])
        assert np.abs(tr.mu[:, r, 0] / mus - 1).max() < (1e-12 if prec == FP64 else 1e-6)
        Pg = tr.pressure[:, r].mean(axis=-1)
        assert np.abs(Pg - Ps).max() < (1e-9 if prec == FP64 else 1e-3) * np.abs(Ps).max()
        assert np.abs(xr - xo).max() < tol, r
        assert np.abs(vr - vo).max() < tol * 100, r
        assert np.abs(Wg[r] - Wo).max() < tol * max(1.0, np.abs(Wo).max()), r
        assert np.abs(np.log(tr.boxes[-1, r] / rep.box)).max() > 1e-4   # the boxes did move


def test_npt_volume_matches_fixed_volume_zero_pressure():
    """bcc 6^3 at 300 K and p0 = 0: the mean lattice parameter of constant-
    pressure runs equals the root of the mean pressure of fixed-volume runs
    (lattice.zero_pressure_lattice) within the errors of both. The volume
    variance equals kB T V beta_T, with beta_T = -1 / (V dp/dV) taken from
    the slope of that root fit, to within 25 %. The barostat's own beta_T
    (0.3 A^3/eV) only sets the relaxation rate."""
    import torch

    import paper_2201_04622_amd.barostat as B
    import paper_2201_04622_amd.eamfe as E
    import paper_2201_04622_amd.lattice as LT
    T, cells = 300.0, (6, 6, 6)
    nvt = LT.zero_pressure_lattice("bcc", 6, T, I.A_BCC_STABLE * 1.001, rel_span=0.004, n_trials=8, n_steps=6000,
                                   discard=1500, iterations=2)
    reps = [I.Replica("bcc", 0, nvt.a0, T, 0.0, 200 + s, cells=cells) for s in range(8)]
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    n_steps, every = 20000, 10
    p = E.protocol("rs", n_steps, 1, 0, 0, lambda_f=1.0, skin=0.3)   # lambda = 1 throughout: plain dynamics
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    tr = B.run_npt(ctx, p, x, v, 0, n_steps, every, B.barostat(0.0, 0.2, 0.3, 0.001, every))
    ctx.close()
    a = tr.boxes[:, :, 0] / cells[0]                     # [moves + 1, replicas]
    late = a[len(a) // 4:]
    a_rep = late.mean(axis=0)
    a_npt, a_err = a_rep.mean(), a_rep.std(ddof=1) / np.sqrt(len(a_rep))
    root_err = np.sqrt((nvt.p_err ** 2).mean() / len(nvt.p_err)) / abs(nvt.slope)
    say(f"a: NPT {a_npt:.6f} +- {a_err:.1e}, fixed-volume root {nvt.a0:.6f} +- {root_err:.1e}")
    assert abs(a_npt - nvt.a0) < 4.0 * np.hypot(a_err, root_err) + 2e-5 * nvt.a0
    V = late ** 3 * np.prod(cells)                       # [samples, replicas]
    var_V = V.var(axis=0, ddof=1).mean()
    Vm = V.mean()
    beta_true = -3.0 / (nvt.a0 * nvt.slope)              # -(1/V) dV/dp with dV/da = 3 V / a
    say(f"volume variance {var_V:.4g} vs kT V beta {KB * T * Vm * beta_true:.4g} A^6")
    assert var_V == pytest.approx(KB * T * Vm * beta_true, rel=0.25)


def _fl_per_atom(reps, t_s, n_eq, n_hold):
    """F0 per atom of each replica (Eq. fl with Eq. cm), FP32 batched FL."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    ctx, x0, _ = make_ctx(reps, FP32, 2, 256)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    p = E.protocol("fl", n_eq, t_s, n_hold, 0, function=2, skin=0.3)
    S = n_eq + 2 * t_s + n_hold
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, S, W_out=W)
    ctx.close()
    Wf, Wb = E.switch_works(p, W.cpu().numpy())
    out = []
    for r, rep in enumerate(reps):
        N = rep.natoms
        F0, _, _ = E.fl_free_energy(Wf[r:r + 1], Wb[r:r + 1], N, rep.T, rep.k, rep.mass, N=N,
                                    V=float(np.prod(rep.box)))
        out.append(F0 / N)
    return np.asarray(out)


def test_rs_at_zero_pressure_matches_fl_at_the_zero_pressure_volume():
    """Gibbs energy at p = 0 by reversible scaling under the barostat, from
    T0 = 300 K to 600 K (lambda_f = 1/2) and back, started from the FL free
    energy at T0 in the box of the zero-pressure lattice parameter there.
    Against FL at 600 K in the box of the zero-pressure lattice parameter at
    600 K (at p = 0, G(T) = F(V*(T), T) up to terms of order kB T per system).
    Gate: 0.5 meV/atom and 3 combined standard errors."""
    import torch

    import paper_2201_04622_amd.barostat as B
    import paper_2201_04622_amd.eamfe as E
    import paper_2201_04622_amd.lattice as LT
    cells, k, T0, Tf = (6, 6, 6), 20.0, 300.0, 600.0
    a = {}
    for T in (T0, Tf):
        a[T] = LT.zero_pressure_lattice("bcc", 6, T, I.A_BCC_STABLE * (1.001 if T == T0 else 1.002), rel_span=0.004,
                                        n_trials=8, n_steps=6000, discard=1500, iterations=2).a0
    # FL at t_s = 32000: its two-way bias at 8000 (dissipation 1.5 meV/atom at 600 K) reaches 0.2 meV/atom
    fl = {T: _fl_per_atom([I.Replica("bcc", 0, a[T], T, k, 300 + s + int(T), cells=cells) for s in range(8)],
                          32000, 2000, 2000) for T in (T0, Tf)}
    reps = [I.Replica("bcc", 0, a[T0], T0, 0.0, 400 + s, cells=cells) for s in range(8)]
    N = reps[0].natoms
    ctx, x0, _ = make_ctx(reps, FP32, 2, 256)
    n_eq, n_sw, n_hold = 2000, 20000, 2000
    p = E.protocol("rs", n_eq, n_sw, n_hold, 0, lambda_f=T0 / Tf, skin=0.3)
    S = n_eq + 2 * n_sw + n_hold
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    tr = B.run_npt(ctx, p, x, v, 0, S, 10, B.barostat(0.0, 0.2, 0.3, 0.001, 10), W_out=W)
    ctx.close()
    W = W.cpu().numpy()
    F0 = fl[T0].mean() * N
    # Eq. rs in its fixed-centre-of-mass form; the volume in Eq. cm is the one at T0 (at 600 K the box is
    # 0.3 % larger, which moves Eq. cm by 1e-6 eV/atom)
    V0 = float(np.prod(reps[0].box))
    G = np.array([E.rs_free_energy_cm(p, W[r], F0, T0, N, V0, reps[0].mass, np.array([Tf]))[0]
                  for r in range(len(reps))]) / N
    a_hot = tr.boxes[n_eq // 10 + n_sw // 10: n_eq // 10 + n_sw // 10 + n_hold // 10, :, 0].mean() / cells[0]
    # the RS estimate inherits F0(T0) / lambda: its error doubles at lambda = 1/2
    se_rs = np.hypot(G.std(ddof=1) / np.sqrt(len(G)), 2.0 * fl[T0].std(ddof=1) / np.sqrt(len(fl[T0])))
    se_fl = fl[Tf].std(ddof=1) / np.sqrt(len(fl[Tf]))
    d = G.mean() - fl[Tf].mean()
    say(f"a*(300) {a[T0]:.6f}, a*(600) {a[Tf]:.6f}, NPT at 600 K {a_hot:.6f}; G_RS(600) {G.mean():.6f} "
        f"+- {se_rs:.1e}, F_FL(600) {fl[Tf].mean():.6f} +- {se_fl:.1e} eV/atom, diff {d * 1e3:+.4f} meV/atom")
    assert a_hot == pytest.approx(a[Tf], rel=3e-4)
    assert abs(d) < 5e-4 and abs(d) < 3.0 * np.hypot(se_rs, se_fl) + 2e-5


def test_barostat_rejects_bad_input_and_too_small_boxes():
    """Non-positive tau_p is EINVAL; a move that would take a box edge to
    2 (r_cut + skin) or below is EBOX and changes neither the boxes nor the
    positions and velocities."""
    import torch

    import paper_2201_04622_amd.barostat as B
    import paper_2201_04622_amd.eamfe as E
    rep = I.Replica("bcc", 0, I.A_BCC_STABLE, 300.0, 0.0, 5, cells=(6, 6, 6))   # edge 11.79 A, 2 (r_c + skin) = 11.2
    ctx, x0, _ = make_ctx([rep], FP64, 2, 256)
    p = E.protocol("rs", 20, 1, 0, 0, lambda_f=1.0, skin=0.3)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.run_switching(p, x, v, 0, 10)
    with pytest.raises(E.EamfeError) as e:
        ctx.barostat_step(B.barostat(0.0, 0.0, 0.3, 0.001, 10), 10, 1.0, x, v)
    assert e.value.code == 1
    xs, vs, L = x.clone(), v.clone(), ctx.boxes()
    # p0 = 10 eV/A^3 (1.6 TPa) with a fast coupling: the box would shrink by several per cent
    with pytest.raises(E.EamfeError) as e:
        ctx.barostat_step(B.barostat(10.0, 0.1, 1.0, 0.001, 10), 10, 1.0, x, v)
    assert e.value.code == 5
    assert np.array_equal(ctx.boxes(), L)
    assert torch.equal(x, xs) and torch.equal(v, vs)
    ctx.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_orthorhombic_npt_trajectory_matches_oracle(oracle_lib, opot, prec):
    """The orthorhombic move (each edge on its own) on an hcp cell started at
    the ideal c/a and a strained bcc cell, reversible scaling from 1 to 0.8
    and back with a move every 10 steps: per-axis boxes, factors and
    pressures, positions, velocities and work agree with the oracle on the
    same noise."""
    import torch

    import paper_2201_04622_amd.barostat as B
    import paper_2201_04622_amd.eamfe as E
    from oracle import barostat as OB
    say(f"orthorhombic npt trajectory prec={prec}")
    reps = [I.Replica("hcp", 0, 1.80, 400.0, 0.0, 21, cells=(7, 4, 4)),
            I.Replica("bcc", 0, I.A_BCC_STABLE * 1.01, 300.0, 0.0, 22, cells=(6, 7, 6))]
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    n_eq, n_sw, n_hold = 10, 40, 10
    p = E.protocol("rs", n_eq, n_sw, n_hold, 0, lambda_f=0.8, skin=0.3)
    S = n_eq + 2 * n_sw + n_hold
    every, p0, tau_p, beta_T = 10, 0.0, 0.1, 1.0
    b = B.barostat(p0, tau_p, beta_T, 0.001, every, aniso=True)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    v_init = E.from_soa(v)
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    tr = B.run_npt(ctx, p, x, v, 0, S, every, b, W_out=W)
    ctx.close()
    lam = oracle_lib.schedule("rs", n_eq, n_sw, n_hold, 0, lambda_f=0.8)
    xg, vg, Wg = E.from_soa(x), E.from_soa(v), W.cpu().numpy()
    tol = 1e-9 if prec == FP64 else 2e-3
    for r, (rep, xr, vr, vi) in enumerate(zip(reps, split(xg, ctx.offsets), split(vg, ctx.offsets),
                                               split(v_init, ctx.offsets))):
        po = oracle_lib.RunParams(mode="rs", T=rep.T, k=0.0, seed=rep.seed, mass=rep.mass)
        xo, vo = rep.sites(), vi.copy()
        boxes, mus, Ps, Wo = OB.run_npt(opot, po, rep.sites(), rep.box, xo, vo, lam, every, p0, tau_p, beta_T,
                                        aniso=True)
        say(f"replica {r}: box {tr.boxes[-1, r]} vs {boxes[-1]}, |dx| {np.abs(xr - xo).max():.1e}")
        assert tr.mu.shape[1:] == (len(reps), 3) and mus.shape == (len(tr.mu), 3)
        assert np.abs(tr.boxes[:, r] / boxes - 1).max() < (1e-12 if prec == FP64 else 1e-6)
        assert np.abs(tr.mu[:, r] / mus - 1).max() < (1e-12 if prec == FP64 else 1e-6)
        assert np.abs(tr.pressure[:, r] - Ps).max() < (1e-9 if prec == FP64 else 1e-3) * np.abs(Ps).max()
        assert np.abs(xr - xo).max() < tol, r
        assert np.abs(vr - vo).max() < tol * 100, r
        assert np.abs(Wg[r] - Wo).max() < tol * max(1.0, np.abs(Wo).max()), r
        # the edges moved by different factors
        assert np.ptp(np.log(tr.boxes[-1, r] / rep.box)) > 1e-4


def test_orthorhombic_barostat_relaxes_hcp_c_over_a():
    """hcp at 10 K and p0 = 0, started at the ideal c/a = sqrt(8/3): under the
    orthorhombic move c/a relaxes to that of lattice.zero_stress_hcp (the
    zero-stress cell from fixed-volume runs) within 1e-3, and a to its a;
    the isotropic move keeps the ideal c/a."""
    import torch

    import paper_2201_04622_amd.barostat as B
    import paper_2201_04622_amd.eamfe as E
    import paper_2201_04622_amd.lattice as LT
    T, cells = 10.0, (7, 4, 5)   # every edge above 2 (r_c + skin) at the trial cells too
    zs = LT.zero_stress_hcp(cells, T, 1.801, 1.56)
    a_zs = zs.a
    res = {}
    for aniso in (True, False):
        reps = [I.Replica("hcp", 0, a_zs * 1.003, T, 0.0, 40 + s, cells=cells) for s in range(4)]
        ctx, x0, _ = make_ctx(reps, FP32, 2, 256)
        p = E.protocol("rs", 6000, 1, 0, 0, lambda_f=1.0, skin=0.3)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        tr = B.run_npt(ctx, p, x, v, 0, 6000, 10, B.barostat(0.0, 0.1, 1.0, 0.001, 10, aniso=aniso))
        ctx.close()
        late = tr.boxes[len(tr.boxes) // 2:]
        a = late[:, :, 0] / cells[0]
        q = late[:, :, 2] / cells[2] / a
        res[aniso] = (a.mean(), q.mean())
    say(f"zero-stress cell: a {a_zs:.5f} c/a {zs.c_over_a:.5f}; orthorhombic barostat: a {res[True][0]:.5f} "
        f"c/a {res[True][1]:.5f}; isotropic: c/a {res[False][1]:.5f}")
    assert abs(res[True][1] - zs.c_over_a) < 1e-3
    assert abs(res[True][0] / a_zs - 1) < 1e-3
    assert abs(res[False][1] - np.sqrt(8.0 / 3.0)) < 1e-9
