"""GPU <-> oracle parity through the C ABI.

Forces and energies (FP64 to 1e-12, FP32 to 1e-5, normwise and per
component against the rms force), neighbour-list edge cases, bit-identical
FP32 results across launch shapes, same-noise trajectories step by step,
initial velocities, the harmonic -> harmonic closed form run on the GPU, and
the error paths the host can force."""
import numpy as np
import pytest

from gpu_common import make_ctx, rel_norm, say, split
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}
ETOL = {FP64: 1e-13, FP32: 1e-6}


def _mixed_batch():
    # uneven sizes, both lattices, verbatim and stable densities, all-pairs and cell lists
    return [
        # cells of edge >= (r_cut + skin)/2 where an edge holds five (0.3 A skin: L >= 14 A)
        I.Replica("bcc", 4, I.A_BCC_VERBATIM, 300.0, 5.0, 1),    # 128 atoms, L = 11.42 -> all-pairs
        I.Replica("fcc", 5, I.A_FCC_VERBATIM, 600.0, 5.0, 2),    # 500, L = 18.25 -> cells 6^3
        I.Replica("bcc", 7, I.A_BCC_STABLE, 900.0, 5.0, 3),      # 686 at high density, all-pairs
        I.Replica("fcc", 5, I.A_FCC_STABLE, 1200.0, 3.0, 4),     # 500 at high density, all-pairs
        I.Replica("bcc", 9, I.A_BCC_VERBATIM, 100.0, 5.0, 5),    # 1458, L = 25.7 -> cells 9^3
    ]


def _oracle_forces(opot, reps, x_aos, offsets):
    out = []
    for r, xr in zip(reps, split(x_aos, offsets)):
        out.append(opot.eam(xr, r.box))
    return out


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("lanes,block", [(1, 64), (4, 256), (16, 1024), (8, 128)])
def test_forces_and_energies_batched(opot, prec, lanes, block):
    import torch

    import paper_2201_04622_amd.eamfe as E
    say(f"forces: prec={prec} lanes={lanes} block={block}")
    reps = _mixed_batch()
    ctx, x0, arrs = make_ctx(reps, prec, lanes, block)
    x = I.displaced(arrs["x0"], 0.05, seed=11)
    xd = E.to_soa(x)
    ctx.neigh_build(xd, 0.3, 0)
    f = torch.zeros_like(xd)
    U = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
    ea = torch.zeros(xd.shape[1], dtype=torch.float64, device="cuda")
    ctx.eam_forces(xd, f, U, ea)
    fg = E.from_soa(f)
    eg = ea.cpu().numpy()
    ref = _oracle_forces(opot, reps, x, ctx.offsets)
    for r, (fr, er, o) in enumerate(zip(split(fg, ctx.offsets), split(eg, ctx.offsets), ref)):
        rms = np.sqrt((o["f"] ** 2).mean())
        assert rel_norm(fr, o["f"]) <= TOL[prec], (r, rel_norm(fr, o["f"]))
        assert np.abs(fr - o["f"]).max() <= TOL[prec] * rms * 10, r
        assert abs(U[r].item() - o["U"]) <= ETOL[prec] * abs(o["U"]), (r, U[r].item(), o["U"])
        assert np.abs(er - o["e_atom"]).max() <= ETOL[prec] * 100 * np.abs(o["e_atom"]).max()
    ctx.close()


def test_fp32_bitwise_identical_across_launch_shapes():
    """FP32 forces and energies are bitwise the same for every lanes x block
    shape, in both forms of the pair kernels: replica slices staged in LDS
    (the default) and the persistent grid gathering from global memory (a
    caller-fixed grid), with or without XCD grouping."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()
    x = None
    outs = []
    for lanes, block, grid, xcd in ((1, 64, 0, 1), (2, 256, 0, 1), (4, 512, 0, 1), (8, 1024, 0, 1), (16, 256, 0, 1),
                                    (2, 1024, 256, 1), (4, 256, 512, 0), (2, 1024, 0, 0)):
        say(f"fp32 shape {lanes}x{block} grid {grid} xcd {xcd}")
        ctx, x0, arrs = make_ctx(reps, FP32, lanes, block)
        ctx.set_xcd_affinity(xcd)
        if grid:
            ctx.set_grid(grid)
        if x is None:
            x = I.displaced(arrs["x0"], 0.06, seed=3)
        xd = E.to_soa(x)
        ctx.neigh_build(xd, 0.3, 0)
        f = torch.zeros_like(xd)
        U = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
        ctx.eam_forces(xd, f, U)
        outs.append((f.cpu().numpy(), U.cpu().numpy()))
        ctx.close()
    for f, U in outs[1:]:
        assert np.array_equal(f, outs[0][0])
        assert np.array_equal(U, outs[0][1])


def test_lists_rebuild_after_large_moves_and_skin_zero(opot):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("fcc", 6, I.A_FCC_VERBATIM, 300.0, 5.0, 9)]
    ctx, x0, arrs = make_ctx(reps, FP64)
    ctx.neigh_build(x0, 0.0, 0)       # skin 0: any motion forces a rebuild
    for seed in (1, 2, 3):
        x = I.displaced(arrs["x0"], 0.4, seed=seed) + 7.3   # big moves, shifted out of the box (unwrapped)
        xd = E.to_soa(x)
        f = torch.zeros_like(xd)
        U = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.eam_forces(xd, f, U)
        o = opot.eam(x, reps[0].box)
        assert rel_norm(E.from_soa(f), o["f"]) < 1e-12
        assert U.item() == pytest.approx(o["U"], rel=1e-13)
    ctx.close()


def test_neighbor_overflow_reported():
    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_VERBATIM, 300.0, 5.0, 9)]
    ctx, x0, arrs = make_ctx(reps, FP64)
    with pytest.raises(E.EamfeError) as e:
        ctx.neigh_build(x0, 0.3, 8)     # 58 neighbours per atom do not fit in 8
    assert e.value.code == 6
    ctx.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_density_beyond_the_table_reported(opot, prec):
    """A table that ends at rho_max = 5 (the stable crystal's densities are
    near 85): the force evaluation reports ETABLE_RANGE, as the oracle flags
    the same configuration."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    from oracle import oracle as O
    knots = I.synthetic_eam_knots(rho_max=5.0)
    rep = I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 9)
    ctx, x0, _ = make_ctx([rep], prec, knots=knots)
    ctx.neigh_build(x0, 0.3, 0)
    f = torch.zeros_like(x0)
    U = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EamfeError) as e:
        ctx.eam_forces(x0, f, U)
    assert e.value.code == 8
    ctx.close()
    assert O.Potential.from_knots(knots).eam(rep.sites(), rep.box)["status"] & O.ETABLE


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_non_finite_position_reported(prec):
    """A NaN coordinate: the lists and the pair passes stay in bounds (box
    codes and cells are bounded for any input), and the evaluation reports
    ENONFINITE."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    rep = I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 9)
    ctx, x0, _ = make_ctx([rep], prec)
    x = rep.sites()
    x[17, 1] = np.nan
    xd = E.to_soa(x)
    ctx.neigh_build(xd, 0.3, 0)
    f = torch.zeros_like(xd)
    U = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EamfeError) as e:
        ctx.eam_forces(xd, f, U)
    assert e.value.code == 9
    ctx.close()


def test_small_box_rejected():
    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 3, I.A_BCC_VERBATIM, 300.0, 5.0, 9)]   # L = 8.57 < 2 (5.3 + 0.3)
    ctx, x0, arrs = make_ctx(reps, FP64)
    with pytest.raises(E.EamfeError) as e:
        ctx.neigh_build(x0, 0.3, 0)
    assert e.value.code == 5
    ctx.close()


def test_init_velocities_match_oracle(oracle_lib):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()
    ctx, x0, arrs = make_ctx(reps, FP64)
    for fix in (True, False):
        v = torch.zeros_like(x0)
        ctx.init_velocities(v, fix)
        vg = E.from_soa(v)
        for r, vr in zip(reps, split(vg, ctx.offsets)):
            p = oracle_lib.RunParams(T=r.T, seed=r.seed, fix_com=fix, mass=r.mass)
            vo = oracle_lib.init_velocities(p, r.natoms)
            assert np.abs(vr - vo).max() < 1e-12 * np.abs(vo).max()
    ctx.close()


def _oracle_traj(oracle_lib, opot, r, x, v, lam, mode, fix_com, step0=0):
    p = oracle_lib.RunParams(mode=mode, T=r.T, k=r.k, k2=r.k2, seed=r.seed, fix_com=fix_com, mass=r.mass)
    xo, vo = x.copy(), v.copy()
    dH, W, _, _ = oracle_lib.run(opot if mode in ("fl", "rs") else None, p, r.sites(), r.box, xo, vo, lam,
                                 step0=step0)
    return xo, vo, dH, W


@pytest.mark.parametrize("prec,mode", [(FP64, "fl"), (FP64, "rs"), (FP32, "fl")])
def test_same_noise_trajectory(oracle_lib, opot, prec, mode):
    """Every replica's x, v, dH/dl and W follow the oracle step by step."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    say(f"trajectory prec={prec} mode={mode}")
    reps = _mixed_batch()[:4]
    ctx, x0, arrs = make_ctx(reps, prec, 4, 256)
    n_eq, n_sw, n_hold, n_hold2 = 10, 30, 5, 5
    p = E.protocol(mode, n_eq, n_sw, n_hold, n_hold2, function=2, lambda_f=0.5)
    S = n_eq + 2 * n_sw + n_hold + n_hold2
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    v_init = E.from_soa(v)
    dH = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    W = torch.zeros_like(dH)
    # two calls: the protocol can be split anywhere
    ctx.run_switching(p, x, v, 0, 37, None, dH, W)
    ctx.run_switching(p, x, v, 37, S, None, dH, W)
    lam = oracle_lib.schedule(mode, n_eq, n_sw, n_hold, n_hold2, function=2, lambda_f=0.5)
    xg, vg = E.from_soa(x), E.from_soa(v)
    dHg, Wg = dH.cpu().numpy(), W.cpu().numpy()
    tol = 1e-9 if prec == FP64 else 2e-3
    for r, (rep, xr, vr, vi) in enumerate(zip(reps, split(xg, ctx.offsets), split(vg, ctx.offsets),
                                               split(v_init, ctx.offsets))):
        xo, vo, dHo, Wo = _oracle_traj(oracle_lib, opot, rep, rep.sites(), vi, lam, mode, True)
        scale_w = max(1.0, np.abs(dHo).max())
        assert np.abs(xr - xo).max() < tol, (r, np.abs(xr - xo).max())
        assert np.abs(vr - vo).max() < tol * 100, (r, np.abs(vr - vo).max())
        assert np.abs(dHg[r] - dHo).max() < tol * scale_w, (r, np.abs(dHg[r] - dHo).max())
        assert np.abs(Wg[r] - Wo).max() < tol * scale_w, (r, np.abs(Wg[r] - Wo).max())
    ctx.close()


@pytest.mark.parametrize("mode", ["fl", "rs"])
def test_fp32_one_step_error_is_the_force_error(oracle_lib, opot, mode):
    """One FP32 step from the oracle's own state, at points across a
    protocol, differs from the oracle's step by no more than the FP32 force
    and energy errors measured at that state imply: with eps_f the largest
    force-component error and eps_u the energy error (GPU FP32 against the
    oracle at x_s, and eps_f' at the oracle's x_{s+1}), one B-A-O-A-B step
    gives |dx| <= (dt^2/2m) eps_f (the first half kick, carried through both
    drifts), |dv| <= (dt/2m)(eps_f + eps_f') plus the first-order change of
    the closing kick's force, |d dH/dl| <= eps_u (plus the grid of the
    replica sum of the spring energies in FL) and |dW| <= |dlambda| times
    that, each with a factor 2 for the rows' rounding groups, above a float64
    floor.  Unlike a whole-trajectory cap, a per-step bound this tight fails
    on any slip in the integration or the work sum."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    say(f"fp32 one-step error mode={mode}")
    reps = _mixed_batch()[:4]
    n_eq, n_sw, n_hold, n_hold2 = 10, 30, 5, 5
    S = n_eq + 2 * n_sw + n_hold + n_hold2
    p = E.protocol(mode, n_eq, n_sw, n_hold, n_hold2, function=2, lambda_f=0.5)
    lam = oracle_lib.schedule(mode, n_eq, n_sw, n_hold, n_hold2, function=2, lambda_f=0.5)
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    v0 = torch.zeros_like(x0)
    ctx.init_velocities(v0, True)
    v_init = split(E.from_soa(v0), ctx.offsets)
    m = reps[0].mass * 1.0364269e-4   # eV ps^2 / A^2
    dt = 0.001
    checks = (0, 12, 25, 40, 55, 70)
    # the oracle's trajectory, its states at the checked steps
    params = [oracle_lib.RunParams(mode=mode, T=r.T, k=r.k, seed=r.seed, fix_com=True, mass=r.mass) for r in reps]
    xs = [r.sites().copy() for r in reps]
    vs = [vi.copy() for vi in v_init]
    states, prev = {}, 0
    for s in checks:
        if s > prev:
            for q, r in enumerate(reps):
                oracle_lib.run(opot if mode in ("fl", "rs") else None, params[q], r.sites(), r.box, xs[q], vs[q],
                               lam[prev: s + 1], step0=prev)
        states[s] = ([a.copy() for a in xs], [a.copy() for a in vs])
        prev = s

    def fp32_errors(xl):
        x = E.to_soa(np.concatenate(xl))
        ctx.neigh_build(x, 0.3, 0)
        f = torch.zeros_like(x)
        U = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
        ctx.eam_forces(x, f, U)
        fg = split(E.from_soa(f), ctx.offsets)
        out = []
        for q, r in enumerate(reps):
            o = opot.eam(xl[q], r.box)
            out.append((float(np.abs(fg[q] - o["f"]).max()), abs(float(U[q]) - o["U"])))
        return out

    worst = 0.0
    for s in checks:
        xl, vl = states[s]
        err0 = fp32_errors(xl)
        x = E.to_soa(np.concatenate(xl))
        v = E.to_soa(np.concatenate(vl))
        W = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
        dH = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
        ctx.switch_step(p, s, x, v, W, dH)
        xg, vg = split(E.from_soa(x), ctx.offsets), split(E.from_soa(v), ctx.offsets)
        x1, v1, dH1, W1 = [], [], [], []
        for q, r in enumerate(reps):
            xo, vo = xl[q].copy(), vl[q].copy()
            dHo, Wo, _, _ = oracle_lib.run(opot, params[q], r.sites(), r.box, xo, vo, lam[s: s + 2], step0=s)
            x1.append(xo); v1.append(vo); dH1.append(float(dHo[0])); W1.append(float(Wo[0]))
        err1 = fp32_errors(x1)
        dlam = abs(lam[s + 1] - lam[s])
        for q, r in enumerate(reps):
            ef0, eu0 = err0[q]
            ef1, _ = err1[q]
            bx = 2.0 * dt * dt / (2.0 * m) * ef0 + 1e-11
            bv = 2.0 * dt / (2.0 * m) * (ef0 + ef1) + 1e-9
            # FL: the spring energies enter the replica sum on the 2^-24 grid (in A^2, times k/2)
            grid = 0.5 * r.k * r.natoms * 2.0 ** -25 if mode == "fl" else 0.0
            bh = 2.0 * eu0 + grid + 1e-9 * max(1.0, abs(dH1[q]))
            bw = dlam * bh + 1e-12
            dx = float(np.abs(xg[q] - x1[q]).max())
            dv = float(np.abs(vg[q] - v1[q]).max())
            dh = abs(float(dH[q]) - dH1[q])
            dw = abs(float(W[q]) - W1[q])
            say(f"step {s} rep {q}: eps_f {ef0:.1e} eps_u {eu0:.1e} | dx {dx:.1e}/{bx:.1e} dv {dv:.1e}/{bv:.1e} "
                f"dH {dh:.1e}/{bh:.1e} dW {dw:.1e}/{bw:.1e}")
            assert dx <= bx and dv <= bv and dh <= bh and dw <= bw, (s, q)
            worst = max(worst, dx / bx, dv / bv, dh / bh)
    say(f"largest share of a bound used: {worst:.2f}")
    ctx.close()


def test_switch_step_matches_run_switching():
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()[:3]
    p = E.protocol("fl", 3, 6, 2, 1)
    res = []
    for how in ("run", "step"):
        ctx, x0, arrs = make_ctx(reps, FP64)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        if how == "run":
            W = torch.zeros(len(reps), 18, dtype=torch.float64, device="cuda")
            ctx.run_switching(p, x, v, 0, 18, None, None, W)
            w = W[:, -1].clone()
        else:
            w = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
            dh = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
            for s in range(18):
                ctx.switch_step(p, s, x, v, w, dh)
        res.append((x.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy()))
        ctx.close()
    for a, b in zip(res[0], res[1]):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_harmonic_switching_on_gpu_reaches_closed_form(oracle_lib):
    """H(l) = (1-l) U_E(k1) + l U_E(k2): the forward/backward estimate run on the
    GPU reaches (3(N-1)/2) kT ln(k2/k1), and every replica's work trace equals
    the oracle's for the same noise."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    from oracle import estimators as OE
    kB = 8.617333262e-5
    T, k1, k2 = 300.0, 2.0, 8.0
    reps = [I.Replica("bcc", 3, 3.0, T, k1, 100 + s, k2=k2) for s in range(32)]   # 54 atoms each
    ctx, x0, arrs = make_ctx(reps, FP64)
    n_eq, n_sw = 1500, 6000
    p = E.protocol("hh", n_eq, n_sw, n_eq, 0)
    S = n_eq * 2 + 2 * n_sw
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    v0 = E.from_soa(v)
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, S, None, None, W)
    Wg = W.cpu().numpy()
    Wf = Wg[:, n_eq + n_sw - 1]
    Wb = Wg[:, -1] - Wf
    dF, ediss, err = OE.forward_backward(Wf, Wb)
    N = reps[0].natoms
    exact = 1.5 * (N - 1) * kB * T * np.log(k2 / k1)
    assert abs(dF - exact) < 4 * err
    lam = oracle_lib.schedule("hh", n_eq, n_sw, n_eq, 0)
    for r in (0, 7, 31):
        _, _, _, Wo = _oracle_traj(oracle_lib, None, reps[r], reps[r].sites(), split(v0, ctx.offsets)[r], lam, "hh",
                                   True)
        assert np.abs(Wg[r] - Wo).max() < 1e-9
    ctx.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_overflow_replay_is_the_same_trajectory(prec):
    """Rows far too short for a dense crystal: run_switching detects the
    overflow, enlarges the lists, replays the chunk, and ends bit-identical
    to a run that had room from the start, with the replayed chunk's list
    work counted once."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 800.0, 5.0, 3), I.Replica("fcc", 5, I.A_FCC_STABLE, 800.0, 5.0, 4)]
    p = E.protocol("fl", 20, 60, 10, 10)
    out = []
    for cap in (32, 0):
        ctx, x0, arrs = make_ctx(reps, prec)
        ctx.set_chunk(40)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        if cap:
            with pytest.raises(E.EamfeError):
                ctx.neigh_build(x, 0.3, cap)
        else:
            ctx.neigh_build(x, 0.3, 0)
        W = torch.zeros(len(reps), 160, dtype=torch.float64, device="cuda")
        ctx.row_history(reset=True)
        ctx.run_switching(p, x, v, 0, 160, None, None, W)
        out.append((x.cpu().numpy(), v.cpu().numpy(), W.cpu().numpy(), ctx.replays(), ctx.list_stats(),
                    ctx.row_history()))
        ctx.close()
    assert out[0][3] > 0 and out[1][3] == 0
    assert out[0][4][2] >= out[0][4][1]
    assert out[0][5][1] == out[1][5][1] == 160 + 4   # one force pass per step plus one per chunk of 40
    assert out[0][5][0] == out[1][5][0]
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shift", [0.0, 13.7])
def test_neighbour_rows_match_brute_force(shift):
    """Every row holds exactly the atoms within r_cut + skin (FP64 brute force),
    up to the candidate test's widening margin, with no duplicates and no self."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()
    ctx, x0, arrs = make_ctx(reps, FP32, 8, 256)
    x = I.displaced(arrs["x0"], 0.3, seed=5) + shift
    xd = E.to_soa(x)
    skin = 0.3
    ctx.neigh_build(xd, skin, 0)
    nnb, nbr = ctx.copy_lists()
    nnb, nbr = nnb.cpu().numpy(), nbr.cpu().numpy()
    rl = I.R_CUT + skin
    for r, rep in enumerate(reps):
        o0, o1 = ctx.offsets[r], ctx.offsets[r + 1]
        xr = x[o0:o1]
        d = xr[:, None, :] - xr[None, :, :]
        d -= rep.box * np.rint(d / rep.box)
        dist = np.sqrt((d ** 2).sum(-1))
        np.fill_diagonal(dist, np.inf)
        for il in range(0, o1 - o0, 7):
            row = nbr[o0 + il, : nnb[o0 + il]] - o0
            assert len(set(row.tolist())) == len(row)
            assert il not in set(row.tolist())
            need = set(np.nonzero(dist[il] < rl - 1e-9)[0].tolist())
            assert need <= set(row.tolist()), (r, il)
            assert np.all(dist[il, row] < rl + 2e-3)
    ctx.close()


def test_row_history_weights_each_step_pass_by_its_rows():
    """The list-work history (mean row length over the step force passes)
    against the rows read back between one-step calls: a call over steps
    s..s+1 runs the force passes of iterations s and s+1, whose rows are the
    lists after the previous call and after this one.  A small skin makes the
    lists change during the run.  A chunked run counts one pass per step plus
    one per chunk."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    skin = 0.1
    p = E.protocol("fl", 20, 40, 0, 0, skin=skin)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, skin, 0)
    rows = [ctx.list_stats()[0]]
    ctx.row_history(reset=True)
    K = 30
    for s in range(K):
        ctx.run_switching(p, x, v, s, s + 1)
        rows.append(ctx.list_stats()[0])
    mean, passes = ctx.row_history(reset=True)
    assert passes == 2 * K
    want = sum(rows[k] + rows[k + 1] for k in range(K)) / (2 * K)
    assert abs(mean - want) <= 1e-12 * want, (mean, want)
    assert len(set(rows)) > 1   # the lists were rebuilt during the run
    ctx.set_chunk(7)
    ctx.run_switching(p, x, v, K, K + 30)
    mean2, passes2 = ctx.row_history()
    assert passes2 == 30 + 5 and min(rows) * 0.8 < mean2 < max(rows) * 1.2
    ctx.close()


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_resume_in_a_new_context_is_bitwise_the_straight_run(prec):
    """A run stopped at step 67, its state saved (x, v, work, list reference
    positions) and the context destroyed, then resumed in a new context,
    gives the positions, velocities and traces of the uninterrupted run bit
    for bit (a small skin makes the lists rebuild on both sides of the
    split)."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()[:4]
    skin, S, mid = 0.2, 150, 67
    p = E.protocol("fl", 10, 60, 10, 10, skin=skin)

    def start():
        ctx, x0, _ = make_ctx(reps, prec, 2, 256)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, skin, 0)
        return ctx, x, v

    ctx, x, v = start()
    dH = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    W = torch.zeros_like(dH)
    ctx.run_switching(p, x, v, 0, S, None, dH, W)
    ctx.close()

    ctx, xs, vs = start()
    dH1, W1 = torch.zeros_like(dH), torch.zeros_like(dH)
    ctx.run_switching(p, xs, vs, 0, mid, None, dH1, W1)
    Wm, xref, sk = ctx.get_state()
    assert sk == skin and np.array_equal(Wm, W1[:, mid - 1].cpu().numpy())
    xs, vs, xref = xs.clone(), vs.clone(), xref.clone()
    ctx.close()
    ctx, _, _ = make_ctx(reps, prec, 2, 256)
    ctx.set_state(Wm, xref, sk)
    ctx.run_switching(p, xs, vs, mid, S, None, dH1, W1)
    assert ctx.list_stats()[0] > 0
    ctx.close()
    assert torch.equal(xs, x) and torch.equal(vs, v)
    assert torch.equal(dH1, dH) and torch.equal(W1, W)


def test_list_rebuild_history_counts_the_rebuilding_passes():
    """With no skin every atom leaves its list's reference position each
    step.  A one-step call runs two force passes: the first at the positions
    its predecessor's last pass listed (nothing to rebuild), the second after
    the step (every replica rebuilt). K calls therefore rebuild K n_rep
    replica lists holding K N atoms, and a reset of the row history clears
    the count."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    p = E.protocol("fl", 20, 40, 0, 0, skin=0.0)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, 0.0, 0)
    ctx.row_history(reset=True)
    assert ctx.list_rebuilds() == (0, 0)
    K = 10
    for s in range(K):
        ctx.run_switching(p, x, v, s, s + 1)
    assert ctx.list_rebuilds() == (K * len(reps), K * ctx.N)
    ctx.row_history(reset=True)
    assert ctx.list_rebuilds() == (0, 0)
    ctx.close()


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_graph_replay_matches_eager(prec):
    """Middle iterations replayed from a captured graph give bit-identical
    trajectories and work traces; every replay is checked, with eager work
    and synchronisations between replays (several calls, several chunks)."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _mixed_batch()[:4]
    p = E.protocol("fl", 30, 80, 20, 30)
    S = 30 + 160 + 20 + 30
    cuts = [0, 37, 90, 91, 170, S]
    out = {}
    for graph in (0, 8):
        ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
        ctx.set_chunk(40)
        ctx.set_graph(graph)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
        snaps = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            ctx.run_switching(p, x, v, a, b, None, None, W)
            torch.cuda.synchronize()
            snaps.append((x.cpu().numpy().copy(), v.cpu().numpy().copy()))
            _ = (x * 2.0).sum().item()          # eager work between replays
        out[graph] = (snaps, W.cpu().numpy())
        ctx.close()
    for (xe, ve), (xg, vg) in zip(out[0][0], out[8][0]):
        assert np.array_equal(xe, xg) and np.array_equal(ve, vg)
    assert np.array_equal(out[0][1], out[8][1])
