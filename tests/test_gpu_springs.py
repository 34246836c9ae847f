"""Spring constants from the mean-squared displacement (Eq. msd) on the GPU."""
import numpy as np
import pytest

from gpu_common import make_ctx, say, split
from oracle import estimators as OE
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP32 = 1


def test_msd_matches_oracle():
    """eamfe_msd against the oracle's MSD per replica, on displaced and
    rigidly shifted positions of uneven replicas."""
    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 1), I.Replica("fcc", 5, I.A_FCC_VERBATIM, 600.0, 5.0, 2),
            I.Replica("bcc", 9, I.A_BCC_VERBATIM, 100.0, 5.0, 3)]
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    off = ctx.offsets
    x = I.displaced(arrs["x0"], 0.15, seed=9)
    x[off[1]:off[2]] += np.array([0.7, -0.2, 1.1])   # a replica's rigid shift is not displacement
    got = ctx.msd(E.to_soa(x))
    want = [OE.msd_com_removed(a, b) for a, b in zip(split(x, off), split(arrs["x0"], off))]
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    ctx.close()


def test_einstein_crystal_gives_back_its_spring_constant():
    """In an Einstein crystal (the lambda = 0 end of the harmonic test path)
    equipartition fixes <(dr)^2> = 3 kB T / k per internal degree of freedom;
    with the centre of mass held fixed, N - 1 of N atoms' worth remain, so the
    MSD route must return k N / (N - 1)."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    import paper_2201_04622_amd.springs as SP
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, T, k, 20 + q)
            for q, (T, k) in enumerate([(300.0, 5.0), (800.0, 5.0), (300.0, 2.0), (1200.0, 8.0)])]
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    k, msd, n = SP.spring_constants(ctx, reps, x, v, 20000, 100, mode="hh", discard=2000)
    N = reps[0].natoms
    for r, kr in zip(reps, k):
        say(f"T {r.T} k {r.k}: MSD route {kr:.4f}, expected {r.k * N / (N - 1):.4f} ({n} samples)")
        assert kr == pytest.approx(r.k * N / (N - 1), rel=0.03)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_per_atom_springs_follow_the_oracle(oracle_lib, opot, prec):
    """FL switching with two species of springs (atom i's spring k s_i) on
    uneven replicas follows the oracle step by step: positions, dH/dl and W;
    clearing the scales gives back the uniform-spring run bit for bit."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 600.0, 5.0, 31), I.Replica("fcc", 5, I.A_FCC_VERBATIM, 300.0, 4.0, 32)]
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    N = x0.shape[1]
    scale = np.where(np.arange(N) % 3 == 0, 2.5, 1.0)
    n_eq, n_sw, n_hold, n_hold2 = 6, 20, 4, 4
    p = E.protocol("fl", n_eq, n_sw, n_hold, n_hold2, function=2)
    S = n_eq + 2 * n_sw + n_hold + n_hold2

    def run(with_scale):
        ctx.set_spring_scale(torch.as_tensor(scale, device="cuda") if with_scale else None)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        vi = E.from_soa(v)
        dH = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
        W = torch.zeros_like(dH)
        ctx.run_switching(p, x, v, 0, S, None, dH, W)
        return E.from_soa(x), vi, dH.cpu().numpy(), W.cpu().numpy()

    xs, vi, dHs, Ws = run(True)
    lam = oracle_lib.schedule("fl", n_eq, n_sw, n_hold, n_hold2, function=2)
    tol = 1e-9 if prec == 0 else 2e-3
    off = ctx.offsets
    for r, rep in enumerate(reps):
        prm = oracle_lib.RunParams(mode="fl", T=rep.T, k=rep.k, seed=rep.seed, fix_com=True, mass=rep.mass)
        xo, vo = rep.sites().copy(), vi[off[r]:off[r + 1]].copy()
        dHo, Wo, _, _ = oracle_lib.run(opot, prm, rep.sites(), rep.box, xo, vo, lam, spring_scale=scale[off[r]:off[r + 1]])
        sc = max(1.0, np.abs(dHo).max())
        say(f"{rep.kind}: max|dx| {np.abs(xs[off[r]:off[r + 1]] - xo).max():.2e}, max|dW| {np.abs(Ws[r] - Wo).max():.2e}")
        assert np.abs(xs[off[r]:off[r + 1]] - xo).max() < tol
        assert np.abs(dHs[r] - dHo).max() < tol * sc and np.abs(Ws[r] - Wo).max() < tol * sc
    x1, _, _, W1 = run(False)
    x2, _, _, W2 = run(False)
    assert np.array_equal(x1, x2) and np.array_equal(W1, W2)
    assert not np.array_equal(W1, Ws)
    ctx.close()
