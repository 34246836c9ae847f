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
