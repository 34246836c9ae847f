"""The switching-time sweep (Sec. p_fl, Fig. fl_convergence) on the GPU:
8 realizations of a stable bcc crystal, three switching times."""
import numpy as np
import pytest

from gpu_common import make_ctx, say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP32 = 1


def test_fl_sweep_converges_and_bounds_hold():
    """The paper's workflow on 8 realizations of a stable bcc crystal: the
    spring constant from the mean-squared displacement (Eq. msd), then FL
    switching at three switching times.  As t_s grows the dissipation (Eq.
    Ediss) falls and the two-way F0 (Eq. fl) settles; at every t_s the
    one-way estimates keep their order: F_E - mean W_fwd <= Jarzynski forward
    and Jarzynski backward <= F_E + mean W_bwd (the exponential average never
    exceeds the mean), and the two-way F0 is the mean of the two one-way means."""
    import torch

    import paper_2201_04622_amd.convergence as CV
    import paper_2201_04622_amd.springs as SP

    T = 300.0
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, T, 5.0, 100 + s) for s in range(8)]
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, 0.3, 0)
    kr, msd, n = SP.spring_constants(ctx, reps, x, v, 6000, 50, mode="fl", discard=1000)
    k = float(np.round(kr.mean(), 2))
    say(f"spring constant from the MSD: {k} eV/A^2 (replicas {np.round(kr, 3)})")
    ctx.close()

    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, T, k, 100 + s) for s in range(8)]
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256)
    N = reps[0].natoms
    pts = CV.fl_sweep(ctx, reps, x0, [500, 2000, 8000], n_eq=1000, n_hold=200)
    for q in pts:
        say(f"t_s {q.t_s}: F0 {q.F0_w12 / N:.6f} +- {q.F0_w12_err / N:.2e} eV/atom, E_diss {q.E_diss / N * 1e3:.4f} meV/atom, "
            f"Jarzynski fwd {q.F0_jarz_fwd / N:.6f} bwd {q.F0_jarz_bwd / N:.6f}")
        assert np.isfinite([q.F0_w12, q.E_diss, q.F0_jarz_fwd, q.F0_jarz_bwd]).all()
        assert q.F0_mean_fwd <= q.F0_jarz_fwd + 1e-9 and q.F0_jarz_bwd <= q.F0_mean_bwd + 1e-9
        assert q.F0_w12 == pytest.approx(0.5 * (q.F0_mean_fwd + q.F0_mean_bwd), abs=1e-9 * abs(q.F0_w12))
    Ed = [q.E_diss for q in pts]
    assert Ed[0] > Ed[1] > Ed[2] > 0.0
    a, b = pts[1], pts[2]
    tol = 3.0 * np.hypot(a.F0_w12_err, b.F0_w12_err) + 0.5e-3 * N
    assert abs(a.F0_w12 - b.F0_w12) <= tol, (a.F0_w12 / N, b.F0_w12 / N, tol / N)
    # the one-way biases shrink with the dissipation
    assert b.F0_w12 - b.F0_mean_fwd < pts[0].F0_w12 - pts[0].F0_mean_fwd
    ctx.close()
