"""Frenkel--Ladd against reversible scaling at fixed volume: the paper's own
consistency check, FL points falling on the RS curve F(T) (Sec. results).

bcc 6^3 at the synthetic potential's zero-pressure lattice parameter (fixed
box), T0 = 300 K: F0(T0) from FL starts an RS scan up to 1200 K
(lambda_f = 1/4, Eq. rs in its fixed-centre-of-mass form, since both paths
hold the centre of mass); independent FL runs at 600, 900 and 1200 K must
agree with the RS curve within 0.5 meV/atom and three combined standard
errors."""
import numpy as np
import pytest

from gpu_common import make_ctx, say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP32 = 1
CELLS = (6, 6, 6)
K = 20.0


def _fl_per_atom(T, seeds, t_s=32000, n_eq=2000, n_hold=2000):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 0, I.A_BCC_STABLE, T, K, s, cells=CELLS) for s in seeds]
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
    N = reps[0].natoms
    V = float(np.prod(reps[0].box))
    return np.array([E.fl_free_energy(Wf[r:r + 1], Wb[r:r + 1], N, T, K, reps[0].mass, N=N, V=V)[0]
                     for r in range(len(reps))]) / N


def test_fl_points_lie_on_the_rs_curve():
    import torch

    import paper_2201_04622_amd.eamfe as E
    T0, Tf, checks = 300.0, 1200.0, (600.0, 900.0, 1200.0)
    f0 = _fl_per_atom(T0, range(8))
    reps = [I.Replica("bcc", 0, I.A_BCC_STABLE, T0, K, 500 + s, cells=CELLS) for s in range(8)]
    N = reps[0].natoms
    ctx, x0, _ = make_ctx(reps, FP32, 2, 256)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    n_eq, n_sw, n_hold = 2000, 80000, 2000   # at 40000 steps the RS bias reaches 0.2 meV/atom at 1200 K
    p = E.protocol("rs", n_eq, n_sw, n_hold, 0, lambda_f=T0 / Tf, skin=0.3)
    S = n_eq + 2 * n_sw + n_hold
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, S, W_out=W)
    ctx.close()
    W = W.cpu().numpy()
    F0 = f0.mean() * N
    grid = np.array(checks)
    V = float(np.prod(reps[0].box))
    F = np.array([E.rs_free_energy_cm(p, W[r], F0, T0, N, V, reps[0].mass, grid) for r in range(len(reps))]) / N
    for q, T in enumerate(checks):
        fl = _fl_per_atom(T, range(100 * q + 100, 100 * q + 108))
        lam = T0 / T
        # the RS value inherits F0(T0) / lambda, so its error carries that factor
        se_rs = np.hypot(F[:, q].std(ddof=1) / np.sqrt(len(F)), f0.std(ddof=1) / np.sqrt(len(f0)) / lam)
        se_fl = fl.std(ddof=1) / np.sqrt(len(fl))
        d = F[:, q].mean() - fl.mean()
        say(f"T {T:.0f} K: RS {F[:, q].mean():.6f} +- {se_rs:.1e}, FL {fl.mean():.6f} +- {se_fl:.1e} eV/atom, "
            f"diff {d * 1e3:+.4f} meV/atom")
        assert abs(d) < 5e-4 and abs(d) < 3.0 * np.hypot(se_rs, se_fl) + 2e-5, (T, d)
