"""dU/dtheta on the GPU through the C ABI (theta = knot values of phi, rho, F):
parity with the oracle's brute-force transpose, exact identities of the EAM
energy, finite differences of GPU energies, weighted reduction, sampling
inside run_switching, and the torch.autograd.Function."""
import numpy as np
import pytest

from gpu_common import make_ctx, say, split
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


def _batch():
    return [I.Replica("bcc", 4, I.A_BCC_VERBATIM, 300.0, 5.0, 1),   # all-pairs lists
            I.Replica("fcc", 5, I.A_FCC_STABLE, 900.0, 5.0, 2),     # cell lists, dense
            I.Replica("bcc", 6, I.A_BCC_VERBATIM, 600.0, 5.0, 3)]


# FP32: pair geometry is float64 in the adjoint, but rho_i and F'(rho_i) come from the
# single-precision density pass.  In the dense crystal (rho ~ 77, |drho/dr| ~ 15 per A at
# the first shell) each FP32 pair term is off by ~5e-6, rho_i by ~6e-5 over ~140 pairs,
# i.e. ~1e-3 of an F interval (width 0.1): the F-knot gradient inherits ~1e-4.
@pytest.mark.parametrize("prec,tol", [(FP64, (1e-9, 1e-9, 1e-9)), (FP32, (2e-6, 1e-5, 5e-4))])
def test_adjoint_matches_oracle(opot, prec, tol):
    import torch

    import paper_2201_04622_amd.eamfe as E
    say(f"adjoint vs oracle prec={prec}")
    reps = _batch()
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    x = I.displaced(arrs["x0"], 0.07, seed=13)
    xd = E.to_soa(x)
    n = I.N_KNOTS
    g = torch.zeros(len(reps), 3, n, dtype=torch.float64, device="cuda")
    ctx.adjoint_theta(xd, g)
    gg = g.cpu().numpy()
    for r, (rep, xr) in enumerate(zip(reps, split(x, ctx.offsets))):
        ref = opot.adjoint_theta(xr, rep.box)
        for f in range(3):
            err = np.linalg.norm(gg[r, f] - ref[f]) / np.linalg.norm(ref[f])
            assert err < tol[f], (r, f, err)
    ctx.close()


def test_adjoint_identities_and_reduction(knots):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _batch()
    ctx, x0, arrs = make_ctx(reps, FP64)
    xd = E.to_soa(I.displaced(arrs["x0"], 0.05, seed=2))
    n = I.N_KNOTS
    g = torch.zeros(len(reps), 3, n, dtype=torch.float64, device="cuda")
    ctx.adjoint_theta(xd, g)
    U = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
    ctx.eam_forces(xd, None, U)
    gg, U = g.cpu().numpy(), U.cpu().numpy()
    for r, rep in enumerate(reps):
        # a natural spline reproduces constants: raising every F knot by c raises U by N c
        assert gg[r, 2].sum() == pytest.approx(rep.natoms, rel=1e-11)
        # U is homogeneous of degree one in the (phi, F) knots together
        assert knots.phi @ gg[r, 0] + knots.embed @ gg[r, 2] == pytest.approx(U[r], rel=1e-11)
    w = np.array([0.5, -2.0, 3.0])
    red = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    ctx.adjoint_theta(xd, red, weights=w, reduce=True)
    assert np.allclose(red.cpu().numpy(), np.tensordot(w, gg, axes=1), rtol=1e-12, atol=1e-9)
    ctx.close()


def test_adjoint_matches_gpu_energy_differences(knots):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("fcc", 5, I.A_FCC_VERBATIM, 600.0, 5.0, 2)]
    ctx, x0, arrs = make_ctx(reps, FP64)
    xd = E.to_soa(I.displaced(arrs["x0"], 0.06, seed=9))
    g = torch.zeros(1, 3, I.N_KNOTS, dtype=torch.float64, device="cuda")
    ctx.adjoint_theta(xd, g)
    g = g.cpu().numpy()[0]
    U = torch.zeros(1, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(4)
    hr = knots.r_cut / (knots.n - 1)
    for f, lo, hi, h in ((0, int(2.0 / hr), knots.n - 1, 1e-3), (1, int(2.0 / hr), knots.n - 1, 1e-5),
                         (2, 40, 60, 1e-3)):
        for k in rng.integers(lo, hi, 3):
            vals = []
            for sgn in (1, -1):
                th = knots.stacked().copy()
                th[f, k] += sgn * h
                ctx.eam_setup(I.PotentialKnots(knots.r_cut, knots.rho_max, th[0], th[1], th[2]))
                ctx.eam_forces(xd, None, U)
                vals.append(U.item())
            fd = (vals[0] - vals[1]) / (2 * h)
            assert g[f, k] == pytest.approx(fd, rel=1e-6, abs=1e-7), (f, k)
    ctx.close()


def test_adjoint_sampling_during_switching():
    """Sampling inside run_switching equals explicit calls at the same states."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _batch()[1:]
    n = I.N_KNOTS
    p = E.protocol("fl", n_eq=4, n_sw=6, n_hold=2, n_hold2=3)
    S = 4 + 12 + 2 + 3
    # sampled run
    ctx, x0, arrs = make_ctx(reps, FP64)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    acc = torch.zeros(len(reps), 3, n, dtype=torch.float64, device="cuda")
    ctx.set_adjoint_sampling(2, acc)
    ctx.run_switching(p, x, v, 0, S)
    samples = ctx.adjoint_samples()
    ctx.set_adjoint_sampling(0)
    ctx.close()
    # explicit: step by step, adjoint where lambda = 0 and s % 2 == 0
    lam = E.lambda_schedule(p)
    ctx, x0, arrs = make_ctx(reps, FP64)
    x = x0.clone()
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ref = torch.zeros_like(acc)
    W = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
    count = 0
    for s in range(S):
        if s % 2 == 0 and lam[s] == 0.0:
            ctx.adjoint_theta(x, ref)
            count += 1
        ctx.switch_step(p, s, x, v, W)
    ctx.close()
    assert samples == count == 5
    assert np.allclose(acc.cpu().numpy(), ref.cpu().numpy(), rtol=1e-10, atol=1e-8)


def test_autograd_function(knots):
    import torch

    import paper_2201_04622_amd.eamfe as E
    from paper_2201_04622_amd.autograd import EAMEnergy
    reps = _batch()
    ctx, x0, arrs = make_ctx(reps, FP64)
    xd = E.to_soa(I.displaced(arrs["x0"], 0.05, seed=3)).requires_grad_(True)
    theta = torch.tensor(knots.stacked(), dtype=torch.float64, requires_grad=True)
    w = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda")
    U = EAMEnergy.apply(theta, xd, ctx, knots.r_cut, knots.rho_max)
    (U * w).sum().backward()
    # dx: forces
    f = torch.zeros_like(xd)
    ctx.eam_forces(xd.detach(), f, None)
    wa = torch.repeat_interleave(w, torch.as_tensor(np.diff(ctx.offsets), device="cuda"))
    assert torch.allclose(xd.grad, -f * wa[None, :], rtol=1e-12, atol=1e-12)
    # dtheta: weighted per-replica adjoints
    g = torch.zeros(len(reps), 3, I.N_KNOTS, dtype=torch.float64, device="cuda")
    ctx.adjoint_theta(xd.detach(), g)
    ref = (g * w[:, None, None]).sum(0).cpu()
    assert torch.allclose(theta.grad, ref, rtol=1e-10, atol=1e-8)
    ctx.close()


def test_autograd_two_applies_on_one_context(knots):
    """Two applies at different theta on one context before one backward
    (a finite difference U(theta) - U(theta + h u) as a graph): each node's
    dU/dtheta must be taken with its own tables, as on a fresh context each,
    and the difference quotient of the energies must match the projected
    gradient."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    from paper_2201_04622_amd.autograd import EAMEnergy
    reps = _batch()
    base = torch.tensor(knots.stacked(), dtype=torch.float64)
    u = torch.zeros_like(base)
    u[1] = torch.linspace(0.0, 1.0, base.shape[1]) * 0.02   # a smooth change of the rho knots
    u[2] = torch.linspace(0.0, 1.0, base.shape[1]) * 0.05   # and of the F knots
    h = 1e-3
    ctx, x0, arrs = make_ctx(reps, FP64)
    xd = E.to_soa(I.displaced(arrs["x0"], 0.05, seed=3))
    t1 = base.clone().requires_grad_(True)
    t2 = (base + h * u).requires_grad_(True)
    w = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda")
    U1 = EAMEnergy.apply(t1, xd, ctx, knots.r_cut, knots.rho_max)
    U2 = EAMEnergy.apply(t2, xd, ctx, knots.r_cut, knots.rho_max)
    ((U2 - U1) * w).sum().backward()
    ctx.close()
    for t, sign in ((t1, -1.0), (t2, 1.0)):
        c2, _, _ = make_ctx(reps, FP64)
        t_ref = t.detach().clone().requires_grad_(True)
        U = EAMEnergy.apply(t_ref, xd, c2, knots.r_cut, knots.rho_max)
        (sign * U * w).sum().backward()
        c2.close()
        assert torch.allclose(t.grad, t_ref.grad, rtol=1e-12, atol=1e-10)
    # central difference along u against the mean of the two gradients
    fd = float(((U2 - U1) * w).sum().detach()) / h
    proj = 0.5 * float(((-t1.grad + t2.grad) * u).sum())
    say(f"two applies: FD {fd:.8e}, adjoint projection {proj:.8e}")
    assert abs(fd - proj) < 1e-6 * abs(fd) + 1e-9
