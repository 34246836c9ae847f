"""Slabs with free surfaces on the GPU: forces and energies against the
oracle, and the surface excess free energy gamma = (F_surf - F_bulk) / A from
batched FL runs (the defect extension of the summary section), pinned at low
temperature by the oracle's relaxed static surface energy."""
import numpy as np
import pytest

from gpu_common import make_ctx, rel_norm, say, split
from paper_2201_04622_amd import inputs as I
from paper_2201_04622_amd import surfaces as S

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}
ETOL = {FP64: 1e-13, FP32: 1e-6}
A_HCP_STABLE = I.A_FCC_STABLE / np.sqrt(2.0)


def _slabs():
    return [
        S.slab(I.Replica("bcc", 0, I.A_BCC_STABLE, 300.0, 50.0, 51, cells=(6, 6, 6)), 8.0),
        S.slab(I.Replica("fcc", 0, I.A_FCC_STABLE, 300.0, 50.0, 52, cells=(5, 5, 5)), 7.0),
        S.slab(I.Replica("hcp", 0, A_HCP_STABLE, 300.0, 50.0, 53, cells=(7, 4, 4)), 9.0),
        I.Replica("bcc", 0, I.A_BCC_STABLE, 300.0, 50.0, 54, cells=(6, 6, 6)),
    ]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_slab_forces_and_energies(opot, prec):
    """Thermally displaced slabs (and a bulk replica in the same batch): the
    cells of the empty region hold no atoms, and the surface atoms' rows are
    short; forces and energies match the oracle to the usual bar."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _slabs()
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    x = I.displaced(arrs["x0"], 0.05, seed=23)
    xd = E.to_soa(x)
    ctx.neigh_build(xd, 0.3, 0)
    f = torch.zeros_like(xd)
    U = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
    ctx.eam_forces(xd, f, U)
    fg = E.from_soa(f)
    for r, (rep, fr, xr) in enumerate(zip(reps, split(fg, ctx.offsets), split(x, ctx.offsets))):
        o = opot.eam(xr, rep.box)
        say(f"{rep.kind} {rep.dims} vacuum {rep.vacuum}: force rel {rel_norm(fr, o['f']):.2e}, "
            f"U {U[r].item():.6f} vs {o['U']:.6f}")
        assert rel_norm(fr, o["f"]) <= TOL[prec], r
        assert abs(U[r].item() - o["U"]) <= ETOL[prec] * abs(o["U"]), r
    ctx.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_surface_free_energy_at_low_temperature_is_the_relaxed_surface_energy(opot, prec):
    """At 10 K the FL estimate of gamma for the bcc (001) slab must reproduce
    the oracle's 0 K relaxed surface energy (FIRE). Two effects separate them,
    each below 1e-3 of gamma: the surface's vibrational free energy, and the
    switching bias left at t_s = 8000 (the oracle's own runs at t_s = 2000 and
    8000 scale as 1 / t_s). Together they measured -0.10 %. The bar is 0.2 %
    plus three standard errors. A wrong area or a sign error in either F0
    would fail it, and so would the unrelaxed surface energy (+9.5 %)."""
    import torch  # noqa: F401

    from oracle.minimize import fire
    T, k = 10.0, 50.0
    bulk = [I.Replica("bcc", 0, I.A_BCC_STABLE, T, k, s, cells=(6, 6, 6)) for s in range(4)]
    slabs = [S.slab(I.Replica("bcc", 0, I.A_BCC_STABLE, T, k, 100 + s, cells=(6, 6, 6)), 8.0) for s in range(4)]
    reps = bulk + slabs
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    res = S.surface_free_energy(ctx, reps, x0, len(bulk), t_s=8000, n_eq=1000, n_hold=500, skin=0.3)
    ctx.close()

    x = bulk[0].sites()
    Ub = opot.eam(x, bulk[0].box)["U"]
    _, Us, _ = fire(opot, x, slabs[0].box, fmax=1e-6)
    g0 = (Us - Ub) / S.surface_area(slabs[0])
    say(f"prec {prec}: gamma {res.gamma:.6f} +- {res.gamma_err:.1e} eV/A^2 vs relaxed {g0:.6f}; "
        f"dissipation bulk {res.E_diss_bulk:.3f} slab {res.E_diss_slab:.3f} eV")
    assert res.area == pytest.approx(2.0 * bulk[0].box[0] * bulk[0].box[1])
    assert abs(res.gamma - g0) <= 2e-3 * g0 + 3.0 * res.gamma_err
    assert 0.0 < res.E_diss_slab < 2.0 and 0.0 < res.E_diss_bulk < 0.5


@pytest.mark.parametrize("kind,a,cells,vacuum", [
    ("fcc", I.A_FCC_STABLE, (5, 5, 5), 8.0),
    ("hcp", A_HCP_STABLE, (7, 4, 4), 9.0),
])
def test_other_faces_at_low_temperature(opot, kind, a, cells, vacuum):
    """The same check for the fcc (001) and hcp basal faces (FP32). The
    reference is the slab relaxed by FIRE from the sites plus a small seeded
    perturbation, so no symmetric saddle holds it."""
    from oracle.minimize import fire
    T, k = 10.0, 50.0
    bulk = [I.Replica(kind, 0, a, T, k, 200 + s, cells=cells) for s in range(4)]
    slabs = [S.slab(I.Replica(kind, 0, a, T, k, 300 + s, cells=cells), vacuum) for s in range(4)]
    reps = bulk + slabs
    ctx, x0, _ = make_ctx(reps, FP32, 2, 256)
    res = S.surface_free_energy(ctx, reps, x0, len(bulk), t_s=8000, n_eq=1000, n_hold=500, skin=0.3)
    ctx.close()
    x = bulk[0].sites()
    Ub = opot.eam(x, bulk[0].box)["U"]
    _, Us, _ = fire(opot, x + 0.01 * np.random.default_rng(2).standard_normal(x.shape), slabs[0].box, fmax=1e-6,
                    max_steps=100000)
    g0 = (Us - Ub) / S.surface_area(slabs[0])
    say(f"{kind}: gamma {res.gamma:.6f} +- {res.gamma_err:.1e} eV/A^2 vs relaxed {g0:.6f} "
        f"({(res.gamma / g0 - 1) * 100:+.3f} %); dissipation slab {res.E_diss_slab:.3f} eV")
    assert abs(res.gamma - g0) <= 2e-3 * g0 + 3.0 * res.gamma_err
