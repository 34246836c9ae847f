"""Spline tables as large as one block's LDS holds, through the C ABI.

The FP32 pair kernels keep the pair table and the density-derivative table
in one block's LDS (16 bytes per interval each, plus one padding interval
per table), and the adjoint keeps four fixed-point words per interval there.
A gfx950 block may take 160 KiB, so FP32 takes at most 5120 knots and the
adjoint at most 5121.

* At those sizes, FP32 forces and energies follow the oracle's tables of
  the same knots. The FP64 adjoint keeps the exact identities of the EAM
  energy.
* One knot more is refused with EAMFE_EINVAL before any kernel runs (an
  adjoint call, or a switching run that samples the adjoint), and the
  context keeps the tables it had.
* FP64 stepping reads its tables from global memory and takes the larger
  table."""
import numpy as np
import pytest

from gpu_common import make_ctx, rel_norm, say, split
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
LDS_BLOCK = 160 * 1024
FP32_KNOTS = LDS_BLOCK // 32          # two tables of 16-byte intervals, padding included
ADJOINT_KNOTS = LDS_BLOCK // 32 + 1   # 32 bytes per interval


def _reps():
    return [I.Replica("bcc", 4, I.A_BCC_VERBATIM, 300.0, 5.0, 7),   # 128 atoms, all-pairs rows
            I.Replica("fcc", 5, I.A_FCC_VERBATIM, 600.0, 5.0, 8)]   # 500 atoms, cell lists


def _forces(ctx, xd, n_rep):
    import torch

    import paper_2201_04622_amd.eamfe as E
    f = torch.zeros_like(xd)
    U = torch.zeros(n_rep, dtype=torch.float64, device="cuda")
    ctx.eam_forces(xd, f, U)
    return E.from_soa(f), U.cpu().numpy()


def _check_forces(opot, reps, x, ctx, fg, U, ftol, etol):
    for r, (rep, xr, fr) in enumerate(zip(reps, split(x, ctx.offsets), split(fg, ctx.offsets))):
        o = opot.eam(xr, rep.box)
        assert rel_norm(fr, o["f"]) <= ftol, (r, rel_norm(fr, o["f"]))
        assert abs(U[r] - o["U"]) <= etol * abs(o["U"]), (r, U[r], o["U"])


def test_fp32_at_the_largest_table_and_one_knot_more(oracle_lib):
    import paper_2201_04622_amd.eamfe as E
    say(f"FP32 tables of {FP32_KNOTS} knots, then {FP32_KNOTS + 1}")
    knots = I.synthetic_eam_knots(FP32_KNOTS)
    opot = oracle_lib.Potential.from_knots(knots)
    reps = _reps()
    ctx, x0, arrs = make_ctx(reps, FP32, 2, 256, knots=knots)
    x = I.displaced(arrs["x0"], 0.05, seed=21)
    xd = E.to_soa(x)
    ctx.neigh_build(xd, 0.3, 0)
    fg, U = _forces(ctx, xd, len(reps))
    _check_forces(opot, reps, x, ctx, fg, U, 1e-5, 1e-6)
    with pytest.raises(E.EamfeError) as err:
        ctx.eam_setup(I.synthetic_eam_knots(FP32_KNOTS + 1))
    assert err.value.code == 1 and "LDS" in str(err.value), err.value   # EAMFE_EINVAL
    # the context keeps the tables it had: the same forces, bit for bit
    fg2, U2 = _forces(ctx, xd, len(reps))
    assert np.array_equal(fg2, fg) and np.array_equal(U2, U)
    ctx.close()


def test_fp64_takes_larger_tables_and_the_adjoint_stops_at_its_limit(oracle_lib):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = _reps()
    # one knot beyond the adjoint's limit: FP64 forces still follow the oracle,
    # the adjoint is refused before any kernel runs
    n = ADJOINT_KNOTS + 1
    say(f"FP64 tables of {n} knots: forces, adjoint refused")
    knots = I.synthetic_eam_knots(n)
    opot = oracle_lib.Potential.from_knots(knots)
    ctx, x0, arrs = make_ctx(reps, FP64, 4, 256, knots=knots)
    x = I.displaced(arrs["x0"], 0.05, seed=22)
    xd = E.to_soa(x)
    ctx.neigh_build(xd, 0.3, 0)
    fg, U = _forces(ctx, xd, len(reps))
    _check_forces(opot, reps, x, ctx, fg, U, 1e-12, 1e-13)
    g = torch.zeros(len(reps), 3, n, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EamfeError) as err:
        ctx.adjoint_theta(xd, g)
    assert err.value.code == 1 and "LDS" in str(err.value), err.value
    assert not g.any().item()   # nothing ran
    # a switching run that samples the adjoint is refused before its first step
    p = E.protocol("fl", n_eq=2, n_sw=2, n_hold=1, n_hold2=1)
    v = torch.zeros_like(xd)
    ctx.init_velocities(v, True)
    xs, vs = xd.clone(), v.clone()
    ctx.set_adjoint_sampling(1, g)
    with pytest.raises(E.EamfeError) as err:
        ctx.run_switching(p, xs, vs, 0, 2 + 4 + 1 + 1)
    assert err.value.code == 1 and "LDS" in str(err.value), err.value
    assert torch.equal(xs, xd) and torch.equal(vs, v) and not g.any().item()
    assert ctx.adjoint_samples() == 0
    ctx.set_adjoint_sampling(0)
    # at the limit the adjoint runs and keeps the energy's exact identities
    n = ADJOINT_KNOTS
    say(f"FP64 adjoint with tables of {n} knots")
    knots = I.synthetic_eam_knots(n)
    ctx.eam_setup(knots)
    g = torch.zeros(len(reps), 3, n, dtype=torch.float64, device="cuda")
    ctx.adjoint_theta(xd, g)
    _, U = _forces(ctx, xd, len(reps))
    gg = g.cpu().numpy()
    for r, rep in enumerate(reps):
        # raising every F knot by c raises U by N c (a natural spline keeps constants)
        assert gg[r, 2].sum() == pytest.approx(rep.natoms, rel=1e-11)
        # U is homogeneous of degree one in the (phi, F) knots together
        assert knots.phi @ gg[r, 0] + knots.embed @ gg[r, 2] == pytest.approx(U[r], rel=1e-11)
    ctx.close()


def test_fp64_tables_from_lds_or_global_memory_give_the_same_bits():
    """The FP64 pair kernels read their tables from LDS in a launch of at
    least two units per compute unit and from global memory otherwise.  The
    same replicas at the same lanes, alone (a small launch) and beside filler
    replicas (a large one), give the same forces and energies bit for bit:
    a replica's arithmetic and its order do not depend on where the table
    sits or on the other replicas."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    lanes, per_unit = 8, 64 // 8
    reps = _reps() + [I.Replica("bcc", 7, I.A_BCC_VERBATIM, 900.0, 5.0, 9)]   # 128 + 500 + 686 atoms
    units = sum(-(-r.natoms // per_unit) for r in reps)
    limit = 2 * torch.cuda.get_device_properties(0).multi_processor_count
    assert units < limit   # alone: global tables
    filler = []
    while units + sum(-(-r.natoms // per_unit) for r in filler) < limit:
        filler.append(I.Replica("fcc", 6, I.A_FCC_VERBATIM, 600.0, 5.0, 20 + len(filler)))
    say(f"FP64 tables: {units} units alone, {units + sum(-(-r.natoms // per_unit) for r in filler)} with "
        f"{len(filler)} filler replicas (LDS from {limit})")
    x_reps = I.displaced(I.batch_arrays(reps)["x0"], 0.05, seed=23)
    x_fill = I.displaced(I.batch_arrays(filler)["x0"], 0.05, seed=24)
    out = []
    for batch, x in ((reps, x_reps), (reps + filler, np.concatenate([x_reps, x_fill]))):
        ctx, x0, arrs = make_ctx(batch, FP64, lanes, 256)
        xd = E.to_soa(x)
        ctx.neigh_build(xd, 0.3, 0)
        f, U = _forces(ctx, xd, len(batch))
        out.append((f[: len(x_reps)], U[: len(reps)]))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
