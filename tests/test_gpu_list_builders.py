"""The two neighbour-list builders give the same lists: rows built from LDS
(replicas of at most 4096 atoms) equal those of the global-memory binning
and row kernels slot for slot, on all-pairs boxes, cell boxes, verbatim
crystals that densify and a mix with replicas too large for LDS; and a
switching run gives bitwise the same trajectory, work and list statistics
with either builder."""
import numpy as np
import pytest

from gpu_common import make_ctx, say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


def _mixed():
    return [I.Replica("bcc", 4, I.A_BCC_VERBATIM, 300.0, 5.0, 1),            # 128 atoms, all-pairs rows
            I.Replica("fcc", 5, I.A_FCC_STABLE, 900.0, 5.0, 2),              # cells
            I.Replica("bcc", 12, I.A_BCC_VERBATIM, 1600.0, 5.0, 3),          # 3456 atoms, 11^3 cells
            I.Replica("fcc", 10, I.A_FCC_VERBATIM, 1200.0, 5.0, 4),          # 4000 atoms
            I.Replica("bcc", 14, I.A_BCC_STABLE, 600.0, 5.0, 5)]             # 5488 atoms: global builder


def _rows(ctx, x):
    ctx.neigh_build(x, 0.3, 0)     # the 128-atom box (11.42 A) takes 0.3 A of skin, and gets all-pairs rows
    nnb, nbr = ctx.copy_lists()
    return nnb.cpu().numpy(), nbr.cpu().numpy()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_builders_give_identical_rows(prec):
    import paper_2201_04622_amd.eamfe as E
    reps = _mixed()
    ctx, x0, arrs = make_ctx(reps, prec, 2, 256)
    for seed, sigma in ((7, 0.05), (8, 0.4)):      # thermal and strongly disordered positions
        x = E.to_soa(I.displaced(arrs["x0"], sigma, seed=seed))
        ctx.set_list_builder(True)
        a = _rows(ctx, x)
        ctx.set_list_builder(False)
        b = _rows(ctx, x)
        say(f"sigma {sigma}: mean row {a[0].mean():.1f}, max {a[0].max()}")
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[1], b[1])
    ctx.close()


def test_builders_give_bitwise_the_same_run():
    import torch

    import paper_2201_04622_amd.eamfe as E
    wl = I.workload("batch64")
    reps = wl.replicas[:16] + [I.Replica("bcc", 14, I.A_BCC_VERBATIM, 800.0, 5.0, 99)]
    out = []
    for lds in (True, False):
        ctx, x0, _ = make_ctx(reps, FP32, 2, 1024)
        ctx.set_list_builder(lds)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, 0.65, 0)
        p = E.protocol("fl", 300, 600, 100, 0, skin=0.65)
        W = torch.zeros(len(reps), 1600, dtype=torch.float64, device="cuda")
        ctx.row_history(reset=True)
        ctx.run_switching(p, x, v, 0, 1600, W_out=W)
        out.append((x.cpu().numpy(), v.cpu().numpy(), W.cpu().numpy(), ctx.row_history(), ctx.list_rebuilds()))
        ctx.close()
    say(f"rebuilds {out[0][4]} vs {out[1][4]}, rows {out[0][3]}")
    assert out[0][4][0] > 0
    for qa, qb in zip(out[0], out[1]):
        assert np.array_equal(np.asarray(qa), np.asarray(qb))


def test_autotune_keeps_the_trajectory():
    # the tuner times launch shapes and both builders on copies of the state and
    # builds the lists again at the caller's positions before it returns; the
    # deterministic FP32 form gives the same bits for every shape and builder,
    # so the tuned run is bitwise the untuned one with its lists rebuilt at the
    # same step (the float32 slot groups follow the rows), and the tuned
    # context's first pass rebuilds no list
    import torch

    import paper_2201_04622_amd.eamfe as E
    wl = I.workload("batch64")
    reps = wl.replicas[:8] + [I.Replica("bcc", 14, I.A_BCC_VERBATIM, 800.0, 5.0, 99)]
    p = E.protocol("fl", 300, 600, 100, 0, skin=0.65)
    out = []
    for tune in (False, True):
        ctx, x0, _ = make_ctx(reps, FP32, 2, 1024)
        x = x0.clone()
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, 0.65, 0)
        W = torch.zeros(len(reps), 1600, dtype=torch.float64, device="cuda")   # [n_rep][S], S = 1600
        ctx.run_switching(p, x, v, 0, 300, W_out=W)
        if tune:
            xs, vs = x.clone(), v.clone()
            tuned = ctx.autotune(p, 300, x, v, trial_steps=4)
            assert torch.equal(x, xs) and torch.equal(v, vs)
            say(f"tuned {tuned}, builder {ctx.get_list_builder()}")
            assert ctx.get_list_builder() in ("lds", "global")
        else:
            ctx.neigh_build(x, 0.65, 0)
        ctx.row_history(reset=True)
        ctx.run_switching(p, x, v, 300, 301)
        # one step from freshly built lists: no replica moved half a skin
        assert ctx.list_rebuilds()[0] == 0
        ctx.run_switching(p, x, v, 301, 600, W_out=W)
        out.append((x.cpu().numpy(), v.cpu().numpy(), W.cpu().numpy()))
        ctx.close()
    for qa, qb in zip(out[0], out[1]):
        assert np.array_equal(qa, qb)


@pytest.mark.parametrize("det", [True, False])
def test_trajectory_across_launch_shapes(det):
    # deterministic form: the replica sums (noise mean, energies, work) are exact,
    # so a run is bitwise the same for every lanes per atom; the plain form adds
    # them in unit order and agrees to round-off, grown by the chaotic dynamics
    import torch

    import paper_2201_04622_amd.eamfe as E
    from gpu_common import rel_norm
    wl = I.workload("batch64")
    reps = wl.replicas[:8]
    # 500 steps of a 600-step switch: a faster switch heats the crystal until
    # atoms held only by the springs at lambda = 1 overlap past the tables
    p = E.protocol("fl", 300, 600, 100, 0, skin=0.65)
    arrs = I.batch_arrays(reps)
    out = []
    for lanes, block in ((1, 256), (2, 1024), (4, 512), (16, 1024)):
        ctx = E.Context(0, E.FP32, deterministic=det)
        ctx.set_launch(lanes, block)
        ctx.eam_setup(I.synthetic_eam_knots())
        x = E.to_soa(arrs["x0"])
        ctx.system_setup(reps, x)
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, 0.65, 0)
        W = torch.zeros(len(reps), 1600, dtype=torch.float64, device="cuda")
        ctx.run_switching(p, x, v, 0, 500, W_out=W)
        out.append((x.cpu().numpy(), v.cpu().numpy(), W.cpu().numpy()))
        ctx.close()
    for q in out[1:]:
        if det:
            for qa, qb in zip(out[0], q):
                assert np.array_equal(qa, qb)
        else:
            assert rel_norm(q[0], out[0][0]) < 1e-6
