"""The ownership contract of the C ABI on the GPU: with a caller's workspace
(the binding's default, one torch tensor) the library allocates no device
memory, a list overflow in the middle of a run that outgrows the workspace
hands the run back at the chunk's start and the resumed run is bitwise the
run of a context that grew its own memory; and the two FP32 accumulation
forms (fixed-point and plain float64 partial sums) both match the oracle."""
import numpy as np
import pytest

from gpu_common import make_ctx, rel_norm, say, split
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _run(workspace, prec):
    import torch

    import paper_2201_04622_amd.eamfe as E
    # verbatim crystals densify under this potential: rows of 64 slots overflow within the run
    reps = [I.Replica("bcc", 4, I.A_BCC_VERBATIM, 1200.0, 5.0, 3), I.Replica("fcc", 4, I.A_FCC_VERBATIM, 900.0, 5.0, 4)]
    ctx = E.Context(0, prec, workspace=workspace)
    ctx.set_launch(2, 256)
    ctx.eam_setup(I.synthetic_eam_knots())
    x = E.to_soa(I.batch_arrays(reps)["x0"])
    ctx.system_setup(reps, x)
    v = torch.zeros_like(x)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, 0.3, 64)       # explicit short rows
    first = ctx.workspace_bytes()
    ctx.set_chunk(200)
    p = E.protocol("fl", 200, 600, 100, 100, skin=0.3)
    S = 1600
    W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, S, W_out=W)
    out = (x.cpu().numpy(), v.cpu().numpy(), W.cpu().numpy(), ctx.device_allocations(), ctx.replays(),
           first, ctx.workspace_bytes(), ctx.list_stats())
    ctx.close()
    return out


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_caller_workspace_allocates_nothing_and_resumes_bitwise(prec):
    xw, vw, Ww, aw, rw, first, last, stats = _run(True, prec)
    xs, vs, Ws, as_, rs, _, _, _ = _run(False, prec)
    say(f"prec {prec}: workspace {first[1]} -> {last[1]} bytes, replays {rw}/{rs}, library allocations {aw}/{as_}, "
        f"rows mean {stats[0]:.1f} max {stats[1]} cap {stats[2]}")
    assert aw == 0 and as_ >= 1
    assert rw >= 1 and rs >= 1            # the rows overflowed and the chunk was replayed
    assert last[1] > first[1]             # the workspace grew in the middle of the run
    assert np.array_equal(xw, xs) and np.array_equal(vw, vs) and np.array_equal(Ww, Ws)


def test_workspace_query_and_rejection():
    import ctypes as C

    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 1)]
    ctx, x0, _ = make_ctx(reps, FP32)
    need, held = ctx.workspace_bytes()
    assert 0 < need <= held
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    code = E.lib().eamfe_set_workspace(ctx._h, C.c_void_p(small.data_ptr()), C.c_size_t(need // 2))
    assert code == E.ENOMEM                # too small: refused, the context keeps its workspace
    f = torch.zeros_like(x0)
    ctx.eam_forces(x0, f)                  # still usable
    assert ctx.device_allocations() == 0
    ctx.close()


@pytest.mark.parametrize("deterministic", [True, False])
def test_fp32_accumulation_forms_match_the_oracle(opot, deterministic):
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 1), I.Replica("fcc", 4, I.A_FCC_VERBATIM, 300.0, 5.0, 2)]
    arrs = I.batch_arrays(reps)
    xs = [I.displaced(r.sites(), 0.05, seed=10 + q) for q, r in enumerate(reps)]
    xd = E.to_soa(np.concatenate(xs))
    got = {}
    for lanes in (1, 4):
        ctx = E.Context(0, FP32, deterministic=deterministic)
        ctx.set_launch(lanes, 256)
        ctx.eam_setup(I.synthetic_eam_knots())
        ctx.system_setup(reps, E.to_soa(arrs["x0"]))
        f = torch.zeros_like(xd)
        U = torch.zeros(len(reps), dtype=torch.float64, device="cuda")
        ctx.eam_forces(xd, f, U)
        f2 = torch.zeros_like(xd)
        ctx.eam_forces(xd, f2)
        assert torch.equal(f, f2)          # run to run, either form
        got[lanes] = (E.from_soa(f), U.cpu().numpy(), ctx.offsets)
        ctx.close()
    for lanes, (fg, Ug, off) in got.items():
        for q, (r, xr) in enumerate(zip(reps, xs)):
            o = opot.eam(xr, r.box)
            assert rel_norm(split(fg, off)[q], o["f"]) < 1e-5
            assert abs(Ug[q] - o["U"]) < 1e-6 * abs(o["U"])
    same = np.array_equal(got[1][0], got[4][0])
    say(f"deterministic={deterministic}: forces bitwise equal across lanes 1 and 4: {same}")
    if deterministic:
        assert same                        # fixed point: independent of the launch shape
