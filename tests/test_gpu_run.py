"""The workload runner: one named workload end to end through the library,
its JSON record against the same estimators called directly."""
import json

import numpy as np
import pytest

from gpu_common import say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_runner_record_matches_the_direct_estimate(tmp_path):
    """fl_bcc4 (stable: bcc 6^3 at a0, 6000 steps, FP64) through the CLI: the
    record's F0 per atom is the FL estimate of the same run made by hand (the
    run is deterministic), and the record carries the run statistics."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    from paper_2201_04622_amd import run as R
    out = tmp_path / "rec.json"
    assert R.main(["fl_bcc4", "--stable", "--precision", "fp64", "--out", str(out)]) == 0
    rec = json.loads(out.read_text())
    wl = I.workload("fl_bcc4", stable=True)
    rep = wl.replicas[0]
    ctx = E.Context(0, E.FP64)
    ctx.eam_setup(I.synthetic_eam_knots())
    x = E.to_soa(I.batch_arrays(wl.replicas)["x0"])
    ctx.system_setup(wl.replicas, x)
    v = torch.zeros_like(x)
    p = E.protocol_from_schedule(wl.schedule, skin=0.3)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, 0.3, 0)
    S = wl.schedule.total_steps
    W = torch.zeros(1, S, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, S, W_out=W)
    ctx.close()
    Wf, Wb = E.switch_works(p, W.cpu().numpy())
    N = rep.natoms
    F0, Ed, _ = E.fl_free_energy(Wf, Wb, N, rep.T, rep.k, rep.mass, N=N, V=float(np.prod(rep.box)))
    sysrec = rec["systems"][0]
    say(f"runner F0 {sysrec['F0_per_atom']:.8f} eV/atom, direct {F0 / N:.8f}; {rec['run']}")
    assert rec["steps"] == S and rec["atoms"] == N and len(rec["systems"]) == 1
    assert sysrec["F0_per_atom"] == F0 / N and sysrec["E_diss_per_atom"] == Ed / N
    assert sysrec["W_fwd"] == Wf.tolist() and sysrec["W_bwd"] == Wb.tolist()
    assert rec["run"]["atom_steps_per_s"] > 0 and rec["run"]["mean_neighbour_row"] > 0
    assert S < rec["run"]["force_passes"] <= S + S // 1000 + 1   # one pass per step plus one per chunk
    assert rec["dF_bcc_to_fcc"] == []


def test_runner_rs_scan_matches_the_direct_estimate():
    """rs_small (stable: 4 x bcc 6^3, 300 -> 600 K) through the runner: its
    companion FL and its F(T) curve (fixed-centre-of-mass Eq. rs) equal the
    same estimators applied by hand to runs with the same seeds."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    from paper_2201_04622_amd import run as R
    rec = R.run_workload("rs_small", stable=True, precision=E.FP32, fl_companion=(500, 2000, 500))
    wl = I.workload("rs_small", stable=True)
    reps, sch = wl.replicas, wl.schedule
    N = reps[0].natoms

    def batch():
        ctx = E.Context(0, E.FP32)
        ctx.eam_setup(I.synthetic_eam_knots())
        x = E.to_soa(I.batch_arrays(reps)["x0"])
        ctx.system_setup(reps, x)
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, 0.3, 0)
        return ctx, x, v

    ctx, x, v = batch()
    pf = E.protocol("fl", 500, 2000, 500, 0, function=2, skin=0.3)
    Wfl = torch.zeros(len(reps), 5000, dtype=torch.float64, device="cuda")
    ctx.run_switching(pf, x, v, 0, 5000, W_out=Wfl)
    ctx.close()
    Wf, Wb = E.switch_works(pf, Wfl.cpu().numpy())
    V = float(np.prod(reps[0].box))
    F0, _, _ = E.fl_free_energy(Wf, Wb, N, reps[0].T, reps[0].k, reps[0].mass, N=N, V=V)
    assert rec["companion_fl"]["system"]["F0_per_atom"] == F0 / N
    ctx, x, v = batch()
    p = E.protocol_from_schedule(sch, skin=0.3)
    W = torch.zeros(len(reps), sch.total_steps, dtype=torch.float64, device="cuda")
    ctx.run_switching(p, x, v, 0, sch.total_steps, W_out=W)
    ctx.close()
    grid = np.array(rec["T_grid"])
    F = np.array([E.rs_free_energy_cm(p, W[q].cpu().numpy(), F0, 300.0, N, V, reps[0].mass, grid)
                  for q in range(len(reps))]) / N
    say(f"runner F(600 K) {rec['F_per_atom'][-1]:.6f} eV/atom, direct {F.mean(axis=0)[-1]:.6f}")
    assert grid[0] == 300.0 and grid[-1] == 600.0 and len(grid) == 301
    assert np.array_equal(np.array(rec["F_per_atom"]), F.mean(axis=0))
