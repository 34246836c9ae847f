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
    F0, Ed, _ = E.fl_free_energy(Wf, Wb, N - 1, rep.T, rep.k, rep.mass, N=N, V=float(np.prod(rep.box)))
    sysrec = rec["systems"][0]
    say(f"runner F0 {sysrec['F0_per_atom']:.8f} eV/atom, direct {F0 / N:.8f}; {rec['run']}")
    assert rec["steps"] == S and rec["atoms"] == N and len(rec["systems"]) == 1
    assert sysrec["F0_per_atom"] == F0 / N and sysrec["E_diss_per_atom"] == Ed / N
    assert sysrec["W_fwd"] == Wf.tolist() and sysrec["W_bwd"] == Wb.tolist()
    assert rec["run"]["atom_steps_per_s"] > 0 and rec["run"]["mean_neighbour_row"] > 0
    assert S < rec["run"]["force_passes"] <= S + S // 1000 + 1   # one pass per step plus one per chunk
    assert rec["dF_bcc_to_fcc"] == []
