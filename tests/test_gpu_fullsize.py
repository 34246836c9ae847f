"""Parity at the full workload sizes, in the launch shapes the benchmark uses.

The oracle is O(N^2) per replica, so at full size it computes sampled
outputs one atom at a time (orc_eam_atom: the force, energy and density of
one atom from brute-force sums over its whole replica), plus whole-replica
energies for a few replicas.  Properties that hold at any size are checked
on every atom: the EAM forces of a replica sum to zero (pair terms are
antisymmetric) and F32 results are identical in two launch shapes.

Workloads: the 64-replica uneven batch (113,090 atoms), the RS scan batch
(8 x bcc 20^3, 128,000 atoms) and the large FL batch (16 bcc 30^3 + 16 fcc
24^3, 1,748,736 atoms), at thermally displaced positions (sigma 0.05 A)."""
import numpy as np
import pytest

from gpu_common import make_ctx, say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1
# the batched parity bar: per component within 10 TOL of the replica's rms force,
# per-atom energies within 100 ETOL relative, replica energies within ETOL
TOL = {FP64: 1e-12, FP32: 1e-5}
ETOL = {FP64: 1e-13, FP32: 1e-6}
N_SAMPLE = 48


def _setup(name, prec, lanes, block):
    import paper_2201_04622_amd.eamfe as E
    reps = I.workload(name).replicas
    ctx, x0, arrs = make_ctx(reps, prec, lanes, block)
    x = I.displaced(arrs["x0"], 0.05, seed=17)
    xd = E.to_soa(x)
    ctx.neigh_build(xd, 0.5, 0)
    return ctx, reps, x, xd


def _forces(ctx, xd):
    import torch
    f = torch.zeros_like(xd)
    U = torch.zeros(ctx.n_rep, dtype=torch.float64, device="cuda")
    ea = torch.zeros(xd.shape[1], dtype=torch.float64, device="cuda")
    ctx.eam_forces(xd, f, U, ea)
    return f, U, ea


@pytest.mark.parametrize("name,prec,lanes,block", [
    ("batch64", FP32, 2, 1024), ("batch64", FP32, 1, 512), ("batch64", FP64, 2, 1024),
    ("rs_scan", FP32, 2, 1024), ("fl_large", FP32, 2, 1024), ("fl_large", FP64, 2, 1024)])
def test_sampled_atoms_match_oracle(opot, name, prec, lanes, block):
    import paper_2201_04622_amd.eamfe as E
    say(f"full size: {name} prec={prec} lanes={lanes} block={block}")
    ctx, reps, x, xd = _setup(name, prec, lanes, block)
    f, U, ea = _forces(ctx, xd)
    fg = E.from_soa(f)
    eg = ea.cpu().numpy()
    Ug = U.cpu().numpy()
    off = ctx.offsets
    ctx.close()
    rng = np.random.default_rng(5)
    atoms = np.sort(rng.choice(x.shape[0], N_SAMPLE, replace=False))
    worst = 0.0
    for gi in atoms:
        r = int(np.searchsorted(off, gi, side="right") - 1)
        i = int(gi - off[r])
        xr = x[off[r]:off[r + 1]]
        o = opot.eam_atom(xr, reps[r].box, i)
        scale = np.sqrt((fg[off[r]:off[r + 1]] ** 2).mean())
        err = np.abs(fg[gi] - o["f"]).max() / scale
        worst = max(worst, err)
        assert err <= 10 * TOL[prec], (name, gi, err)
        assert abs(eg[gi] - o["e_atom"]) <= 100 * ETOL[prec] * abs(o["e_atom"]), (name, gi, eg[gi], o["e_atom"])
    say(f"  worst sampled force error {worst:.2e} of the rms force")
    # every atom: the EAM forces of a replica sum to zero
    for r in range(len(reps)):
        fr = fg[off[r]:off[r + 1]]
        scale = np.sqrt((fr ** 2).mean()) * np.sqrt(fr.shape[0])
        assert np.abs(fr.sum(axis=0)).max() <= 10 * TOL[prec] * scale, (name, r)
    # whole-replica energies of the smallest and the largest replica
    sizes = [rp.natoms for rp in reps]
    for r in sorted({int(np.argmin(sizes)), int(np.argmax(sizes))}):
        if sizes[r] > 20000:
            continue   # O(N^2) oracle energy is too slow here; sampled atoms cover these replicas
        o = opot.eam(x[off[r]:off[r + 1]], reps[r].box)
        assert abs(Ug[r] - o["U"]) <= ETOL[prec] * abs(o["U"]), (name, r, Ug[r], o["U"])


def test_fp32_full_batch_identical_in_two_launch_shapes():
    """Fixed-point FP32 sums: the 113,090-atom batch gives the same bits with
    2 lanes x 1024 threads and 1 lane x 512 threads."""
    out = []
    for lanes, block in ((2, 1024), (1, 512)):
        ctx, reps, x, xd = _setup("batch64", FP32, lanes, block)
        f, U, ea = _forces(ctx, xd)
        out.append((f.cpu().numpy(), U.cpu().numpy(), ea.cpu().numpy()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])       # forces
    assert np.array_equal(out[0][2], out[1][2])       # per-atom energies
    # replica totals are float64 sums over tiles, whose boundaries differ between the shapes
    assert np.allclose(out[0][1], out[1][1], rtol=1e-14, atol=0)
