"""Run one of the named workloads end to end and write its results as JSON.

    python -m paper_2201_04622_amd.run fl_mid --stable --precision fp32 --out fl_mid.json

Frenkel--Ladd workloads: every replica runs the workload's protocol in one
batched launch; replicas of one system (same lattice, cells, lattice
parameter, T, k and mass) are realizations, and each system gets F0 (Eq. fl
with Eq. cm) per atom with its standard error, the dissipation (Eq. Ediss)
and the one-way Jarzynski estimates (Eq. jarz).  For every temperature with
both a bcc and an fcc system, dF(bcc -> fcc) per atom follows.

Reversible-scaling workloads: a companion FL run at T0 on the same cells
gives F0(T0) (the reading of the paper's scans that starts each from an FL
result), then every replica's work trace gives F(T) on a 1 K grid from T0 to
T0 / lambda_f (Eq. rs), averaged over replicas with its standard error.

The record also holds the run's throughput (atom-steps/s over the switching
calls, by HIP events), the time-averaged neighbour row and the list
rebuilds.  Every step runs through the library; this module only sequences
the calls and groups the results.
"""
from __future__ import annotations

import argparse
import json
import sys
from collections import OrderedDict

import numpy as np

from . import eamfe as E
from . import fl as FL
from . import inputs as I


def _system_key(r):
    return (r.kind, tuple(r.dims), float(r.a), float(r.T), float(r.k), float(r.mass), float(r.vacuum))


def _run(ctx, p, x, v, S):
    import torch
    W = torch.zeros(ctx.n_rep, S, dtype=torch.float64, device="cuda")
    ctx.row_history(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.run_switching(p, x, v, 0, S, W_out=W, sync=False)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1)
    mean_row, passes = ctx.row_history()
    rebuilt_reps, rebuilt_atoms = ctx.list_rebuilds()
    stats = {"atom_steps_per_s": ctx.N * S / (ms / 1e3), "ms_per_step": ms / S, "mean_neighbour_row": mean_row,
             "force_passes": passes, "list_rebuilds_per_step": rebuilt_reps / S,
             "atoms_rebuilt_per_step": rebuilt_atoms / S}
    return W.cpu().numpy(), stats


def _context(reps, precision, skin):
    import torch
    ctx = E.Context(0, precision)
    ctx.eam_setup(I.synthetic_eam_knots())
    arrs = I.batch_arrays(reps)
    x = E.to_soa(arrs["x0"])
    ctx.system_setup(reps, x)
    v = torch.zeros_like(x)
    return ctx, x, v


def fl_results(reps, p, W):
    """Per-system FL estimates from the work traces W [n_rep, S]."""
    Wf, Wb = E.switch_works(p, W)
    systems = OrderedDict()
    for q, r in enumerate(reps):
        systems.setdefault(_system_key(r), []).append(q)
    out = []
    for key, rows in systems.items():
        r0 = reps[rows[0]]
        N = r0.natoms
        n_eff = N   # Eq. fl: all N oscillators; the held centre of mass enters through Eq. cm
        V = float(np.prod(r0.box))
        F0, Ed, err = FL.system_free_energy(p, Wf[rows], Wb[rows], r0, V)
        FE = E.einstein_free_energy(n_eff, r0.T, r0.k, r0.mass)
        cm = E.fixed_cm_correction(N, V, r0.T, r0.k) if p.fix_com else 0.0
        jf, jfe = E.jarzynski(Wf[rows], r0.T)
        jb, jbe = E.jarzynski(Wb[rows], r0.T)
        out.append({"kind": r0.kind, "cells": list(r0.dims), "a": r0.a, "T": r0.T, "k": r0.k, "atoms": N,
                    "vacuum": r0.vacuum, "realizations": len(rows), "F0": F0, "F0_per_atom": F0 / N,
                    "F0_err_per_atom": err / N, "E_diss_per_atom": Ed / N,
                    "F0_jarzynski_fwd_per_atom": (FE + cm - jf) / N, "F0_jarzynski_fwd_err": jfe / N,
                    "F0_jarzynski_bwd_per_atom": (FE + cm + jb) / N, "F0_jarzynski_bwd_err": jbe / N,
                    "W_fwd": Wf[rows].tolist(), "W_bwd": Wb[rows].tolist()})
    diffs = []
    for s in out:
        if s["kind"] != "bcc" or s["vacuum"]:
            continue
        for t in out:
            if t["kind"] == "fcc" and not t["vacuum"] and t["T"] == s["T"]:
                diffs.append({"T": s["T"], "dF_bcc_to_fcc_per_atom": t["F0_per_atom"] - s["F0_per_atom"],
                              "err": float(np.hypot(s["F0_err_per_atom"], t["F0_err_per_atom"]))})
    return out, diffs


def msd_springs(reps, precision, skin, n_steps=4000, every=100, discard=1000):
    """The replicas with each system's spring constant replaced by k = 3 kB T
    / msd (Eq. msd), the mean over the system's realizations of an
    equilibrium run of H0 (springs.spring_constants)."""
    import dataclasses

    from . import springs as SP
    ctx, x, v = _context(reps, precision, skin)
    ctx.init_velocities(v, True)
    ctx.neigh_build(x, skin, 0)
    k, _, _ = SP.spring_constants(ctx, reps, x, v, n_steps, every, skin=skin, discard=discard)
    ctx.close()
    groups = OrderedDict()
    for q, r in enumerate(reps):
        groups.setdefault(_system_key(r), []).append(q)
    out = list(reps)
    for rows in groups.values():
        km = float(np.mean(k[rows]))
        for q in rows:
            out[q] = dataclasses.replace(reps[q], k=km)
    return out


def run_workload(name, stable=False, precision=E.FP32, skin=0.3, fl_companion=(2000, 20000, 2000), k_msd=False):
    """``k_msd``: replace the workload's spring constants by the ones the
    mean-squared displacement gives (for the FL runs, including the RS
    scan's companion)."""
    wl = I.workload(name, stable=stable)
    reps, sch = wl.replicas, wl.schedule
    p = E.protocol_from_schedule(sch, skin=skin)
    S = sch.total_steps
    rec = {"workload": wl.name, "description": wl.description, "precision": "fp32" if precision == E.FP32 else "fp64",
           "replicas": len(reps), "atoms": int(sum(r.natoms for r in reps)), "steps": S, "skin": skin,
           "data": "synthetic"}
    if sch.mode == "fl":
        if k_msd:
            reps = msd_springs(reps, precision, skin)
        ctx, x, v = _context(reps, precision, skin)
        ctx.init_velocities(v, sch.fix_com)
        ctx.neigh_build(x, skin, 0)
        W, stats = _run(ctx, p, x, v, S)
        ctx.close()
        rec["run"] = stats
        rec["systems"], rec["dF_bcc_to_fcc"] = fl_results(reps, p, W)
    elif sch.mode == "rs":
        T0 = reps[0].T
        if any(r.T != T0 for r in reps):
            raise ValueError("run: the replicas of an RS scan share T0")
        n_eq, n_sw, n_hold = fl_companion
        pf = E.protocol("fl", n_eq, n_sw, n_hold, 0, function=2, dt=sch.dt, damp=sch.damp, fix_com=sch.fix_com,
                        skin=skin)
        creps = msd_springs(reps, precision, skin) if k_msd else reps   # the companion FL's replicas
        ctx, x, v = _context(creps, precision, skin)
        ctx.init_velocities(v, sch.fix_com)
        ctx.neigh_build(x, skin, 0)
        Wfl, fstats = _run(ctx, pf, x, v, n_eq + 2 * n_sw + n_hold)
        ctx.close()
        fl_sys, _ = fl_results(creps, pf, Wfl)
        F0_T0 = fl_sys[0]["F0"] if len(fl_sys) == 1 else None   # the system's F0 itself, not per atom times N
        if F0_T0 is None:
            raise ValueError("run: the replicas of an RS scan must be realizations of one system")
        ctx, x, v = _context(reps, precision, skin)
        ctx.init_velocities(v, sch.fix_com)
        ctx.neigh_build(x, skin, 0)
        W, stats = _run(ctx, p, x, v, S)
        ctx.close()
        N = reps[0].natoms
        Tf = T0 / sch.lambda_f
        grid = np.arange(T0, Tf + 0.5, 1.0)
        if sch.fix_com:   # F0(T0) includes Eq. cm, the run keeps the centre of mass fixed
            V = float(np.prod(reps[0].box))
            F = np.array([E.rs_free_energy_cm(p, W[q], F0_T0, T0, N, V, reps[0].mass, grid)
                          for q in range(len(reps))]) / N
        else:
            F = np.array([E.rs_free_energy(p, W[q], F0_T0, T0, N, grid) for q in range(len(reps))]) / N
        rec["run"] = stats
        rec["companion_fl"] = {"run": fstats, "system": fl_sys[0]}
        rec["T_grid"] = grid.tolist()
        rec["F_per_atom"] = F.mean(axis=0).tolist()
        rec["F_err_per_atom"] = (F.std(axis=0, ddof=1) / np.sqrt(len(reps))).tolist() if len(reps) > 1 else None
    else:
        raise ValueError(f"run: workload mode {sch.mode!r} is not a free-energy run")
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("workload", help="fl_bcc4 | fl_mid | batch64 | rs_scan | fl_large")
    ap.add_argument("--stable", action="store_true", help="the potential's own zero-pressure lattice constants")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--skin", type=float, default=0.3)
    ap.add_argument("--k-msd", action="store_true", help="spring constants from the mean-squared displacement")
    ap.add_argument("--out", default=None, help="JSON file (default: stdout)")
    args = ap.parse_args(argv)
    rec = run_workload(args.workload, args.stable, E.FP32 if args.precision == "fp32" else E.FP64, args.skin,
                       k_msd=args.k_msd)
    text = json.dumps(rec)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    else:
        print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
