#!/usr/bin/env python
"""Throughput of batched EAM switching MD on one MI355X.

Default workload: 64 independent Frenkel--Ladd switching replicas of uneven
size (bcc 6..12^3 and fcc 5..10^3 cubic supercells, 113,090 atoms, T on a
16-point grid over 100..1600 K, k = 5 eV/A^2, 20k forward + 20k backward
steps with 2k-step holds), FP32 pair arithmetic with FP64 positions,
energies and work, one launch per pass over all replicas.

A "step" is one MD step of every replica: neighbour-list upkeep, density
pass, force pass with the fused spring/blend/BAOAB update and the work
increment.  The metric is atom-steps/s over the K timed steps (inputs
resident on the device, protocol continued from the W warm-up steps).

Also reported, in the same JSON line:
  * the dominant kernel's (the force pass's) roofline figure, its sampled
    launches stamped with their own start and end by HIP's extended launch
    on the library's stream, with counter traffic and issue shares from a
    committed summary of the same run;
  * the plain single-replica FP64 path (bcc 10^3, 2000 atoms);
  * bounded runs of the other workloads (stable lattice, FP64 batch, eager
    against hipGraph, RS scan, large FL batch);
  * an FP32 against FP64 free-energy check on the stable batch;
  * the FP64 CPU oracle timed on a bounded sample on the host cores.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-fp64] [--no-configs] [--no-dF]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2201_04622_amd/csrc/eamfe_kernels.hip", "paper_2201_04622_amd/csrc/eamfe_internal.h",
                  "paper_2201_04622_amd/build.py")   # the build flags shape the code too
# worker threads of the all-core oracle leg: at most the host share of one GPU
CPU_THREADS_MAX = 16


def timing_stride(steps):
    """Iterations between two HIP-event samples of the dominant kernel inside
    the timed region.  The first timed iteration is always sampled, then every
    stride-th.  An event pair adds about 5 us of stream time to a step of
    60-80 us, so one sample in ten or fewer keeps the timed value within
    about 1 % of an unsampled run (measured: 10 % at one in two); long runs
    take one in fifty."""
    return max(10, min(50, steps // 10))


def force_bytes_per_atom(n_list, prec):
    """Algorithmic bytes of the force pass per atom: x read and written,
    v read and written, x0 read (3 x 8 B each), own F' (4 or 8 B), the row
    length (4 B) and the row of n_list int32 neighbour ids.  Neighbour
    positions and F' gathers are reuse of data already counted."""
    fp = 4 if prec == "fp32" else 8
    return 24 * 2 + 24 * 2 + 24 + fp + 4 + 4 * n_list


def density_bytes_per_atom(n_list, prec):
    """x read, row length and row, F' and F written."""
    fp = 4 if prec == "fp32" else 8
    return 24 + 4 + 4 * n_list + fp + 8


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _summary_fields(path, sectioned=False):
    """The "name: value" fields of a committed profile summary.  Sectioned:
    the header fields before the first "kernel:" line, and the fields of
    each per-kernel section, keyed by its kernel."""
    head, sections, cur = {}, {}, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            v = v.split("#", 1)[0].strip()
            if sectioned and k == "kernel":
                cur = sections.setdefault(v, {})
            elif cur is not None:
                cur[k] = v
            else:
                head.setdefault(k, v)
    return head, sections


def _summary_covers(head, workload, prec, launch, skin, steps, warmup):
    """True when a summary was taken with the current kernel sources on this
    run: the same workload, precision, launch shape, skin and run length
    (timed steps and warm-up steps: the neighbour rows, and so the bytes a
    launch moves, follow the state the crystal has reached)."""
    try:
        return (head.get("kernel_source_sha256") == kernel_source_hash()
                and head.get("workload") == workload and head.get("precision") == prec
                and head.get("launch") == f"lanes {launch[0]} block {launch[1]} grid {launch[2]}"
                and float(head["skin"]) == float(skin)
                and int(head["steps"]) == int(steps) and int(head["warmup"]) == int(warmup))
    except (KeyError, ValueError, TypeError):
        return False


def measured_traffic(kernel, workload, prec, launch, skin, steps, warmup):
    """HBM bytes per launch of ``kernel`` from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the factor the same
    counter reads for a plain copy), or None when no summary covers this
    kernel, workload, precision, launch shape, skin and run length, or the
    kernel sources have changed since the counters were taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_*_hbm_traffic.txt"))):
        head, _ = _summary_fields(path)
        if head.get("kernel", "").split("<")[0] == kernel and \
                _summary_covers(head, workload, prec, launch, skin, steps, warmup):
            return float(head["traffic_bytes_per_launch"])
    return None


def measured_issue(kernel, workload, prec, launch, skin, steps, warmup):
    """VALU issue and LDS bank-conflict shares of ``kernel``'s cycles over the
    timed dispatches, from a committed SQ counter summary, or None when none
    covers this kernel, workload, precision, launch, skin and run length, or
    the kernel sources have changed since the counters were taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "k_force_k_density_*_issue_utilisation.txt"))):
        head, sections = _summary_fields(path, sectioned=True)
        if not _summary_covers(head, workload, prec, launch, skin, steps, warmup):
            continue
        for name, kv in sections.items():
            if name.split("<")[0] == kernel and "valu_issue" in kv:
                return {"valu_issue": float(kv["valu_issue"]), "lds_conflict": float(kv["lds_conflict"]),
                        "resident_waves_per_simd": float(kv["resident_waves_per_simd"])}
    return None


def run_gpu(workload, prec, steps, warmup, lanes, block, autotune, skin, only=None, stride=None, graph=0,
            list_builder="auto", stable=False, grid=-1):
    """Run warmup + steps steps of a workload's protocol on the GPU; the
    last `steps` are timed with HIP events around one run_switching call on
    the library's stream (torch's current stream).  Inside the timed region
    the force pass of the first timed iteration and then of every
    stride-th one is stamped with its own start and end (stride 0: none)."""
    import torch

    import paper_2201_04622_amd.eamfe as E
    from paper_2201_04622_amd import inputs as I

    wl = I.workload(workload, stable=stable)
    sch = wl.schedule
    # extend the trailing hold so the protocol covers warm-up + timed steps
    need = warmup + steps
    if sch.total_steps < need:
        sch = I.Schedule(**{**sch.__dict__, "n_hold2": sch.n_hold2 + need - sch.total_steps})
    p = E.protocol_from_schedule(sch, skin=skin)
    reps = wl.replicas if only is None else [wl.replicas[i] for i in only]
    arrs = I.batch_arrays(reps)
    ctx = E.Context(0, E.FP32 if prec == "fp32" else E.FP64)
    if list_builder != "auto":
        ctx.set_list_builder(list_builder == "lds")
    if lanes:
        ctx.set_launch(lanes, block)
    if grid >= 0:
        ctx.set_grid(grid)
    ctx.eam_setup(I.synthetic_eam_knots())
    x = E.to_soa(arrs["x0"])
    ctx.system_setup(reps, x)
    v = torch.zeros_like(x)
    ctx.init_velocities(v, sch.fix_com)
    ctx.neigh_build(x, skin, 0)
    tuned = None
    if warmup:
        ctx.run_switching(p, x, v, 0, warmup, sync=True)
    if autotune and not lanes:
        tuned = ctx.autotune(p, warmup, x, v, trial_steps=20)
        if list_builder != "auto":   # the tuner times both builders; an explicit choice stands
            ctx.set_list_builder(list_builder == "lds")
    if graph:
        ctx.set_graph(graph)
    natoms = int(arrs["x0"].shape[0])
    torch.cuda.synchronize()
    stride = timing_stride(steps) if stride is None else stride
    ctx.set_kernel_timing(stride, kinds=("force",))
    ctx.row_history(reset=True)   # list work of the timed passes only
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    ctx.run_switching(p, x, v, warmup, warmup + steps, sync=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kt = ctx.kernel_timing()
    ctx.set_kernel_timing(0)
    ctx.check()
    mean_nl, passes = ctx.row_history()   # time average over the timed force passes
    rebuilt_reps, rebuilt_atoms = ctx.list_rebuilds()
    end_nl, max_nl, cap = ctx.list_stats()
    launch = (*ctx.get_launch(), ctx.get_grid())   # lanes per atom, block threads, grid blocks (0: one per slice)
    builder = ctx.get_list_builder()
    ctx.close()
    return {
        "natoms": natoms, "n_rep": len(reps), "steps": steps, "warmup": warmup, "ms": ms, "wall_s": wall, "kt": kt,
        "stride": stride, "mean_nl": mean_nl, "passes": passes, "rebuilt_reps": rebuilt_reps,
        "rebuilt_atoms": rebuilt_atoms, "end_nl": end_nl, "max_nl": max_nl, "cap": cap, "launch": launch,
        "tuned": tuned, "desc": wl.description, "list_builder": builder,
    }


def roofline(run, prec, workload, skin):
    """The dominant kernel's (the force pass's) HBM roofline figure from a
    run_gpu record: algorithmic bytes per launch (per-atom bytes at the mean
    row length of the timed passes, times the atoms one launch processes)
    over the mean event-timed launch duration.  None when the timed region
    had no sampled launch (timing switched off)."""
    ms, n = run["kt"]["force"]
    if n <= 0 or not ms > 0.0:
        return None
    avg_ms = ms / n
    bpa = force_bytes_per_atom(run["mean_nl"], prec)
    bytes_launch = bpa * run["natoms"]
    achieved = bytes_launch / (avg_ms / 1e3) / 1e9
    return {
        "bound": "hbm", "kernel": "k_force",
        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": measured_traffic("k_force", workload, prec, run["launch"], skin, run["steps"], run["warmup"]),
        "algorithmic_bytes": bytes_launch, "bytes_per_atom": bpa,
        # the same kernel's VALU issue and LDS-conflict shares from SQ counters (what bounds it)
        "issue": measured_issue("k_force", workload, prec, run["launch"], skin, run["steps"], run["warmup"]),
        "avg_launch_us": avg_ms * 1e3, "launches_timed": n, "timing_stride": run["stride"],
    }


def host_cpu():
    """Threads this process may run on (the machine's host share, capped) and the
    host's CPU model and clock as /proc/cpuinfo reports them."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                if k.strip() == "model name" and model == "unknown":
                    model = v.strip()
                elif k.strip() == "cpu MHz" and mhz is None:
                    mhz = float(v)
    except OSError:
        pass
    return {"threads_available": avail, "model": model, "mhz": mhz}


def cpu_baseline(target_s=8.0):
    """The FP64 oracle as it stands (plain C, scalar loops, Verlet candidate
    lists with a 0.3 A skin), timed on the host on a bounded sample of the
    default workload's Frenkel--Ladd protocol from the lattice start:
      * one core: replica 4 of the batch (bcc 10^3, 2000 atoms) for about
        target_s seconds;
      * all cores: one worker thread per available core (at most
        CPU_THREADS_MAX), each running a different replica of the batch
        (uneven sizes, replicas 0, 1, ...) in 20-step chunks for about
        target_s seconds; the rate is all atom-steps over the leg's wall time.
    The oracle is a single C call per chunk (ctypes releases the GIL), so the
    threads run concurrently.  `value` is the all-core rate."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2201_04622_amd import inputs as I
    O.build()
    wl = I.workload("batch64")
    pot = O.Potential.from_knots(I.synthetic_eam_knots())
    lam = O.schedule("fl", 2000, 20000, 2000, 0)

    def leg(r, budget, chunk=20):
        """Steps of replica r in chunks until `budget` seconds have passed;
        (atom-steps done, seconds used)."""
        prm = O.RunParams(mode="fl", T=r.T, k=r.k, seed=r.seed, fix_com=True, skin=0.3, nlist_cap=512)
        x0 = r.sites()
        x, v = x0.copy(), O.init_velocities(prm, r.natoms)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            O.run(pot, prm, x0, r.box, x, v, lam[done: done + chunk + 1], step0=done)
            done += chunk
        return r.natoms * done, time.perf_counter() - t0

    one = wl.replicas[4]
    as1, t1 = leg(one, target_s)
    rate1 = as1 / t1
    host = host_cpu()
    n_thr = max(1, min(CPU_THREADS_MAX, host["threads_available"]))
    reps = [wl.replicas[q % len(wl.replicas)] for q in range(n_thr)]
    t = time.perf_counter()
    with ThreadPoolExecutor(n_thr) as ex:
        res = list(ex.map(lambda r: leg(r, target_s), reps))
    wall = time.perf_counter() - t
    as_all = sum(a for a, _ in res)
    steps_each = [a // r.natoms for (a, _), r in zip(res, reps)]
    return {
        "value": as_all / wall, "unit": "atom-steps/s", "cores": n_thr, "kind": "oracle",
        "sample": (f"FP64 oracle, {n_thr} threads each running one replica of the 64-replica batch "
                   f"({sum(r.natoms for r in reps)} atoms in all, {min(steps_each)}-{max(steps_each)} FL steps "
                   f"each from the lattice start, {wall:.1f} s wall); one core: bcc 10^3 (2000 atoms), "
                   f"{as1 // one.natoms} steps in {t1:.1f} s"),
        "single_core": {"value": rate1, "unit": "atom-steps/s", "cores": 1},
        "host": host,
    }


# The other workloads, each a bounded run of its own protocol from the lattice
# start (warm-up untimed): name, workload, stable lattice, precision, timed
# steps, warm-up steps, graph iterations (0: eager), skin (None: the bench's;
# the stable lattice's smallest boxes, 11.79 A, take at most 0.59 A).  The
# graph/eager pair times without sampled kernel events, which a captured step
# does not take.
CONFIGS = (
    ("batch64_stable_fp32", "batch64", True, "fp32", 4000, 2000, 0, 0.45),
    ("batch64_fp64", "batch64", False, "fp64", 1000, 500, 0, None),
    ("batch64_fp32_eager", "batch64", False, "fp32", 4000, 2000, 0, None),
    ("batch64_fp32_graph", "batch64", False, "fp32", 4000, 2000, 64, None),
    ("rs_scan_fp32", "rs_scan", False, "fp32", 2000, 1000, 0, None),
    ("fl_large_fp32", "fl_large", False, "fp32", 400, 200, 0, None),
)


def config_record(name, run, prec, workload, skin, graph):
    """Summary of one extra configuration's run_gpu record."""
    rf = None if graph or name.endswith("_eager") else roofline(run, prec, workload, skin)
    return {
        "workload": f"{name}: {run['desc']}", "replicas": run["n_rep"], "atoms": run["natoms"],
        "value": run["natoms"] * run["steps"] / (run["ms"] / 1e3), "unit": "atom-steps/s",
        "steps": run["steps"], "ms_per_step": run["ms"] / run["steps"],
        "mean_neighbour_row": round(run["mean_nl"], 2),
        "launch": {"lanes_per_atom": run["launch"][0], "block_threads": run["launch"][1],
                   "grid_blocks": run["launch"][2]},
        "list_builder": run["list_builder"], "graph_iterations": graph, "skin": skin,
        "force_roofline_frac": None if rf is None else rf["frac"],
        "force_avg_launch_us": None if rf is None else rf["avg_launch_us"],
    }


def run_configs(skin):
    out = {}
    for name, wl, stable, prec, steps, warmup, graph, sk in CONFIGS:
        sk = skin if sk is None else sk
        plain = graph or name.endswith("_eager")
        run = run_gpu(wl, prec, steps, warmup, 0, 0, True, sk, stride=0 if plain else None, graph=graph,
                      stable=stable)
        out[name] = config_record(name, run, prec, wl, sk, graph)
    g, e = out["batch64_fp32_graph"], out["batch64_fp32_eager"]
    out["graph_over_eager"] = g["value"] / e["value"]
    return out


def free_energy_check(skin=0.45, n_eq=500, n_sw=2000, n_hold=500, t_max=1200.0):
    """The metric's accuracy gate, measured: the replicas of the stable
    64-replica batch at up to t_max kelvin run one bounded Frenkel--Ladd
    protocol (n_eq steps at lambda = 0, n_sw forward, n_hold at lambda = 1,
    n_sw backward) in FP32 and in FP64, from the same lattice and with the
    same noise (each replica's seed).  In the hottest replicas the atoms,
    free oscillators on k = 5 eV/A^2 springs at lambda = 1, come close enough
    that a density passes the table's end (ETABLE_RANGE at 1600 K), so they
    are left out with a margin.  Per
    replica the switching estimate (W_fwd - W_bwd)/2 of Eq. fl is taken per
    atom in both precisions; the Einstein term and the centre-of-mass
    correction are the same closed forms in both and cancel in the
    difference.  Returns the mean, standard error and largest magnitude of
    FP32 - FP64 over the replicas in meV/atom, the replicas' temperature at
    that largest one, and the 0.5 meV/atom gate."""
    import numpy as np
    import torch

    import paper_2201_04622_amd.eamfe as E
    from paper_2201_04622_amd import inputs as I
    wl = I.workload("batch64", stable=True)
    reps = [r for r in wl.replicas if r.T <= t_max]
    arrs = I.batch_arrays(reps)
    p = E.protocol("fl", n_eq, n_sw, n_hold, 0, skin=skin)
    S = len(E.lambda_schedule(p)) - 1
    natoms = np.array([r.natoms for r in reps], dtype=np.float64)
    t0 = time.perf_counter()
    est = {}
    for prec in (E.FP32, E.FP64):
        ctx = E.Context(0, prec)
        ctx.eam_setup(I.synthetic_eam_knots())
        x = E.to_soa(arrs["x0"])
        ctx.system_setup(reps, x)
        v = torch.zeros_like(x)
        ctx.init_velocities(v, True)
        ctx.neigh_build(x, skin, 0)
        W = torch.zeros(len(reps), S, dtype=torch.float64, device="cuda")
        ctx.run_switching(p, x, v, 0, S, W_out=W)
        torch.cuda.synchronize()
        Wf, Wb = E.switch_works(p, W.cpu().numpy())
        ctx.check()
        ctx.close()
        est[prec] = (Wf - Wb) / 2.0 / natoms
    return free_energy_summary(est[E.FP32], est[E.FP64], [r.T for r in reps],
                               f"{wl.description}, stable lattice, the replicas at T <= {t_max:g} K",
                               (n_eq, n_sw, n_hold),
                               time.perf_counter() - t0)


def free_energy_summary(d32, d64, temps, workload, legs, wall_s, gate_mev=0.5):
    """The free_energy_check record from per-replica per-atom estimates (eV)."""
    import numpy as np
    d = (np.asarray(d32, dtype=np.float64) - np.asarray(d64, dtype=np.float64)) * 1e3   # meV/atom
    if d.size == 0 or not np.all(np.isfinite(d)):
        raise ValueError("free_energy_check: no finite per-replica estimates")
    i = int(np.argmax(np.abs(d)))
    mean = float(d.mean())
    se = float(d.std(ddof=1) / np.sqrt(d.size)) if d.size > 1 else 0.0
    return {
        "workload": workload, "replicas": int(d.size),
        "protocol": f"FL, {legs[0]} steps at lambda 0, {legs[1]} forward, {legs[2]} at lambda 1, {legs[1]} backward",
        "quantity": "(W_fwd - W_bwd) / 2 per atom, Eq. fl, FP32 minus FP64, same noise",
        "mean_meV_per_atom": mean, "se_meV_per_atom": se, "max_abs_meV_per_atom": float(abs(d[i])),
        "T_at_max_K": float(temps[i]), "gate_meV_per_atom": gate_mev,
        "within_gate": bool(abs(mean) <= gate_mev), "wall_s": round(wall_s, 2),
    }


def result_line(args, main_run, plain, cpu, configs=None, dF=None):
    """The bench's one JSON line from the measured legs (no GPU calls here)."""
    value = main_run["natoms"] * main_run["steps"] / (main_run["ms"] / 1e3)
    kt = main_run["kt"]
    out = {
        "metric": "atom-steps/s, EAM switching MD: batched FP32 vs plain FP64, dF <=0.5 meV/atom",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": main_run["steps"],
        "warmup": args.warmup,
        "ms_per_step": main_run["ms"] / main_run["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {main_run['desc']}",
            "replicas": main_run["n_rep"],
            "atoms": main_run["natoms"],
            "precision": ("f32 pair terms and densities, f64 positions/velocities/energies/work, "
                          "2^-32 fixed-point per-atom sums") if args.precision == "fp32" else "f64 throughout",
            "mean_neighbour_row": round(main_run["mean_nl"], 2),   # over the timed force passes
            "final_neighbour_row": round(main_run["end_nl"], 2),
            "max_neighbour_row": main_run["max_nl"],
            "force_passes": main_run["passes"],
            # list rebuilds of the timed passes: replica lists per step, atoms per step
            "list_rebuilds_per_step": round(main_run["rebuilt_reps"] / main_run["steps"], 3),
            "atoms_rebuilt_per_step": round(main_run["rebuilt_atoms"] / main_run["steps"], 1),
            "launch": {"lanes_per_atom": main_run["launch"][0], "block_threads": main_run["launch"][1],
                       "grid_blocks": main_run["launch"][2],
                       "autotuned": main_run["tuned"] is not None},
            "skin": args.skin,
            "list_builder": main_run["list_builder"],
            "force_kernel_ms_sampled": round(kt["force"][0], 4),
            "force_launches_sampled": kt["force"][1],
        },
        "roofline": roofline(main_run, args.precision, args.workload, args.skin),
        "fp64_plain_single_replica": plain,
        "cpu_baseline": cpu,
        "other_configs": configs,
        "fp32_free_energy_check": dF,
    }
    if plain:
        out["batched_fp32_over_plain_fp64"] = value / plain["value"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # default: the 2000-step equilibration untimed, then every remaining step of
    # the protocol (forward switch, hold, backward switch) timed
    ap.add_argument("--steps", type=int, default=42000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--grid", type=int, default=-1,
                    help="pair-pass grid in blocks (0: one block per staged slice; -1: the library's default), "
                         "with --lanes and --no-autotune to repeat a tuned launch")
    ap.add_argument("--skin", type=float, default=0.65)   # fastest of a 0.35..1.2 sweep on the 64-replica batch
    ap.add_argument("--timing-stride", type=int, default=None,
                    help="iterations between event-timed force passes in the timed region (0: none)")
    ap.add_argument("--list-builder", default="auto", choices=["auto", "lds", "global"],
                    help="neighbour rows of small replicas built from LDS or all in global memory "
                         "(auto: the autotuner's choice, else LDS)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads' bounded runs")
    ap.add_argument("--no-dF", action="store_true",
                    help="skip the FP32 against FP64 free-energy check on the stable batch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration * 131072, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(replicas would shard across GPUs with only a final gather of the work traces)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    main_run = run_gpu(args.workload, args.precision, args.steps, args.warmup, args.lanes, args.block,
                       not args.no_autotune, args.skin, stride=args.timing_stride, list_builder=args.list_builder,
                       grid=args.grid)
    plain = None
    if not args.no_fp64:
        pr = run_gpu("fl_mid", "fp64", 2000, 500, 0, 0, True, args.skin, only=[0], stride=0)
        plain = {
            "value": pr["natoms"] * 2000 / (pr["ms"] / 1e3), "unit": "atom-steps/s",
            "workload": "one FL replica, bcc 10^3 (2000 atoms), T=1400 K, k=3, FP64, autotuned launch",
            "ms_per_step": pr["ms"] / 2000,
        }
    configs = None if args.no_configs else run_configs(args.skin)
    dF = None if args.no_dF else free_energy_check()
    cpu = None if args.no_cpu else cpu_baseline()
    print(json.dumps(result_line(args, main_run, plain, cpu, configs, dF)), flush=True)


if __name__ == "__main__":
    main()
