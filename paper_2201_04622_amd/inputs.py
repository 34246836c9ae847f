"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds none of the method's arithmetic: no spline construction, no
EAM sums, no integrator, no lambda schedule and no free-energy estimator.  It
only produces the *inputs* a user of the method would bring:

* the tabulated potential: knot values of a synthetic analytic EAM (it stands in
  for the Fe potential the paper uses, Sec. "bulk", which is not available),
* crystal lattice sites (bcc / fcc cubic supercells, atom id = cell-major),
* randomly displaced configurations for force tests (numpy Generator, seeded),
* replica batches with their temperatures, spring constants and seeds.

Units are LAMMPS "metal": eV, Angstrom, ps, amu, K.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Synthetic analytic EAM (stands in for the paper's Fe potential)
# ---------------------------------------------------------------------------
R_CUT = 5.3          # Angstrom, outer cutoff of phi and rho
R_TAPER = 4.8        # Angstrom, start of the cosine taper
N_KNOTS = 2000       # knots per tabulated function
RHO_MAX = 200.0      # upper end of the embedding-function table
MASS_FE = 55.845     # amu

A_BCC_VERBATIM = 2.855   # lattice constants as configured (physical Fe values)
A_FCC_VERBATIM = 3.65
# Zero-pressure 0 K lattice constants of the synthetic potential itself, where
# both structures are mechanically stable (the verbatim ones are not).
A_BCC_STABLE = 1.9646
A_FCC_STABLE = 2.5216


def taper(r):
    """Cosine taper: 1 below R_TAPER, 0 above R_CUT, half-cosine in between."""
    r = np.asarray(r, dtype=np.float64)
    s = np.where(r <= R_TAPER, 1.0, 0.5 * (1.0 + np.cos(np.pi * (r - R_TAPER) / (R_CUT - R_TAPER))))
    return np.where(r >= R_CUT, 0.0, s)


def phi_analytic(r):
    r = np.asarray(r, dtype=np.float64)
    x = r / 2.48 - 1.0
    return (0.5 * np.exp(-7.0 * x) - 0.9 * np.exp(-3.5 * x)) * taper(r)


def rho_analytic(r):
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-6.0 * (r / 2.48 - 1.0)) * taper(r)


def embed_analytic(rho):
    return -2.0 * np.sqrt(np.asarray(rho, dtype=np.float64))


@dataclass(frozen=True)
class PotentialKnots:
    """Knot values on uniform grids: r_k = k*r_cut/(n-1), rho_k = k*rho_max/(n-1)."""
    r_cut: float
    rho_max: float
    phi: np.ndarray   # [n] eV
    rho: np.ndarray   # [n]
    embed: np.ndarray  # [n] eV

    @property
    def n(self) -> int:
        return int(self.phi.shape[0])

    def stacked(self) -> np.ndarray:
        """[3][n] in the order (phi, rho, F)."""
        return np.stack([self.phi, self.rho, self.embed]).astype(np.float64)


def synthetic_eam_knots(n: int = N_KNOTS, r_cut: float = R_CUT, rho_max: float = RHO_MAX) -> PotentialKnots:
    r = np.arange(n, dtype=np.float64) * (r_cut / (n - 1))
    rho = np.arange(n, dtype=np.float64) * (rho_max / (n - 1))
    return PotentialKnots(r_cut, rho_max, phi_analytic(r), rho_analytic(r), embed_analytic(rho))


# ---------------------------------------------------------------------------
# Lattices
# ---------------------------------------------------------------------------
# Basis of each lattice's conventional cell in fractional coordinates, and
# the cell's edges in units of the lattice parameter a.  hcp uses the
# orthorhombic cell (a, sqrt(3) a, c) of two close-packed layers with the
# ideal c = sqrt(8/3) a, so every site has 12 neighbours at distance a.
BASIS = {
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "fcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]),
    "hcp": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 5.0 / 6.0, 0.5], [0.0, 1.0 / 3.0, 0.5]]),
}
CELL = {
    "bcc": np.array([1.0, 1.0, 1.0]),
    "fcc": np.array([1.0, 1.0, 1.0]),
    "hcp": np.array([1.0, np.sqrt(3.0), np.sqrt(8.0 / 3.0)]),
}


def cell_counts(n) -> tuple:
    """Cells per axis: n for a cube of n^3 cells, or (nx, ny, nz)."""
    if np.isscalar(n):
        return (int(n),) * 3
    nx, ny, nz = (int(v) for v in n)
    return nx, ny, nz


def lattice_sites(kind: str, n, a: float) -> np.ndarray:
    """Sites of a supercell of nx x ny x nz conventional cells (n an int for a
    cube), shape [N, 3], id = ((ix*ny+iy)*nz+iz)*nb + b."""
    nx, ny, nz = cell_counts(n)
    basis = BASIS[kind]
    cells = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), axis=-1).reshape(-1, 3)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * (CELL[kind] * a)
    return np.ascontiguousarray(pos, dtype=np.float64)


# ---------------------------------------------------------------------------
# Replicas and workloads
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Replica:
    kind: str            # "bcc" | "fcc" | "hcp"
    n: int               # conventional cells per edge (a cube); see cells
    a: float             # lattice constant (Angstrom)
    T: float             # thermostat temperature (K)
    k: float             # Einstein spring constant (eV/A^2); k1 for the harmonic test mode
    seed: int            # Philox key
    mass: float = MASS_FE
    k2: float = 0.0      # second spring constant (harmonic -> harmonic test mode only)
    cells: tuple = None  # (nx, ny, nz) conventional cells of an orthorhombic supercell; None: n per edge
    vacuum: float = 0.0  # empty space added to the box along z (A): a slab with two free z faces
    vacancies: tuple = ()  # site ids (of the full supercell) left empty: point defects
    c_over_a: float = None  # hcp only: c / a of the cell (None: the ideal sqrt(8/3))

    @property
    def dims(self) -> tuple:
        return cell_counts(self.n if self.cells is None else self.cells)

    @property
    def natoms(self) -> int:
        return len(BASIS[self.kind]) * int(np.prod(self.dims)) - len(set(self.vacancies))

    def _zscale(self) -> float:
        if self.c_over_a is None:
            return 1.0
        if self.kind != "hcp":
            raise ValueError("c_over_a applies to hcp only")
        return float(self.c_over_a) / float(CELL["hcp"][2])

    @property
    def box(self) -> np.ndarray:
        L = np.asarray(self.dims, dtype=np.float64) * CELL[self.kind] * self.a
        L[2] *= self._zscale()
        L[2] += self.vacuum
        return L

    def sites(self) -> np.ndarray:
        x = lattice_sites(self.kind, self.dims, self.a)
        x[:, 2] *= self._zscale()
        if self.vacancies:
            keep = np.ones(len(x), dtype=bool)
            keep[list(set(self.vacancies))] = False
            x = np.ascontiguousarray(x[keep])
        return x


@dataclass(frozen=True)
class Schedule:
    """Segment lengths of a switching run (steps).  mode: "fl" | "rs" | "hh" | "ein_rs"."""
    mode: str
    n_eq: int
    n_sw: int
    n_hold: int
    n_hold2: int
    function: int = 2          # lambda(tau) form for FL/HH: 1 linear, 2 smooth-step polynomial
    lambda_f: float = 1.0      # RS end point lambda_f = T0 / T_f
    dt: float = 0.001          # ps
    damp: float = 0.1          # ps (gamma = 1/damp)
    fix_com: bool = True

    @property
    def total_steps(self) -> int:
        return self.n_eq + 2 * self.n_sw + self.n_hold + self.n_hold2


@dataclass
class Workload:
    name: str
    replicas: List[Replica]
    schedule: Schedule
    description: str = ""

    @property
    def natoms(self) -> int:
        return sum(r.natoms for r in self.replicas)

    @property
    def atom_steps(self) -> int:
        return self.natoms * self.schedule.total_steps


def _batch_shapes(a_bcc: float, a_fcc: float):
    return [("bcc", n, a_bcc) for n in range(6, 13)] + [("fcc", n, a_fcc) for n in range(5, 11)]


def workload(name: str, stable: bool = False) -> Workload:
    """The workloads, by name:

    fl_bcc4   FL in FP64, one bcc 4^3 replica (128 atoms), T=100 K, k=5
    fl_mid    FL, one bcc 10^3 (2000) and one fcc 8^3 (2048) replica, T=1400 K, k=3
    batch64   64 FL replicas of uneven size (bcc 6..12^3, fcc 5..10^3; 113,090
              atoms), T = 100 (1 + r mod 16) K, k=5, seeds 0..63
    rs_scan   RS scan 100 -> 1600 K, 8 bcc 20^3 replicas (128,000 atoms)
    rs_small  RS scan 300 -> 600 K, 4 bcc 6^3 replicas (1,728 atoms), k=20
    fl_large  FL, 16 bcc 30^3 + 16 fcc 24^3 replicas (1,748,736 atoms), T=1200 K

    ``stable`` swaps in the synthetic
    potential's own zero-pressure lattice constants (and the smallest box that
    keeps L > 2*(r_cut + skin))."""
    ab = A_BCC_STABLE if stable else A_BCC_VERBATIM
    af = A_FCC_STABLE if stable else A_FCC_VERBATIM
    if name == "fl_bcc4":
        n = 6 if stable else 4
        reps = [Replica("bcc", n, ab, 100.0, 5.0, 0)]
        sch = Schedule("fl", 1000, 2000, 500, 500, function=2)
        desc = f"FL FP64, 1 x bcc {n}^3, T=100 K, k=5"
    elif name == "fl_mid":
        reps = [Replica("bcc", 10, ab, 1400.0, 3.0, 0), Replica("fcc", 8, af, 1400.0, 3.0, 0)]
        sch = Schedule("fl", 10000, 50000, 10000, 10000, function=2)
        desc = "FL single replicas bcc 10^3 / fcc 8^3, T=1400 K, k=3"
    elif name == "batch64":
        shapes = _batch_shapes(ab, af)
        reps = []
        for r in range(64):
            kind, n, a = shapes[r % len(shapes)]
            reps.append(Replica(kind, n, a, 100.0 * (1 + (r % 16)), 5.0, r))
        sch = Schedule("fl", 2000, 20000, 2000, 0, function=2)
        desc = "64 batched FL replicas, bcc 6..12^3 / fcc 5..10^3, T in 100..1600 K, k=5"
    elif name == "rs_scan":
        reps = [Replica("bcc", 20, ab, 100.0, 5.0, s) for s in range(8)]
        sch = Schedule("rs", 10000, 100000, 10000, 0, lambda_f=100.0 / 1600.0)
        desc = "RS scan 100->1600 K, 8 x bcc 20^3"
    elif name == "rs_small":
        n = 6 if stable else 4
        reps = [Replica("bcc", n, ab, 300.0, 20.0, s) for s in range(4)]
        sch = Schedule("rs", 1000, 8000, 1000, 0, lambda_f=0.5)
        desc = f"RS scan 300->600 K, 4 x bcc {n}^3"
    elif name == "fl_large":
        reps = [Replica("bcc", 30, ab, 1200.0, 5.0, s) for s in range(16)]
        reps += [Replica("fcc", 24, af, 1200.0, 5.0, s) for s in range(16)]
        sch = Schedule("fl", 3000, 30000, 3000, 0, function=2)
        desc = "FL for dF/dtheta, 16 x bcc 30^3 + 16 x fcc 24^3, T=1200 K"
    else:
        raise ValueError(f"unknown workload {name!r}")
    return Workload(name + ("_stable" if stable else ""), reps, sch, desc)


def batch_arrays(replicas: Sequence[Replica]):
    """Concatenate replica descriptions into flat host arrays.

    Returns dict with n_atoms[int32 R], box[float64 R,3], x0[float64 N_tot,3]
    (AoS, replica-major), T, k, k2, mass [float64 R], seed [uint64 R].
    """
    x0 = np.concatenate([r.sites() for r in replicas], axis=0)
    return {
        "n_atoms": np.array([r.natoms for r in replicas], dtype=np.int32),
        "box": np.stack([r.box for r in replicas]).astype(np.float64),
        "x0": np.ascontiguousarray(x0, dtype=np.float64),
        "T": np.array([r.T for r in replicas], dtype=np.float64),
        "k": np.array([r.k for r in replicas], dtype=np.float64),
        "k2": np.array([r.k2 for r in replicas], dtype=np.float64),
        "mass": np.array([r.mass for r in replicas], dtype=np.float64),
        "seed": np.array([r.seed for r in replicas], dtype=np.uint64),
    }


def displaced(x0: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """x0 + N(0, sigma^2) per component, numpy PCG64 seeded by ``seed``."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(x0 + sigma * rng.standard_normal(x0.shape), dtype=np.float64)


def random_velocities(n: int, scale: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(scale * rng.standard_normal((n, 3)), dtype=np.float64)
