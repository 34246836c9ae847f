"""Python binding of the C ABI in include/eamfe.h (ctypes; argument marshalling only).

Device arrays are torch tensors on a ROCm device, float64, SoA [3, N]
(positions, velocities, forces) or flat; the library reads and writes them
through data_ptr() on torch's current HIP stream.  Every computation happens
in the HIP library; if it is not built this module raises on import of the
library (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeamfe.so")

FP64, FP32 = 0, 1
MODES = {"fl": 0, "rs": 1, "hh": 2, "ein_rs": 3}
ERRORS = {
    0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EBOX",
    6: "ENEIGH_OVERFLOW", 7: "ECELL_OVERFLOW", 8: "ETABLE_RANGE", 9: "ENONFINITE",
}


class EamfeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Replica(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("pad_", C.c_int32), ("box", C.c_double * 3), ("T", C.c_double),
                ("k", C.c_double), ("k2", C.c_double), ("mass", C.c_double), ("seed", C.c_uint64)]


class Protocol(C.Structure):
    _fields_ = [("mode", C.c_int32), ("function", C.c_int32), ("fix_com", C.c_int32), ("n_eq", C.c_int32),
                ("n_sw", C.c_int32), ("n_hold", C.c_int32), ("n_hold2", C.c_int32), ("pad_", C.c_int32),
                ("dt", C.c_double), ("damp", C.c_double), ("lambda_f", C.c_double), ("skin", C.c_double)]


class Barostat(C.Structure):
    _fields_ = [("p0", C.c_double), ("tau_p", C.c_double), ("beta_T", C.c_double), ("dt", C.c_double),
                ("aniso", C.c_int32), ("pad_", C.c_int32)]


_dp = C.POINTER(C.c_double)
_lib = None


def lib():
    """Load the built library; raise if it is missing (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "eamfe_create": (i32, [C.POINTER(vp), i32, vp, i32, i32]),
        "eamfe_workspace_bytes": (i32, [vp, C.POINTER(C.c_size_t)]),
        "eamfe_set_workspace": (i32, [vp, vp, C.c_size_t]),
        "eamfe_resume_step": (i32, [vp, C.POINTER(i64)]),
        "eamfe_device_allocations": (i32, [vp, C.POINTER(i64)]),
        "eamfe_destroy": (i32, [vp]),
        "eamfe_last_error": (C.c_char_p, [vp]),
        "eamfe_set_stream": (i32, [vp, vp]),
        "eamfe_set_launch": (i32, [vp, i32, i32]),
        "eamfe_get_launch": (i32, [vp, C.POINTER(i32), C.POINTER(i32)]),
        "eamfe_set_grid": (i32, [vp, i32]),
        "eamfe_set_graph": (i32, [vp, i32]),
        "eamfe_get_grid": (i32, [vp, C.POINTER(i32)]),
        "eamfe_set_xcd_affinity": (i32, [vp, i32]),
        "eamfe_set_list_builder": (i32, [vp, i32]),
        "eamfe_get_list_builder": (i32, [vp, C.POINTER(i32)]),
        "eamfe_check": (i32, [vp]),
        "eamfe_set_kernel_timing": (i32, [vp, i32, i32]),
        "eamfe_autotune": (i32, [vp, C.POINTER(Protocol), i64, vp, vp, i32, C.POINTER(i32), C.POINTER(i32), _dp]),
        "eamfe_kernel_timing": (i32, [vp, _dp, C.POINTER(i64)]),
        "eamfe_list_stats": (i32, [vp, _dp, C.POINTER(i32), C.POINTER(i32)]),
        "eamfe_row_history": (i32, [vp, _dp, C.POINTER(i64), i32]),
        "eamfe_list_rebuilds": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
        "eamfe_msd": (i32, [vp, vp, _dp]),
        "eamfe_set_spring_scale": (i32, [vp, vp]),
        "eamfe_pressure": (i32, [vp, vp, vp, _dp]),
        "eamfe_barostat_step": (i32, [vp, C.POINTER(Barostat), i64, dbl, vp, vp, _dp, _dp]),
        "eamfe_get_boxes": (i32, [vp, _dp]),
        "eamfe_copy_lists": (i32, [vp, vp, vp, i32]),
        "eam_setup": (i32, [vp, i32, dbl, _dp, _dp, i32, dbl, _dp]),
        "eamfe_system_setup": (i32, [vp, i32, C.POINTER(Replica), vp]),
        "neigh_build": (i32, [vp, vp, dbl, i32]),
        "eam_forces": (i32, [vp, vp, vp, vp, vp]),
        "eamfe_init_velocities": (i32, [vp, vp, i32]),
        "eamfe_lambda_schedule": (i32, [C.POINTER(Protocol), _dp, C.POINTER(i64)]),
        "run_switching": (i32, [vp, C.POINTER(Protocol), i64, i64, vp, vp, vp, vp, vp, i32]),
        "switch_step": (i32, [vp, C.POINTER(Protocol), i64, vp, vp, vp, vp]),
        "eamfe_get_work": (i32, [vp, _dp]),
        "eamfe_get_state": (i32, [vp, _dp, vp, _dp]),
        "eamfe_set_state": (i32, [vp, _dp, vp, dbl]),
        "eamfe_set_chunk": (i32, [vp, i64]),
        "eamfe_replays": (i32, [vp, C.POINTER(i64)]),
        "eamfe_adjoint_theta": (i32, [vp, vp, _dp, i32, vp]),
        "eamfe_set_adjoint_sampling": (i32, [vp, i32, _dp, i32, vp]),
        "eamfe_adjoint_samples": (i32, [vp, C.POINTER(i64)]),
        "eamfe_einstein_free_energy": (dbl, [dbl, dbl, dbl, dbl]),
        "eamfe_spring_constant": (dbl, [dbl, dbl]),
        "eamfe_fixed_cm_correction": (dbl, [dbl, dbl, dbl, dbl]),
        "eamfe_fl_free_energy": (i32, [i32, _dp, _dp, dbl, dbl, dbl, dbl, dbl, dbl, i32, _dp, _dp, _dp]),
        "eamfe_rs_free_energy": (i32, [C.POINTER(Protocol), _dp, dbl, dbl, dbl, i32, _dp, _dp]),
        "eamfe_rs_free_energy_cm": (i32, [C.POINTER(Protocol), _dp, dbl, dbl, dbl, dbl, dbl, i32, _dp, _dp]),
        "eamfe_jarzynski": (i32, [i32, _dp, dbl, _dp, _dp]),
        "eamfe_switch_works": (i32, [C.POINTER(Protocol), i32, _dp, i64, _dp, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def protocol(mode="fl", n_eq=0, n_sw=1, n_hold=0, n_hold2=0, function=2, lambda_f=1.0, dt=0.001, damp=0.1,
             fix_com=True, skin=0.3) -> Protocol:
    return Protocol(MODES[mode] if isinstance(mode, str) else int(mode), int(function), int(bool(fix_com)),
                    int(n_eq), int(n_sw), int(n_hold), int(n_hold2), 0, float(dt), float(damp), float(lambda_f),
                    float(skin))


def protocol_from_schedule(sch, skin=0.3) -> Protocol:
    """From paper_2201_04622_amd.inputs.Schedule."""
    return protocol(sch.mode, sch.n_eq, sch.n_sw, sch.n_hold, sch.n_hold2, sch.function, sch.lambda_f, sch.dt,
                    sch.damp, sch.fix_com, skin)


def lambda_schedule(p: Protocol) -> np.ndarray:
    S = C.c_int64()
    _chk(None, lib().eamfe_lambda_schedule(C.byref(p), None, C.byref(S)))
    lam = np.zeros(S.value + 1)
    _chk(None, lib().eamfe_lambda_schedule(C.byref(p), lam.ctypes.data_as(_dp), C.byref(S)))
    return lam


def spring_constant(msd, T):
    """k = 3 kB T / msd (Eq. msd), eV/A^2."""
    return lib().eamfe_spring_constant(float(msd), float(T))


def einstein_free_energy(n_eff, T, k, mass):
    return lib().eamfe_einstein_free_energy(float(n_eff), float(T), float(k), float(mass))


def fixed_cm_correction(N, V, T, k):
    return lib().eamfe_fixed_cm_correction(float(N), float(V), float(T), float(k))


def fl_free_energy(W_fwd, W_bwd, n_eff, T, k, mass, N=None, V=None):
    Wf = np.ascontiguousarray(W_fwd, dtype=np.float64)
    Wb = np.ascontiguousarray(W_bwd, dtype=np.float64)
    F0, Ed, err = C.c_double(), C.c_double(), C.c_double()
    add = N is not None and V is not None
    _chk(None, lib().eamfe_fl_free_energy(len(Wf), Wf.ctypes.data_as(_dp), Wb.ctypes.data_as(_dp), float(n_eff),
                                          float(N or 0), float(V or 0), float(T), float(k), float(mass), int(add),
                                          C.byref(F0), C.byref(Ed), C.byref(err)))
    return F0.value, Ed.value, err.value


def jarzynski(W, T):
    """(dF, standard error) of one switching leg's works (Eq. jarz)."""
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    dF, err = C.c_double(), C.c_double()
    _chk(None, lib().eamfe_jarzynski(len(Wc), Wc.ctypes.data_as(_dp), float(T), C.byref(dF), C.byref(err)))
    return dF.value, err.value


def switch_works(p: Protocol, W_trace):
    """(W_fwd, W_bwd) per replica from cumulative work traces [n_rep, S]."""
    W = np.ascontiguousarray(np.atleast_2d(W_trace), dtype=np.float64)
    Wf, Wb = np.zeros(W.shape[0]), np.zeros(W.shape[0])
    _chk(None, lib().eamfe_switch_works(C.byref(p), W.shape[0], W.ctypes.data_as(_dp), W.shape[1],
                                        Wf.ctypes.data_as(_dp), Wb.ctypes.data_as(_dp)))
    return Wf, Wb


def rs_free_energy_cm(p: Protocol, W_trace, F0_T0, T0, N, V, mass, T_grid):
    """Eq. rs for a run with the centre of mass held, from the free crystal's
    F0(T0) (Eq. fl + Eq. cm): F(T) on T_grid."""
    W = np.ascontiguousarray(W_trace, dtype=np.float64)
    Tg = np.ascontiguousarray(T_grid, dtype=np.float64)
    out = np.zeros_like(Tg)
    _chk(None, lib().eamfe_rs_free_energy_cm(C.byref(p), W.ctypes.data_as(_dp), float(F0_T0), float(T0),
                                             float(N), float(V), float(mass), len(Tg),
                                             Tg.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
    return out


def rs_free_energy(p: Protocol, W_trace, F0_T0, T0, n_eff, T_grid):
    W = np.ascontiguousarray(W_trace, dtype=np.float64)
    Tg = np.ascontiguousarray(T_grid, dtype=np.float64)
    out = np.zeros_like(Tg)
    _chk(None, lib().eamfe_rs_free_energy(C.byref(p), W.ctypes.data_as(_dp), float(F0_T0), float(T0), float(n_eff),
                                          len(Tg), Tg.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
    return out


def _chk(ctx, code, what=""):
    if code != 0:
        msg = lib().eamfe_last_error(ctx).decode() if ctx else what
        raise EamfeError(code, msg or what)


def _ptr(t, n=None, what="tensor"):
    """Device address of a contiguous float64 tensor on the GPU holding at
    least n elements (the library's kernels read or write that many; a
    shorter buffer is refused here, since the C ABI takes a bare pointer)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{what}: a contiguous float64 tensor on the GPU is expected")
    if n is not None and t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} elements, the call needs {n}")
    return C.c_void_p(t.data_ptr())


def to_soa(x_aos, device="cuda"):
    """[N, 3] host array -> float64 [3, N] device tensor."""
    import torch
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x_aos, dtype=np.float64).T), device=device).contiguous()


def from_soa(t) -> np.ndarray:
    return t.detach().cpu().numpy().T.copy()


ENOMEM = 2


class Context:
    """An eamfe_ctx on one device.  Methods are the ABI entry points.

    With ``workspace=True`` (the default) every device buffer of the context
    is carved from one torch uint8 tensor that this object owns (the
    library allocates no device memory): a call that needs more memory
    returns EAMFE_ENOMEM, the tensor is replaced by a larger one (the
    library moves the buffers over) and the call is repeated, a switching
    run from the step where it stopped.  ``deterministic`` selects the
    FP32 form's fixed-point per-atom sums (bitwise shape-independent) or
    plain float64 sums of the float32 partials."""

    def __init__(self, device: int = 0, precision: int = FP64, stream=None, deterministic: bool = True,
                 workspace: bool = True):
        import torch
        self._lib = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        code = self._lib.eamfe_create(C.byref(h), int(device), C.c_void_p(stream), int(precision),
                                      int(bool(deterministic)))
        if code:
            raise EamfeError(code, "eamfe_create failed")
        self._h = h
        self.precision = precision
        self.deterministic = bool(deterministic)
        self.n_rep = 0
        self.N = 0
        self.offsets = None
        self.knots = None          # the knots of the current tables (last eam_setup)
        self.table_version = 0     # counts eam_setup calls
        self._ws, self._ws_bytes = None, 0
        self._own_ws = bool(workspace)
        if self._own_ws:
            self._c(self._lib.eamfe_set_workspace(self._h, None, 0))

    def _grow(self):
        """Replace the workspace by one of the size the context asks for;
        False when it is already that large (then the failure is not a
        shortfall of workspace)."""
        if not self._own_ws:
            return False
        import torch
        need = C.c_size_t()
        self._c(self._lib.eamfe_workspace_bytes(self._h, C.byref(need)))
        if need.value <= self._ws_bytes:
            return False
        nbytes = max(need.value, self._ws_bytes + self._ws_bytes // 4)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        self._c(self._lib.eamfe_set_workspace(self._h, C.c_void_p(ws.data_ptr()), C.c_size_t(nbytes)))
        self._ws, self._ws_bytes = ws, nbytes   # the previous tensor is released after the move
        return True

    def _r(self, fn, *args):
        """Call entry point fn(ctx, *args), enlarging the workspace and
        repeating the call while it runs short."""
        while True:
            code = fn(self._h, *args)
            if code == ENOMEM and self._grow():
                continue
            return self._c(code)

    def workspace_bytes(self):
        """(bytes the context's buffers need, bytes of the workspace held)."""
        n = C.c_size_t()
        self._c(self._lib.eamfe_workspace_bytes(self._h, C.byref(n)))
        return n.value, self._ws_bytes

    def device_allocations(self):
        """hipMalloc calls the library itself has made for this context."""
        n = C.c_int64()
        self._c(self._lib.eamfe_device_allocations(self._h, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.eamfe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, code):
        _chk(self._h, code)

    # -- configuration -------------------------------------------------------
    def set_launch(self, lanes_per_atom=0, block_threads=0):
        self._c(self._lib.eamfe_set_launch(self._h, int(lanes_per_atom), int(block_threads)))

    def get_launch(self):
        a, b = C.c_int(), C.c_int()
        self._c(self._lib.eamfe_get_launch(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_graph(self, iters):
        self._c(self._lib.eamfe_set_graph(self._h, int(iters)))

    def set_grid(self, blocks):
        self._c(self._lib.eamfe_set_grid(self._h, int(blocks)))

    def get_grid(self):
        g = C.c_int()
        self._c(self._lib.eamfe_get_grid(self._h, C.byref(g)))
        return g.value

    def set_list_builder(self, lds: bool):
        """True: rows of replicas that fit one block's LDS built from LDS (default); False: all in global memory."""
        self._c(self._lib.eamfe_set_list_builder(self._h, int(bool(lds))))

    def get_list_builder(self):
        """"lds" or "global": the builder of the neighbour rows."""
        v = C.c_int()
        self._c(self._lib.eamfe_get_list_builder(self._h, C.byref(v)))
        return "lds" if v.value else "global"

    def set_xcd_affinity(self, on: bool):
        self._c(self._lib.eamfe_set_xcd_affinity(self._h, int(bool(on))))

    def check(self):
        self._c(self._lib.eamfe_check(self._h))

    def autotune(self, p: Protocol, step, x, v, trial_steps=20):
        a, b, ms = C.c_int(), C.c_int(), C.c_double()
        self._r(self._lib.eamfe_autotune, C.byref(p), int(step), _ptr(x, 3 * self.N, "x"), _ptr(v, 3 * self.N, "v"),
                int(trial_steps),
                                         C.byref(a), C.byref(b), C.byref(ms))
        return a.value, b.value, ms.value

    def set_kernel_timing(self, stride=1, kinds=("density", "force", "lists")):
        """Time the kernels of the first and then every stride-th iteration with
        HIP events (0 = off); kinds: which of density, force, lists."""
        mask = sum(1 << q for q, k in enumerate(("density", "force", "lists")) if k in kinds)
        self._c(self._lib.eamfe_set_kernel_timing(self._h, int(stride), int(mask)))

    def kernel_timing(self):
        """{'density'|'force'|'lists': (total ms, launches)} since timing was enabled."""
        ms = np.zeros(3)
        n = (C.c_int64 * 3)()
        self._c(self._lib.eamfe_kernel_timing(self._h, ms.ctypes.data_as(_dp), n))
        return {k: (float(ms[q]), int(n[q])) for q, k in enumerate(("density", "force", "lists"))}

    def copy_lists(self):
        """(row lengths [N], rows [N, cap]) as device int32 tensors."""
        import torch
        _, _, cap = self.list_stats()
        nnb = torch.zeros(self.N, dtype=torch.int32, device="cuda")
        nbr = torch.zeros(self.N, cap, dtype=torch.int32, device="cuda")
        self._c(self._lib.eamfe_copy_lists(self._h, C.c_void_p(nnb.data_ptr()), C.c_void_p(nbr.data_ptr()), cap))
        return nnb, nbr

    def pressure(self, x, v=None):
        """Per-replica diagonal pressure tensor [n_rep, 3] (eV/A^3) at x (and
        velocities v, or the configurational part only)."""
        out = np.zeros((self.n_rep, 3))
        self._r(self._lib.eamfe_pressure, _ptr(x, 3 * self.N, "x"), _ptr(v, 3 * self.N, "v"),
                out.ctypes.data_as(_dp))
        return out

    def barostat_step(self, b: Barostat, step, w_eam, x, v):
        """One stochastic cell-rescaling move at the step boundary ``step``
        (``w_eam``: weight of U_EAM in the Hamiltonian there): scales x,
        v and the boxes in place; returns (mu[n_rep, 3] per-axis factors,
        P[n_rep, 3] diagonal internal pressures, eV/A^3)."""
        mu, P = np.zeros((self.n_rep, 3)), np.zeros((self.n_rep, 3))
        self._r(self._lib.eamfe_barostat_step, C.byref(b), int(step), float(w_eam), _ptr(x, 3 * self.N, "x"),
                _ptr(v, 3 * self.N, "v"),
                mu.ctypes.data_as(_dp), P.ctypes.data_as(_dp))
        return mu, P

    def boxes(self):
        """Current box edges [n_rep, 3] (A)."""
        L = np.zeros((self.n_rep, 3))
        self._c(self._lib.eamfe_get_boxes(self._h, L.ctypes.data_as(_dp)))
        return L

    def set_spring_scale(self, s=None):
        """Per-atom spring scales s_i (device float64 [N_tot]; atom i's spring
        is k s_i) or None for uniform springs."""
        self._c(self._lib.eamfe_set_spring_scale(self._h, _ptr(s, self.N, "spring scales")))

    def msd(self, x):
        """Per-replica mean-squared displacement (A^2) of x from the lattice
        sites, centre of mass removed (Eq. msd)."""
        out = np.zeros(self.n_rep)
        self._c(self._lib.eamfe_msd(self._h, _ptr(x, 3 * self.N, "x"), out.ctypes.data_as(_dp)))
        return out

    def row_history(self, reset=False):
        """(mean row length over the step force passes since the last reset, passes)."""
        m, n = C.c_double(), C.c_int64()
        self._c(self._lib.eamfe_row_history(self._h, C.byref(m), C.byref(n), int(bool(reset))))
        return m.value, n.value

    def list_rebuilds(self):
        """(replica list rebuilds, atoms rebuilt) of the step passes since the
        last row-history reset."""
        r, a = C.c_int64(), C.c_int64()
        self._c(self._lib.eamfe_list_rebuilds(self._h, C.byref(r), C.byref(a)))
        return r.value, a.value

    def list_stats(self):
        m, mx, cap = C.c_double(), C.c_int(), C.c_int()
        self._c(self._lib.eamfe_list_stats(self._h, C.byref(m), C.byref(mx), C.byref(cap)))
        return m.value, mx.value, cap.value

    # -- ABI -----------------------------------------------------------------
    def eam_setup(self, knots):
        """knots: paper_2201_04622_amd.inputs.PotentialKnots."""
        phi = np.ascontiguousarray(knots.phi, dtype=np.float64)
        rho = np.ascontiguousarray(knots.rho, dtype=np.float64)
        F = np.ascontiguousarray(knots.embed, dtype=np.float64)
        self._r(self._lib.eam_setup, len(phi), float(knots.r_cut), phi.ctypes.data_as(_dp),
                                    rho.ctypes.data_as(_dp), len(F), float(knots.rho_max), F.ctypes.data_as(_dp))
        self.knots = knots
        self.table_version += 1

    def system_setup(self, replicas: Sequence, x0_soa):
        """replicas: inputs.Replica list; x0_soa: device float64 [3, N_tot]."""
        n_tot = sum(int(r.natoms) for r in replicas)
        if tuple(x0_soa.shape) != (3, n_tot):
            raise ValueError(f"system_setup: x0 has shape {tuple(x0_soa.shape)}, the replicas hold (3, {n_tot})")
        arr = (Replica * len(replicas))()
        for q, r in zip(arr, replicas):
            q.n_atoms = r.natoms
            for d in range(3):
                q.box[d] = float(r.box[d])
            q.T, q.k, q.k2, q.mass, q.seed = float(r.T), float(r.k), float(r.k2), float(r.mass), int(r.seed)
        self._r(self._lib.eamfe_system_setup, len(replicas), arr, _ptr(x0_soa))
        self.n_rep = len(replicas)
        self.N = int(x0_soa.shape[1])
        self.offsets = np.concatenate([[0], np.cumsum([r.natoms for r in replicas])])

    def neigh_build(self, x, skin=0.3, max_neighbors=0):
        self._r(self._lib.neigh_build, _ptr(x, 3 * self.N, "x"), float(skin), int(max_neighbors))

    def eam_forces(self, x, f=None, U=None, e_atom=None):
        self._r(self._lib.eam_forces, _ptr(x, 3 * self.N, "x"), _ptr(f, 3 * self.N, "f"), _ptr(U, self.n_rep, "U"),
                _ptr(e_atom, self.N, "e_atom"))

    def init_velocities(self, v, fix_com=True):
        self._c(self._lib.eamfe_init_velocities(self._h, _ptr(v, 3 * self.N, "v"), int(bool(fix_com))))

    def run_switching(self, p: Protocol, x, v, step_begin=0, step_end=None, lam_out=None, dHdl_out=None, W_out=None,
                      sync=True):
        if step_end is None:
            S = C.c_int64()
            _chk(None, self._lib.eamfe_lambda_schedule(C.byref(p), None, C.byref(S)))
            step_end = S.value
        S = C.c_int64()
        _chk(None, self._lib.eamfe_lambda_schedule(C.byref(p), None, C.byref(S)))
        args = (_ptr(x, 3 * self.N, "x"), _ptr(v, 3 * self.N, "v"), _ptr(lam_out, S.value + 1, "lam_out"),
                _ptr(dHdl_out, self.n_rep * S.value, "dHdl_out"), _ptr(W_out, self.n_rep * S.value, "W_out"))
        s0 = int(step_begin)
        while True:
            code = self._lib.run_switching(self._h, C.byref(p), s0, int(step_end), *args, int(bool(sync)))
            if code == ENOMEM and self._grow():
                r = C.c_int64()
                self._c(self._lib.eamfe_resume_step(self._h, C.byref(r)))
                if r.value >= 0:
                    s0 = r.value   # x, v and the work are the state at that step
                continue
            return self._c(code)

    def switch_step(self, p: Protocol, step, x, v, W, dHdl=None):
        self._r(self._lib.switch_step, C.byref(p), int(step), _ptr(x, 3 * self.N, "x"), _ptr(v, 3 * self.N, "v"),
                _ptr(W, self.n_rep, "W"), _ptr(dHdl, self.n_rep, "dHdl"))

    def set_chunk(self, steps):
        self._c(self._lib.eamfe_set_chunk(self._h, int(steps)))

    def replays(self):
        n = C.c_int64()
        self._c(self._lib.eamfe_replays(self._h, C.byref(n)))
        return n.value

    def get_work(self):
        W = np.zeros(self.n_rep)
        self._c(self._lib.eamfe_get_work(self._h, W.ctypes.data_as(_dp)))
        return W

    def get_state(self):
        """(work [n_rep], list reference positions (device [3, N_tot]), skin):
        with x, v and the step index, what a resumed run needs."""
        import torch
        W, skin = np.zeros(self.n_rep), C.c_double()
        xref = torch.zeros(3, self.N, dtype=torch.float64, device="cuda")
        self._c(self._lib.eamfe_get_state(self._h, W.ctypes.data_as(_dp), _ptr(xref), C.byref(skin)))
        return W, xref, skin.value

    def set_state(self, W, xref, skin):
        """Load a saved work vector and build the lists at the saved reference positions."""
        Wc = np.ascontiguousarray(W, dtype=np.float64)
        if Wc.size < self.n_rep:
            raise ValueError(f"set_state: {Wc.size} work values for {self.n_rep} replicas")
        self._r(self._lib.eamfe_set_state, Wc.ctypes.data_as(_dp), _ptr(xref, 3 * self.N, "xref"), float(skin))

    def adjoint_theta(self, x, dtheta, weights=None, reduce=False):
        """dtheta (device float64, [n_rep, 3, n] or [3, n] with reduce) += w_r dU_r/dtheta."""
        w = self._adjoint_weights(weights)
        self._r(self._lib.eamfe_adjoint_theta, _ptr(x, 3 * self.N, "x"), None if w is None else w.ctypes.data_as(_dp),
                int(bool(reduce)), _ptr(dtheta, self._dtheta_size(reduce), "dtheta"))

    def _adjoint_weights(self, weights):
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        if w is not None and w.size < self.n_rep:
            raise ValueError(f"adjoint: {w.size} weights for {self.n_rep} replicas")
        return w

    def _dtheta_size(self, reduce):
        """Elements of dU/dtheta: 3 functions x n knots, per replica unless reduced."""
        n = len(self.knots.phi) if getattr(self, "knots", None) is not None else 0
        return 3 * n * (1 if reduce else self.n_rep)

    def set_adjoint_sampling(self, every, dtheta=None, weights=None, reduce=False):
        w = self._adjoint_weights(weights)
        self._adj_keep = (dtheta, w)
        self._c(self._lib.eamfe_set_adjoint_sampling(self._h, int(every), None if w is None else w.ctypes.data_as(_dp),
                                                     int(bool(reduce)),
                                                     _ptr(dtheta, self._dtheta_size(reduce), "dtheta")))

    def adjoint_samples(self):
        n = C.c_int64()
        self._c(self._lib.eamfe_adjoint_samples(self._h, C.byref(n)))
        return n.value
