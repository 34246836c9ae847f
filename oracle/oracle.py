"""ctypes front end of the FP64 CPU oracle (``eam_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
Arrays on this side are AoS ``[N, 3]`` float64 (the HIP library uses SoA).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

FL, RS, HH, EIN_RS = 0, 1, 2, 3
MODES = {"fl": FL, "rs": RS, "hh": HH, "ein_rs": EIN_RS}
ETABLE, EBOX = 4, 8

_dp = C.POINTER(C.c_double)


class _Params(C.Structure):
    _fields_ = [
        ("mode", C.c_int), ("fix_com", C.c_int),
        ("T", C.c_double), ("gamma", C.c_double), ("dt", C.c_double), ("mass", C.c_double),
        ("k", C.c_double), ("k2", C.c_double), ("seed", C.c_uint64),
        ("skin", C.c_double), ("nlist_cap", C.c_int),
    ]


_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    src = os.path.join(_HERE, "eam_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        import subprocess
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_spline_natural.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.orc_spline_eval.argtypes = [C.c_int, C.c_double, _dp, C.c_double, _dp]
        L.orc_spline_eval.restype = C.c_double
        L.orc_pot_create.argtypes = [C.c_int, C.c_double, _dp, _dp, C.c_int, C.c_double, _dp]
        L.orc_pot_create.restype = C.c_void_p
        L.orc_pot_free.argtypes = [C.c_void_p]
        L.orc_pot_coefficients.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_eam.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_pressure.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_eam_atom.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_int, _dp, _dp, _dp]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, _dp]
        L.orc_lambda_fl.argtypes = [C.c_int, C.c_double]
        L.orc_lambda_fl.restype = C.c_double
        L.orc_lambda_rs.argtypes = [C.c_double, C.c_double]
        L.orc_lambda_rs.restype = C.c_double
        L.orc_schedule.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, _dp]
        L.orc_init_velocities.argtypes = [C.POINTER(_Params), C.c_int, _dp]
        L.orc_run.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_int, _dp, _dp, _dp, _dp, C.c_int, _dp,
                              C.c_int64, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_adjoint_theta.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------------------
def spline_coefficients(y, h):
    y = _f64(y)
    c = np.zeros((len(y) - 1, 4))
    st = lib().orc_spline_natural(len(y), float(h), _p(y), _p(c))
    if st:
        raise ValueError("spline: bad input")
    return c


def spline_eval(coef, h, x):
    coef = _f64(coef)
    n = coef.shape[0] + 1
    d = C.c_double()
    v = lib().orc_spline_eval(n, float(h), _p(coef), float(x), C.byref(d))
    return v, d.value


class Potential:
    """Tabulated EAM (phi, rho on [0, r_cut]; F on [0, rho_max])."""

    def __init__(self, phi, rho, F, r_cut, rho_max):
        self.phi_knots, self.rho_knots, self.F_knots = _f64(phi), _f64(rho), _f64(F)
        self.r_cut, self.rho_max = float(r_cut), float(rho_max)
        self.n_r, self.n_rho = len(self.phi_knots), len(self.F_knots)
        self._h = lib().orc_pot_create(self.n_r, self.r_cut, _p(self.phi_knots), _p(self.rho_knots),
                                       self.n_rho, self.rho_max, _p(self.F_knots))
        if not self._h:
            raise ValueError("orc_pot_create failed")

    @classmethod
    def from_knots(cls, knots):
        return cls(knots.phi, knots.rho, knots.embed, knots.r_cut, knots.rho_max)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_pot_free(h)
            self._h = None

    def coefficients(self):
        a = np.zeros((self.n_r - 1, 4)); b = np.zeros((self.n_r - 1, 4)); c = np.zeros((self.n_rho - 1, 4))
        lib().orc_pot_coefficients(self._h, _p(a), _p(b), _p(c))
        return a, b, c

    def eam(self, x, L):
        """Returns dict U, f[N,3], e_atom[N], rho[N], Fp[N], status."""
        x = _f64(x, (-1, 3)); L = _f64(L, (3,))
        N = x.shape[0]
        f = np.zeros((N, 3)); e = np.zeros(N); rho = np.zeros(N); Fp = np.zeros(N); U = np.zeros(1)
        st = lib().orc_eam(self._h, N, _p(x), _p(L), _p(f), _p(U), _p(e), _p(rho), _p(Fp))
        if st & EBOX:
            raise ValueError("box too small for a single periodic image")
        return {"U": float(U[0]), "f": f, "e_atom": e, "rho": rho, "Fp": Fp, "status": st}

    def pressure(self, x, L, v=None, mass=55.845):
        """Diagonal pressure tensor P_aa = (sum m v_a^2 + W_aa) / V, eV/A^3."""
        x = _f64(x, (-1, 3)); L = _f64(L, (3,))
        vv = None if v is None else _f64(v, (-1, 3))
        P = np.zeros(3)
        st = lib().orc_pressure(self._h, x.shape[0], _p(x), _p(vv), float(mass), _p(L), _p(P))
        if st & EBOX:
            raise ValueError("box too small for a single periodic image")
        return P

    def eam_atom(self, x, L, i):
        x = _f64(x, (-1, 3)); L = _f64(L, (3,))
        f = np.zeros(3); e = np.zeros(1); r = np.zeros(1)
        st = lib().orc_eam_atom(self._h, x.shape[0], _p(x), _p(L), int(i), _p(f), _p(e), _p(r))
        return {"f": f, "e_atom": float(e[0]), "rho": float(r[0]), "status": st}

    def adjoint_theta(self, x, L):
        """dU/d(knot values), [3][n] in the order (phi, rho, F) (n_r == n_rho assumed)."""
        x = _f64(x, (-1, 3)); L = _f64(L, (3,))
        g = np.zeros(2 * self.n_r + self.n_rho)
        st = lib().orc_adjoint_theta(self._h, x.shape[0], _p(x), _p(L), _p(g))
        if st & ~ETABLE:
            raise RuntimeError(f"adjoint failed: {st}")
        return np.stack([g[: self.n_r], g[self.n_r: 2 * self.n_r], g[2 * self.n_r:]])


# ---------------------------------------------------------------------------
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def gauss3(seed, atom, step, stream):
    z = np.zeros(3)
    lib().orc_gauss3(int(seed), int(atom), int(step), int(stream), _p(z))
    return z


def lambda_fl(function, tau):
    return lib().orc_lambda_fl(int(function), float(tau))


def lambda_rs(lambda_f, tau):
    return lib().orc_lambda_rs(float(lambda_f), float(tau))


def schedule(mode, n_eq, n_sw, n_hold, n_hold2, function=2, lambda_f=1.0):
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    S = n_eq + 2 * n_sw + n_hold + n_hold2
    lam = np.zeros(S + 1)
    st = lib().orc_schedule(m, int(function), float(lambda_f), n_eq, n_sw, n_hold, n_hold2, _p(lam))
    if st:
        raise ValueError("bad schedule")
    return lam


@dataclass
class RunParams:
    mode: str = "fl"
    T: float = 100.0
    gamma: float = 10.0
    dt: float = 0.001
    mass: float = 55.845
    k: float = 5.0
    k2: float = 0.0
    seed: int = 0
    fix_com: bool = True
    skin: float = 0.0       # > 0: Verlet candidate list (rebuilt on skin/2 displacement)
    nlist_cap: int = 512

    def c(self):
        return _Params(MODES[self.mode], int(self.fix_com), self.T, self.gamma, self.dt, self.mass,
                       self.k, self.k2, int(self.seed), self.skin, self.nlist_cap)


def init_velocities(params: RunParams, N: int):
    v = np.zeros((N, 3))
    P = params.c()
    lib().orc_init_velocities(C.byref(P), N, _p(v))
    return v


def run(pot, params: RunParams, x0, L, x, v, lam, step0=0, W0=0.0, energies=False, spring_scale=None):
    """Advance (x, v) in place over len(lam)-1 steps.  Returns dHdl[S], W[S], e[S] or None, status.
    spring_scale: per-atom factors s_i of the spring constant (atom i's spring is k s_i), or None."""
    x0 = _f64(x0, (-1, 3)); L = _f64(L, (3,)); lam = _f64(lam)
    assert x.dtype == np.float64 and x.flags.c_contiguous and v.dtype == np.float64 and v.flags.c_contiguous
    N = x0.shape[0]
    S = len(lam) - 1
    dH = np.zeros(S); W = np.zeros(S); e = np.zeros(S) if energies else None
    P = params.c()
    hp = pot._h if pot is not None else None
    if hp is None and params.mode in ("fl", "rs"):
        raise ValueError("EAM modes need a potential")
    ks = None if spring_scale is None else _f64(spring_scale, (N,))
    st = lib().orc_run(hp, C.byref(P), N, _p(x0), _p(L), _p(x), _p(v), S, _p(lam), int(step0), float(W0),
                       _p(dH), _p(W), _p(e), _p(ks))
    if st & EBOX:
        raise ValueError("box too small")
    if st & ~ETABLE:
        raise RuntimeError(f"oracle run failed: status {st}")
    return dH, W, e, st
