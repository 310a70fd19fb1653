"""ctypes front end of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None


class OraParams(C.Structure):
    _fields_ = [
        ("q", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("periodic", C.c_int32), ("open_x", C.c_int32),
        ("porous_x0", C.c_int32), ("porous_x1", C.c_int32),
        ("bc_set", C.c_int32), ("collision", C.c_int32),
        ("half_force_shift", C.c_int32), ("mrt_sj_mode", C.c_int32),
        ("tau", C.c_double * 2), ("G", C.c_double), ("xi", C.c_double),
        ("rho_in1", C.c_double), ("rho_out2", C.c_double),
        ("rho_in2", C.c_double), ("rho_out1", C.c_double),
        ("g", C.c_double * 3), ("lam", C.c_double),
        ("s_e", C.c_double), ("s_eps", C.c_double),
        ("eq26_mode", C.c_int32), ("ivsd_frozen", C.c_int32),
    ]


class OraObs(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass", C.c_double * 2), ("n_fluid", C.c_double),
        ("n_window", C.c_double), ("sw_count", C.c_double),
        ("sum_rho_w", C.c_double), ("sum_rho", C.c_double),
        ("s_w", C.c_double), ("s_w_weighted", C.c_double),
        ("p_in", C.c_double), ("p_out", C.c_double), ("pc", C.c_double),
        ("n_in", C.c_double), ("n_out", C.c_double),
        ("flux_in", C.c_double * 2), ("flux_out", C.c_double * 2),
        ("flags", C.c_int32), ("pad", C.c_int32), ("stag", C.c_double * 3),
    ]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [C.POINTER(OraParams), C.c_void_p, C.c_void_p, C.c_char_p]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_step.argtypes = [C.c_void_p, C.c_int64]
        L.ora_set_bc.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.ora_get_step.restype = C.c_int64
        L.ora_get_step.argtypes = [C.c_void_p]
        for name in ("ora_density", "ora_force", "ora_psi", "ora_get_fstar", "ora_set_fstar"):
            getattr(L, name).argtypes = [C.c_void_p, C.c_void_p]
        L.ora_observables.argtypes = [C.c_void_p, C.POINTER(OraObs)]
        L.ora_lattice.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp]
        L.ora_forcing.argtypes = [C.c_int, dp, dp, dp]
        L.ora_collide_node.argtypes = [C.POINTER(OraParams), dp, dp, dp]
        L.ora_zouhe.argtypes = [C.c_int, dp, C.c_double, C.c_int]
        L.ora_mrt_matrix.argtypes = [C.c_int, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(problem=None, **kw) -> OraParams:
    """OraParams from an inputs.Problem (or plain keywords)."""
    d = {}
    if problem is not None:
        p = problem
        d = dict(q=p.q, nx=p.nx, ny=p.ny, nz=p.nz, periodic=p.periodic, open_x=p.open_x,
                 porous_x0=p.porous_x0, porous_x1=p.porous_x1, bc_set=p.bc_set,
                 collision=p.collision, half_force_shift=p.half_force_shift,
                 mrt_sj_mode=p.mrt_sj_mode, tau=p.tau, G=p.G, xi=p.xi,
                 rho_in1=p.rho_in1, rho_out2=p.rho_out2, rho_in2=p.rho_in2,
                 rho_out1=p.rho_out1, g=p.g, lam=p.lam, s_e=p.s_e, s_eps=p.s_eps,
                 eq26_mode=p.eq26_mode, ivsd_frozen=p.ivsd_frozen)
    d.update(kw)
    P = OraParams()
    defaults = dict(q=9, nx=1, ny=1, nz=1, periodic=0, open_x=0, porous_x0=0, porous_x1=0,
                    bc_set=3, collision=0, half_force_shift=1, mrt_sj_mode=0,
                    tau=(1.0, 1.0), G=0.0, xi=0.0, rho_in1=1.0, rho_out2=1.0,
                    rho_in2=0.0, rho_out1=0.0, g=(0.0, 0.0, 0.0), lam=3.0 / 16.0,
                    s_e=1.0, s_eps=1.0, eq26_mode=0, ivsd_frozen=0)
    defaults.update(d)
    for k, v in defaults.items():
        if k == "tau":
            P.tau[0], P.tau[1] = float(v[0]), float(v[1])
        elif k == "g":
            for i in range(3):
                P.g[i] = float(v[i])
        else:
            setattr(P, k, v)
    return P


def lattice(q: int):
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, dtype=np.int32)
    if lib().ora_lattice(q, e.ctypes.data, w.ctypes.data, opp.ctypes.data):
        raise ValueError(q)
    return e, w, opp


def equilibrium(q, rho, u):
    u = np.asarray(u, dtype=np.float64).reshape(3).copy()
    out = np.zeros(q)
    lib().ora_equilibrium(q, float(rho), _dp(u), _dp(out))
    return out


def forcing(q, u, F):
    u = np.asarray(u, dtype=np.float64).reshape(3).copy()
    F = np.asarray(F, dtype=np.float64).reshape(3).copy()
    out = np.zeros(q)
    lib().ora_forcing(q, _dp(u), _dp(F), _dp(out))
    return out


def collide_node(params: OraParams, fin, F):
    q = params.q
    fin = np.ascontiguousarray(fin, dtype=np.float64).reshape(2 * q)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(6)
    out = np.zeros(2 * q)
    lib().ora_collide_node(C.byref(params), _dp(fin), _dp(F), _dp(out))
    return out.reshape(2, q)


def mrt_matrix(q):
    out = np.zeros(q * q)
    lib().ora_mrt_matrix(q, _dp(out))
    return out.reshape(q, q)


def zouhe(q, f, rho_bc, normal):
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    lib().ora_zouhe(q, _dp(f), float(rho_bc), int(normal))
    return f


class OracleSim:
    """One oracle simulation of an inputs.Problem (or explicit params)."""

    def __init__(self, problem=None, params: OraParams | None = None, mask=None, rho0=None):
        if params is None:
            params = make_params(problem)
        if mask is None:
            mask = problem.mask
        if rho0 is None:
            rho0 = problem.rho0
        self.params = params
        self.shape = mask.shape
        self.N = int(mask.size)
        self.q = params.q
        self._mask = np.ascontiguousarray(mask, dtype=np.uint8)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        err = C.create_string_buffer(256)
        self._h = lib().ora_create(C.byref(params), self._mask.ctypes.data,
                                   rho0.ctypes.data, err)
        if not self._h:
            raise ValueError(err.value.decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        lib().ora_step(self._h, int(n))

    def set_bc(self, rho_in1, rho_out2):
        lib().ora_set_bc(self._h, float(rho_in1), float(rho_out2))

    @property
    def t(self):
        return lib().ora_get_step(self._h)

    def density(self):
        out = np.zeros((2,) + self.shape)
        lib().ora_density(self._h, out.ctypes.data)
        return out

    def psi(self):
        out = np.zeros((2,) + self.shape)
        lib().ora_psi(self._h, out.ctypes.data)
        return out

    def force(self):
        out = np.zeros((2, 3) + self.shape)
        lib().ora_force(self._h, out.ctypes.data)
        return out

    def fstar(self):
        out = np.zeros((2, self.q) + self.shape)
        lib().ora_get_fstar(self._h, out.ctypes.data)
        return out

    def set_fstar(self, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        assert arr.size == 2 * self.q * self.N
        lib().ora_set_fstar(self._h, arr.ctypes.data)

    def observables(self) -> dict:
        o = OraObs()
        lib().ora_observables(self._h, C.byref(o))
        return o.to_dict()


def num_threads() -> int:
    return lib().ora_num_threads()
