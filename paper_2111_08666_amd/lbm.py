"""Python binding of liblbm.so: argument marshalling only.

Every step of the method runs in the library's HIP kernels; torch provides
the device workspace and the stream.  The library must be built in-tree
(`python -m paper_2111_08666_amd.build`); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
SRT, MRT, TRT = 0, 1, 2
STORE_F32, STORE_BF16DEV = 0, 1
MATH_F32, MATH_F64 = 0, 1
AUTO, FUSED, SPLIT, COMPACT, FUSED_LIST, COMPACT_FUSED = 0, 1, 2, 3, 4, 5

EXPORTS = [
    "lbm_workspace_bytes", "lbm_create", "lbm_set_bc", "lbm_step", "lbm_step_graph",
    "lbm_observables", "lbm_get_density", "lbm_init_from_saturation", "lbm_debug_poke", "lbm_save", "lbm_load",
    "lbm_get_step",
    "lbm_destroy", "lbm_last_error", "lbm_kernel_info", "lbm_autotune", "lbm_batch_workspace_bytes",
    "lbm_batch_create", "lbm_batch_step", "lbm_batch_step_graph", "lbm_batch_observables",
    "lbm_batch_get_density", "lbm_batch_destroy", "lbm_batch_last_error", "lbm_batch_kernel_info",
    "lbm_batch_autotune", "lbm_batch_set_active",
]


class Geometry(C.Structure):
    _fields_ = [("q", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("solid", C.c_void_p), ("periodic", C.c_uint32), ("open_x", C.c_int32),
                ("porous_x0", C.c_int32), ("porous_x1", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("tau", C.c_double * 2), ("G", C.c_double), ("xi", C.c_double),
                ("rho_in1", C.c_double), ("rho_out2", C.c_double),
                ("rho_in2", C.c_double), ("rho_out1", C.c_double),
                ("g", C.c_double * 3), ("collision", C.c_int32), ("bc_set", C.c_int32),
                ("half_force_shift", C.c_int32), ("mrt_sj_mode", C.c_int32),
                ("lam", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double),
                ("storage", C.c_int32), ("math", C.c_int32),
                ("strategy", C.c_int32), ("tile_rows", C.c_int32), ("eq26_mode", C.c_int32),
                ("ivsd_frozen", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double * 2), ("n_fluid", C.c_double),
                ("n_window", C.c_double), ("sw_count", C.c_double),
                ("sum_rho_w", C.c_double), ("sum_rho", C.c_double),
                ("s_w", C.c_double), ("s_w_weighted", C.c_double),
                ("p_in", C.c_double), ("p_out", C.c_double), ("pc", C.c_double),
                ("n_in", C.c_double), ("n_out", C.c_double),
                ("flags", C.c_int32), ("reserved", C.c_int32), ("stag", C.c_double * 3)]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2111_08666_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        G, P = C.POINTER(Geometry), C.POINTER(Params)
        L.lbm_workspace_bytes.restype = sz
        L.lbm_workspace_bytes.argtypes = [G, P]
        L.lbm_create.argtypes = [G, P, vp, vp, sz, vp, C.POINTER(vp)]
        L.lbm_set_bc.argtypes = [vp, C.c_double, C.c_double]
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_step_graph.argtypes = [vp, i64, i64]
        L.lbm_observables.argtypes = [vp, C.POINTER(Obs)]
        L.lbm_get_density.argtypes = [vp, vp, i32]
        L.lbm_save.argtypes = [vp, vp, C.POINTER(sz)]
        L.lbm_load.argtypes = [vp, vp, sz]
        L.lbm_init_from_saturation.argtypes = [vp, vp, i32, C.c_double, C.c_double, C.c_double]
        L.lbm_debug_poke.argtypes = [vp, i32, i32, i32, i32, i32, C.c_float]
        L.lbm_get_step.restype = i64
        L.lbm_get_step.argtypes = [vp]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_last_error.argtypes = [vp]
        L.lbm_kernel_info.argtypes = [vp, C.c_char_p, sz, C.POINTER(i64), C.POINTER(i32)]
        L.lbm_autotune.argtypes = [vp, i64, C.c_char_p, sz]
        L.lbm_batch_workspace_bytes.restype = sz
        L.lbm_batch_workspace_bytes.argtypes = [i32, G, P]
        L.lbm_batch_create.argtypes = [i32, G, P, C.POINTER(vp), vp, sz, vp, C.POINTER(vp)]
        L.lbm_batch_step.argtypes = [vp, i64]
        L.lbm_batch_step_graph.argtypes = [vp, i64, i64]
        L.lbm_batch_observables.argtypes = [vp, C.POINTER(Obs)]
        L.lbm_batch_get_density.argtypes = [vp, i32, vp, i32]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_last_error.restype = C.c_char_p
        L.lbm_batch_last_error.argtypes = [vp]
        L.lbm_batch_kernel_info.argtypes = [vp, C.c_char_p, sz, C.POINTER(i64), C.POINTER(i32)]
        L.lbm_batch_autotune.argtypes = [vp, i64, C.c_char_p, sz]
        L.lbm_batch_set_active.argtypes = [vp, C.POINTER(i32)]
        for name in ("lbm_create", "lbm_set_bc", "lbm_step", "lbm_step_graph", "lbm_observables",
                     "lbm_get_density", "lbm_save", "lbm_load", "lbm_destroy", "lbm_kernel_info",
                     "lbm_autotune",
                     "lbm_batch_create", "lbm_batch_step", "lbm_batch_step_graph",
                     "lbm_batch_observables", "lbm_batch_get_density", "lbm_batch_destroy",
                     "lbm_batch_kernel_info", "lbm_batch_autotune", "lbm_batch_set_active"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def make_geometry(problem, keep: list) -> Geometry:
    mask = np.ascontiguousarray(problem.mask, dtype=np.uint8)
    keep.append(mask)
    g = Geometry()
    g.q, g.nx, g.ny, g.nz = problem.q, problem.nx, problem.ny, problem.nz
    g.solid = mask.ctypes.data
    g.periodic, g.open_x = problem.periodic, problem.open_x
    g.porous_x0, g.porous_x1 = problem.porous_x0, problem.porous_x1
    return g


def make_params(problem, storage=STORE_F32, math=MATH_F32, strategy=AUTO, tile_rows=0) -> Params:
    p = Params()
    p.tau[0], p.tau[1] = problem.tau
    p.G, p.xi = problem.G, problem.xi
    p.rho_in1, p.rho_out2 = problem.rho_in1, problem.rho_out2
    p.rho_in2, p.rho_out1 = problem.rho_in2, problem.rho_out1
    for i in range(3):
        p.g[i] = problem.g[i]
    p.collision, p.bc_set = problem.collision, problem.bc_set
    p.half_force_shift, p.mrt_sj_mode = problem.half_force_shift, problem.mrt_sj_mode
    p.lam, p.s_e, p.s_eps = problem.lam, problem.s_e, problem.s_eps
    p.storage = storage
    p.math = math
    p.strategy = strategy
    p.tile_rows = tile_rows
    p.eq26_mode = getattr(problem, "eq26_mode", 0)
    p.ivsd_frozen = getattr(problem, "ivsd_frozen", 0)
    return p


def workspace_bytes(problem, storage=STORE_F32, strategy=AUTO) -> int:
    keep = []
    g = make_geometry(problem, keep)
    p = make_params(problem, storage, strategy=strategy)
    return lib().lbm_workspace_bytes(C.byref(g), C.byref(p))


def _check(status, err_fn, handle=None):
    if status != LBM_OK:
        msg = err_fn(handle)
        raise LbmError(status, msg.decode() if msg else "")


def _torch_stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream


class Solver:
    """One instance on one GPU.  torch allocates the workspace; every kernel
    runs on `stream` (default: a new non-default torch stream)."""

    def __init__(self, problem, storage=STORE_F32, device="cuda:0", stream=None, math=MATH_F32,
                 strategy=AUTO, tile_rows=0):
        import torch
        self.problem = problem
        self.shape = problem.mask.shape
        self.N = problem.n_nodes
        L = lib()
        keep = []
        self._g = make_geometry(problem, keep)
        self._p = make_params(problem, storage, math, strategy, tile_rows)
        self._keep = keep
        nbytes = L.lbm_workspace_bytes(C.byref(self._g), C.byref(self._p))
        if nbytes == 0:
            # run create for the precise message
            h = C.c_void_p()
            rho0 = np.ascontiguousarray(problem.rho0, dtype=np.float64)
            st = L.lbm_create(C.byref(self._g), C.byref(self._p), rho0.ctypes.data, None, 0, None,
                              C.byref(h))
            _check(st, L.lbm_last_error)
            raise LbmError(LBM_EINVAL, "workspace size query failed")
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        rho0 = np.ascontiguousarray(problem.rho0, dtype=np.float64)
        self._h = C.c_void_p()
        st = L.lbm_create(C.byref(self._g), C.byref(self._p), rho0.ctypes.data, self.ws.data_ptr(),
                          nbytes, self.stream.cuda_stream, C.byref(self._h))
        _check(st, L.lbm_last_error)

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        _check(st, lib().lbm_last_error, self._h)

    def step(self, n=1):
        self._chk(lib().lbm_step(self._h, int(n)))

    def step_graph(self, n, reps=1):
        self._chk(lib().lbm_step_graph(self._h, int(n), int(reps)))

    def set_bc(self, rho_in1, rho_out2):
        self._chk(lib().lbm_set_bc(self._h, float(rho_in1), float(rho_out2)))

    @property
    def t(self):
        return lib().lbm_get_step(self._h)

    def observables(self, allow_unstable=False) -> dict:
        o = Obs()
        st = lib().lbm_observables(self._h, C.byref(o))
        if st == LBM_EUNSTABLE and allow_unstable:
            return o.to_dict()
        self._chk(st)
        return o.to_dict()

    def density(self) -> np.ndarray:
        out = np.empty((2,) + self.shape, dtype=np.float32)
        self._chk(lib().lbm_get_density(self._h, out.ctypes.data, 0))
        return out

    def init_from_saturation(self, sat, threshold=0.5, rho_major=None, rho_minor=None):
        """Warm start (lbm_init_from_saturation) from a saturation field of
        the grid's shape: a torch tensor on the solver's device or a host
        array.  The densities default to the problem's major and minor
        phase densities (largest component-2 and smallest component-1 initial
        density over the fluid)."""
        fluid = self.problem.mask == 0
        rho0 = np.asarray(self.problem.rho0)
        major = float(rho0[1][fluid].max()) if rho_major is None else float(rho_major)
        minor = float(rho0[0][fluid].min()) if rho_minor is None else float(rho_minor)
        if hasattr(sat, "data_ptr"):
            import torch
            t = sat.to(device=self.device, dtype=torch.float32).contiguous()
            if tuple(t.shape) != tuple(self.shape):
                raise ValueError(f"saturation shape {tuple(t.shape)} != grid {self.shape}")
            # the library reads it on its own stream
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            self._chk(lib().lbm_init_from_saturation(self._h, t.data_ptr(), 1, float(threshold), major, minor))
            t.record_stream(self.stream)
        else:
            a = np.ascontiguousarray(sat, dtype=np.float32)
            if a.shape != tuple(self.shape):
                raise ValueError(f"saturation shape {a.shape} != grid {self.shape}")
            self._chk(lib().lbm_init_from_saturation(self._h, a.ctypes.data, 0, float(threshold), major, minor))

    def debug_poke(self, x, y, z, s, i, value):
        """Overwrite one stored value of fluid node (x, y, z) (lbm_debug_poke):
        population i of component s with FP32 storage, the component's density
        word with BF16-deviation storage."""
        self._chk(lib().lbm_debug_poke(self._h, int(x), int(y), int(z), int(s), int(i), float(value)))

    def density_device(self, out=None):
        import torch
        if out is None:
            out = torch.empty((2,) + self.shape, dtype=torch.float32, device=self.device)
        self._chk(lib().lbm_get_density(self._h, out.data_ptr(), 1))
        return out

    def save(self) -> bytes:
        n = C.c_size_t(0)
        self._chk(lib().lbm_save(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._chk(lib().lbm_save(self._h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._chk(lib().lbm_load(self._h, buf, len(blob)))

    def autotune(self, steps=20) -> str:
        rep = C.create_string_buffer(1024)
        self._chk(lib().lbm_autotune(self._h, int(steps), rep, 1024))
        return rep.value.decode()

    def kernel_info(self):
        name = C.create_string_buffer(128)
        g = C.c_int64()
        b = C.c_int32()
        self._chk(lib().lbm_kernel_info(self._h, name, 128, C.byref(g), C.byref(b)))
        return name.value.decode(), g.value, b.value


class BatchSolver:
    """Many instances advanced by one launch per step (flat block table)."""

    def __init__(self, problems, storage=STORE_F32, device="cuda:0", stream=None, math=MATH_F32,
                 strategy=AUTO, tile_rows=0):
        import torch
        self.problems = list(problems)
        k = len(self.problems)
        L = lib()
        keep = []
        self._g = (Geometry * k)(*[make_geometry(p, keep) for p in self.problems])
        self._p = (Params * k)(*[make_params(p, storage, math, strategy, tile_rows) for p in self.problems])
        self._keep = keep
        nbytes = L.lbm_batch_workspace_bytes(k, self._g, self._p)
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "invalid batch description")
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        rhos = [np.ascontiguousarray(p.rho0, dtype=np.float64) for p in self.problems]
        self._rhos = rhos
        ptrs = (C.c_void_p * k)(*[r.ctypes.data for r in rhos])
        self._h = C.c_void_p()
        st = L.lbm_batch_create(k, self._g, self._p, ptrs, self.ws.data_ptr(), nbytes,
                                self.stream.cuda_stream, C.byref(self._h))
        _check(st, L.lbm_batch_last_error)

    def _chk(self, st):
        _check(st, lib().lbm_batch_last_error, self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._chk(lib().lbm_batch_step(self._h, int(n)))

    def step_graph(self, n, reps=1):
        self._chk(lib().lbm_batch_step_graph(self._h, int(n), int(reps)))

    def observables(self, allow_unstable=False):
        k = len(self.problems)
        o = (Obs * k)()
        st = lib().lbm_batch_observables(self._h, o)
        if not (st == LBM_EUNSTABLE and allow_unstable):
            self._chk(st)
        return [x.to_dict() for x in o]

    def density(self, i) -> np.ndarray:
        p = self.problems[i]
        out = np.empty((2,) + p.mask.shape, dtype=np.float32)
        self._chk(lib().lbm_batch_get_density(self._h, int(i), out.ctypes.data, 0))
        return out

    def set_active(self, active):
        """Retire (False) or re-admit (True) instances: one flag per instance."""
        flags = [1 if a else 0 for a in active]
        if len(flags) != len(self.problems):
            raise ValueError("need one flag per instance")
        self._chk(lib().lbm_batch_set_active(self._h, (C.c_int32 * len(flags))(*flags)))

    def autotune(self, steps=20) -> str:
        rep = C.create_string_buffer(1024)
        self._chk(lib().lbm_batch_autotune(self._h, int(steps), rep, 1024))
        return rep.value.decode()

    def kernel_info(self):
        name = C.create_string_buffer(128)
        g = C.c_int64()
        b = C.c_int32()
        self._chk(lib().lbm_batch_kernel_info(self._h, name, 128, C.byref(g), C.byref(b)))
        return name.value.decode(), g.value, b.value

    @property
    def n_nodes(self):
        return sum(p.n_nodes for p in self.problems)

    @property
    def n_fluid(self):
        return sum(p.n_fluid for p in self.problems)
