"""Thin ctypes binding of libbgk (C-ABI declared in include/bgk.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libbgk.so. PyTorch provides device memory (the solver workspace
and exchange buffers) and the stream. There is no fallback: if the library
is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbgk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bgk.h")

BGK_OK = 0
BGK_HOST, BGK_DEVICE = 0, 1
FP64, FP32, BF16 = 0, 1, 2
PRECISION_NAME = {0: "fp64", 1: "fp32", 2: "bf16"}
STATUS = {0: "BGK_OK", 1: "BGK_ERR_INVALID_ARG", 2: "BGK_ERR_UNSUPPORTED",
          3: "BGK_ERR_OUT_OF_MEMORY", 4: "BGK_ERR_DEVICE", 5: "BGK_ERR_NEWTON",
          6: "BGK_ERR_NONFINITE", 7: "BGK_ERR_STATE"}


class BGKError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("order", C.c_int32),
        ("nelem", C.c_int32 * 3),
        ("xlo", C.c_double * 3), ("xhi", C.c_double * 3),
        ("bc", (C.c_int32 * 2) * 3),
        ("nvel", C.c_int32 * 3),
        ("vlo", C.c_double * 3), ("vhi", C.c_double * 3),
        ("mu_ref", C.c_double), ("theta_ref", C.c_double), ("omega", C.c_double),
        ("gamma", C.c_double),
        ("precision", C.c_int32), ("limiter", C.c_int32),
        ("newton_maxit", C.c_int32),
        ("newton_tol", C.c_double),
        ("equilibrium", C.c_int32),
        ("wall_theta", (C.c_double * 2) * 3),
        ("wall_vel", ((C.c_double * 3) * 2) * 3),
        ("sutherland", C.c_double),
    ]


class Timing(C.Structure):
    _fields_ = [("stage_launches", C.c_int64), ("stage_ms", C.c_double),
                ("newton_launches", C.c_int64), ("newton_ms", C.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if k.endswith("ms") else int(getattr(self, k)))
                for k, _ in self._fields_}


class Diag(C.Structure):
    _fields_ = [("newton_it_max", C.c_int64), ("newton_fail", C.c_int64),
                ("limiter_hits", C.c_int64), ("limiter_bad", C.c_int64),
                ("stages", C.c_int64), ("positivity_violations", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def problem_struct(pb: dict, precision: int = FP64) -> Problem:
    """bgk_problem from a plain problem dict (see workloads.problem)."""
    s = Problem()
    s.dim, s.order = int(pb["dim"]), int(pb["order"])
    for k in range(3):
        s.nelem[k] = int(pb["nelem"][k])
        s.xlo[k], s.xhi[k] = float(pb["xlo"][k]), float(pb["xhi"][k])
        s.bc[k][0], s.bc[k][1] = int(pb["bc"][k][0]), int(pb["bc"][k][1])
        s.nvel[k] = int(pb["nvel"][k])
        s.vlo[k], s.vhi[k] = float(pb["vlo"][k]), float(pb["vhi"][k])
    s.mu_ref, s.theta_ref = float(pb["mu_ref"]), float(pb["theta_ref"])
    s.omega, s.gamma = float(pb["omega"]), float(pb["gamma"])
    s.precision, s.limiter = int(precision), int(pb["limiter"])
    s.newton_maxit, s.newton_tol = int(pb["newton_maxit"]), float(pb["newton_tol"])
    s.equilibrium = int(pb.get("equilibrium", 0))
    s.sutherland = float(pb.get("sutherland", 0.0))
    wt = pb.get("wall_theta", [(1.0, 1.0)] * 3)
    wv = pb.get("wall_vel", [((0.0,) * 3,) * 2] * 3)
    for k in range(3):
        for side in range(2):
            s.wall_theta[k][side] = float(wt[k][side])
            for c in range(3):
                s.wall_vel[k][side][c] = float(wv[k][side][c])
    return s


_lib = None


def exported_names() -> list:
    """Function names declared in include/bgk.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:bgk_status|const char\*|int32_t)\s+(bgk_\w+)\s*\(", txt,
                                 re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int32
        pp = C.POINTER(Problem)
        sig = {
            "bgk_query_footprint": [pp, C.POINTER(C.c_size_t), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)],
            "bgk_create": [pp, vp, C.c_size_t, vp, C.POINTER(vp)],
            "bgk_destroy": [vp],
            "bgk_node_coords": [vp, dp],
            "bgk_velocity_grid": [vp, dp, dp],
            "bgk_set_state": [vp, vp, i32],
            "bgk_set_maxwellian": [vp, vp, i32],
            "bgk_get_state": [vp, vp, i32],
            "bgk_residual": [vp, vp, vp, i32],
            "bgk_rk3_step": [vp, C.c_double, i32],
            "bgk_moments": [vp, vp, i32],
            "bgk_collision_moments": [vp, vp, i32],
            "bgk_residual_noalloc": [pp, vp, vp, vp],
            "bgk_stable_dt": [vp, C.c_double, dp],
            "bgk_diagnostics": [vp, C.POINTER(Diag)],
            "bgk_synchronize": [vp],
            "bgk_timing_enable": [vp, i32],
            "bgk_timing_read": [vp, C.POINTER(Timing)],
            "bgk_set_stream": [vp, vp],
            "bgk_batch_query_footprint": [i32, C.POINTER(C.c_size_t)],
            "bgk_batch_create": [vp, i32, vp, C.c_size_t, C.POINTER(vp)],
            "bgk_batch_add": [vp, vp, C.c_double, C.c_int64],
            "bgk_batch_step": [vp, i32],
            "bgk_batch_poll": [vp, C.POINTER(vp), C.POINTER(i32), i32, C.POINTER(i32)],
            "bgk_batch_poll_ready": [vp, C.POINTER(vp), C.POINTER(i32), i32, C.POINTER(i32)],
            "bgk_batch_remove": [vp, vp],
            "bgk_batch_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.bgk_batch_size.argtypes = [vp]
        L.bgk_batch_size.restype = C.c_int32
        L.bgk_status_str.argtypes = [C.c_int]
        L.bgk_status_str.restype = C.c_char_p
        L.bgk_last_error.argtypes = []
        L.bgk_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st: int):
    if st != BGK_OK:
        raise BGKError(st, lib().bgk_last_error().decode())


def footprint(pb: dict, precision: int = FP64):
    s = problem_struct(pb, precision)
    b, nx, nv = C.c_size_t(0), C.c_int64(0), C.c_int64(0)
    _check(lib().bgk_query_footprint(C.byref(s), C.byref(b), C.byref(nx), C.byref(nv)))
    return int(b.value), int(nx.value), int(nv.value)


def residual_noalloc(pb: dict, f_in, out=None, precision: int = FP64, stream=None):
    """Residual L(f) of problem pb for a device tensor f_in (canonical FP64
    layout) without a solver or workspace: the library keeps its scratch in a
    static device array (bgk_residual_noalloc). out: a float64 device tensor of
    the same size, or None for a new one (allocated here by torch, outside the
    library call). Queued on `stream` (default: torch's current stream)."""
    import torch
    assert isinstance(f_in, torch.Tensor) and f_in.is_cuda and f_in.dtype == torch.float64
    assert f_in.is_contiguous()
    if out is None:
        out = torch.empty_like(f_in)
    assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
    assert out.numel() == f_in.numel()
    st = problem_struct(pb, precision)
    stream = stream if stream is not None else torch.cuda.current_stream(f_in.device)
    _check(lib().bgk_residual_noalloc(C.byref(st), C.c_void_p(f_in.data_ptr()),
                                      C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream)))
    return out


class Solver:
    """One problem instance on one GPU. The workspace is a torch uint8 tensor
    owned by this object; the stream defaults to torch's current stream."""

    def __init__(self, pb: dict, precision: int = FP64, device="cuda:0", stream=None,
                 workspace=None):
        import torch

        self.torch = torch
        self.pb = pb
        self.precision = precision
        self.device = torch.device(device)
        nbytes, self.nx, self.nv = footprint(pb, precision)
        self.ne = int(np.prod(pb["nelem"][: pb["dim"]]))
        self.ns = (pb["order"] + 1) ** pb["dim"]
        self.workspace_bytes = nbytes
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        assert workspace.numel() >= nbytes and workspace.data_ptr() % 256 == 0
        self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._s = C.c_void_p()
        st = problem_struct(pb, precision)
        _check(lib().bgk_create(C.byref(st), C.c_void_p(workspace.data_ptr()), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(self._s)))

    # -- lifetime ------------------------------------------------------------
    def close(self, sync: bool = True):
        """Release the solver and its workspace. sync=False skips waiting for
        the solver's stream: only for a solver whose work is known to have
        completed (a batch member handed back by Batch.poll)."""
        if self._s:
            _check(lib().bgk_destroy(self._s))
            self._s = C.c_void_p()
            # queued work on the solver's stream may still use the workspace
            if sync:
                self.stream.synchronize()
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------
    @property
    def shape(self):
        return (self.ne, self.ns, self.nv)

    def _arg(self, a, n: int):
        """(pointer, where, keepalive) for a float64 array of n values."""
        torch = self.torch
        if isinstance(a, torch.Tensor):
            assert a.dtype == torch.float64 and a.is_contiguous() and a.numel() == n
            if a.is_cuda:
                return C.c_void_p(a.data_ptr()), BGK_DEVICE, a
            a = a.numpy()
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.size == n
        return C.c_void_p(a.ctypes.data), BGK_HOST, a

    # -- C-ABI wrappers ----------------------------------------------------------
    def node_coords(self) -> np.ndarray:
        x = np.zeros((self.nx, self.pb["dim"]))
        _check(lib().bgk_node_coords(self._s, x.ctypes.data_as(C.POINTER(C.c_double))))
        return x

    def velocity_grid(self):
        u, w = np.zeros((self.nv, 3)), np.zeros(self.nv)
        _check(lib().bgk_velocity_grid(self._s, u.ctypes.data_as(C.POINTER(C.c_double)),
                                       w.ctypes.data_as(C.POINTER(C.c_double))))
        return u, w

    def set_state(self, f):
        p, where, keep = self._arg(f, self.nx * self.nv)
        _check(lib().bgk_set_state(self._s, p, where))
        return keep

    def set_maxwellian(self, prim):
        p, where, keep = self._arg(prim, self.nx * 5)
        _check(lib().bgk_set_maxwellian(self._s, p, where))
        return keep

    def get_state(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        p, where, keep = self._arg(out, self.nx * self.nv)
        _check(lib().bgk_get_state(self._s, p, where))
        return out if where == BGK_DEVICE or isinstance(out, torch.Tensor) else keep

    def residual(self, f_in=None, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        po, where, keep_o = self._arg(out, self.nx * self.nv)
        pi = None
        keep_i = None
        if f_in is not None:
            pi, where_i, keep_i = self._arg(f_in, self.nx * self.nv)
            assert where_i == where, "f_in and out must both be host or both device"
        _check(lib().bgk_residual(self._s, pi, po, where))
        return out if isinstance(out, torch.Tensor) else keep_o

    def rk3_step(self, dt: float, nsteps: int = 1):
        _check(lib().bgk_rk3_step(self._s, float(dt), int(nsteps)))

    def moments(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty((self.nx, 5), dtype=torch.float64, device=self.device)
        p, where, keep = self._arg(out, self.nx * 5)
        _check(lib().bgk_moments(self._s, p, where))
        return out if isinstance(out, torch.Tensor) else keep

    def collision_moments(self, out=None):
        """Discrete moments [nx, 5] of the collision term of the installed state,
        formed as the stage kernels form it (bgk_collision_moments)."""
        torch = self.torch
        if out is None:
            out = torch.empty((self.nx, 5), dtype=torch.float64, device=self.device)
        p, where, keep = self._arg(out, self.nx * 5)
        _check(lib().bgk_collision_moments(self._s, p, where))
        return out if isinstance(out, torch.Tensor) else keep

    def stable_dt(self, cfl: float) -> float:
        dt = C.c_double(0.0)
        _check(lib().bgk_stable_dt(self._s, float(cfl), C.byref(dt)))
        return float(dt.value)

    def diagnostics(self, raise_on_failure: bool = True) -> dict:
        d = Diag()
        st = lib().bgk_diagnostics(self._s, C.byref(d))
        if raise_on_failure:
            _check(st)
        return d.as_dict()

    def synchronize(self):
        _check(lib().bgk_synchronize(self._s))

    def set_stream(self, stream):
        _check(lib().bgk_set_stream(self._s, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def timing(self, on: bool):
        _check(lib().bgk_timing_enable(self._s, 1 if on else 0))

    def timing_read(self) -> dict:
        t = Timing()
        _check(lib().bgk_timing_read(self._s, C.byref(t)))
        return t.as_dict()


class Batch:
    """Resident solvers advanced together by launches over descriptor tables
    (libbgk batch C-ABI): one launch per kernel family covers all its members. Members must be created on the batch's stream;
    FP64 or FP32 storage, 1-D or 2-D problems. The tables live in a torch
    device buffer owned by this object."""

    def __init__(self, stream, max_members: int = 64):
        import torch
        self.stream = stream
        self.max_members = max_members
        nbytes = C.c_size_t(0)
        _check(lib().bgk_batch_query_footprint(int(max_members), C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=stream.device)
        base = self.workspace.data_ptr()
        ptr = (base + 255) // 256 * 256
        self._b = C.c_void_p()
        _check(lib().bgk_batch_create(C.c_void_p(stream.cuda_stream), int(max_members),
                                      C.c_void_p(ptr), nbytes.value, C.byref(self._b)))
        self._members = {}

    def add(self, solver: Solver, dt: float, nsteps: int):
        _check(lib().bgk_batch_add(self._b, solver._s, float(dt), int(nsteps)))
        self._members[solver._s.value] = solver

    def step(self, nsteps: int):
        _check(lib().bgk_batch_step(self._b, int(nsteps)))

    def size(self) -> int:
        return int(lib().bgk_batch_size(self._b))

    def poll(self, block: bool = True):
        """[(solver, None | error message)] of members that completed; with
        block=False only those whose work the device has already executed."""
        cap = max(1, len(self._members))
        done = (C.c_void_p * cap)()
        st = (C.c_int32 * cap)()
        n = C.c_int32(0)
        fn = lib().bgk_batch_poll if block else lib().bgk_batch_poll_ready
        _check(fn(self._b, done, st, cap, C.byref(n)))
        out = []
        for i in range(n.value):
            s = self._members.pop(done[i])
            out.append((s, None if st[i] == 0 else STATUS.get(st[i], str(st[i]))))
        return out

    def remove(self, solver: Solver):
        _check(lib().bgk_batch_remove(self._b, solver._s))
        self._members.pop(solver._s.value, None)

    def close(self):
        if self._b:
            lib().bgk_batch_destroy(self._b)  # waits for the batch stream
            self._b = C.c_void_p()
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
