"""FP64 CPU oracle for the discrete-velocity Boltzmann-BGK residual (test infrastructure).

This module loads ``liborc.so`` (built from ``bgk_oracle.c``) and exposes its
functions on numpy arrays. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the HIP product path never does,
and the two share no code.

Every function follows Dzanic & Martinelli (arXiv 2308.06196):
Sec. 2 (BGK model: moments, Maxwellian, tau = mu/P), Sec. 2.1 (nodal FR
transport with DG-recovering corrections, upwind flux, Zhang-Shu limiter,
trapezoidal velocity quadrature, discretely conservative equilibrium by Newton),
Sec. 2.2 (explicit time stepping, SSP-RK3 here). The readings taken where the
paper is silent are listed at the top of ``bgk_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bgk_oracle.c")
# BGK_ORACLE_LIB names another build of the same source (used to check that
# planted mistakes in a scratch copy of the oracle fail its pins)
_LIB = os.environ.get("BGK_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if os.environ.get("BGK_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
             "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("order", C.c_int32),
        ("nelem", C.c_int32 * 3),
        ("xlo", C.c_double * 3), ("xhi", C.c_double * 3),
        ("bc", (C.c_int32 * 2) * 3),
        ("nvel", C.c_int32 * 3),
        ("vlo", C.c_double * 3), ("vhi", C.c_double * 3),
        ("mu_ref", C.c_double), ("theta_ref", C.c_double), ("omega", C.c_double),
        ("gamma", C.c_double),
        ("limiter", C.c_int32), ("newton_maxit", C.c_int32),
        ("newton_tol", C.c_double),
        ("equilibrium", C.c_int32),
        ("wall_theta", (C.c_double * 2) * 3),
        ("wall_vel", ((C.c_double * 3) * 2) * 3),
        ("sutherland", C.c_double),
    ]


class Diag(C.Structure):
    _fields_ = [("newton_it_max", C.c_int64), ("newton_fail", C.c_int64),
                ("limiter_hits", C.c_int64), ("limiter_bad", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


@dataclass
class Problem:
    """Uniform Cartesian box in d dims, nodal FR order p, 3-D velocity grid.

    bc[k] = (left, right) with 0 = periodic, 1 = specular wall, 2 = diffuse
    (Maxwell) wall at temperature wall_theta[k][side] moving with
    wall_vel[k][side].
    equilibrium: 0 = discretely conservative Maxwellian (Newton), 1 = the
    continuous Maxwellian sampled at the nodes (non-conservative model).
    mu = mu_ref (theta/theta_ref)^omega, tau = mu / P; mu_ref <= 0 turns the
    collision term off. gamma <= 0 means 5/3.
    """
    dim: int
    order: int
    nelem: tuple
    xlo: tuple
    xhi: tuple
    nvel: tuple
    vlo: tuple
    vhi: tuple
    bc: tuple = ((0, 0), (0, 0), (0, 0))
    mu_ref: float = 1e-2
    theta_ref: float = 1.0
    omega: float = 0.0
    gamma: float = 0.0
    limiter: int = 1
    newton_maxit: int = 20
    newton_tol: float = 1e-14
    equilibrium: int = 0
    wall_theta: tuple = ((1.0, 1.0), (1.0, 1.0), (1.0, 1.0))
    wall_vel: tuple = (((0.0,) * 3,) * 2,) * 3
    sutherland: float = 0.0

    def cstruct(self) -> _Problem:
        s = _Problem()
        s.dim, s.order = self.dim, self.order
        for k in range(3):
            s.nelem[k] = int(self.nelem[k]) if k < len(self.nelem) else 1
            s.xlo[k] = float(self.xlo[k]) if k < len(self.xlo) else 0.0
            s.xhi[k] = float(self.xhi[k]) if k < len(self.xhi) else 1.0
            s.nvel[k] = int(self.nvel[k])
            s.vlo[k] = float(self.vlo[k])
            s.vhi[k] = float(self.vhi[k])
            bck = self.bc[k] if k < len(self.bc) else (0, 0)
            s.bc[k][0], s.bc[k][1] = int(bck[0]), int(bck[1])
        s.mu_ref, s.theta_ref, s.omega, s.gamma = self.mu_ref, self.theta_ref, self.omega, self.gamma
        s.limiter, s.newton_maxit, s.newton_tol = self.limiter, self.newton_maxit, self.newton_tol
        s.equilibrium = int(self.equilibrium)
        s.sutherland = float(self.sutherland)
        for k in range(3):
            for side in range(2):
                s.wall_theta[k][side] = float(self.wall_theta[k][side])
                for c in range(3):
                    s.wall_vel[k][side][c] = float(self.wall_vel[k][side][c])
        return s

    @property
    def ns(self) -> int:
        return (self.order + 1) ** self.dim

    @property
    def ne(self) -> int:
        return int(np.prod(self.nelem[: self.dim]))

    @property
    def nx(self) -> int:
        return self.ne * self.ns

    @property
    def nv(self) -> int:
        return int(np.prod(self.nvel))


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(_Problem)
        L.orc_gauss_legendre.argtypes = [C.c_int, dp, dp]
        L.orc_lagrange.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_dg_correction.argtypes = [C.c_int, dp, dp, dp]
        L.orc_velocity_grid.argtypes = [pp, dp, dp]
        L.orc_node_coords.argtypes = [pp, dp]
        L.orc_maxwellian.argtypes = [pp, dp, dp]
        L.orc_moments.argtypes = [pp, dp, dp]
        L.orc_newton_node.argtypes = [pp, dp, dp, C.POINTER(C.c_int), dp]
        L.orc_transport.argtypes = [pp, dp, dp]
        L.orc_collision.argtypes = [pp, dp, dp, C.POINTER(Diag)]
        L.orc_residual.argtypes = [pp, dp, dp, C.POINTER(Diag)]
        L.orc_residual_elems.argtypes = [pp, dp, C.POINTER(C.c_int64), C.c_int64, dp,
                                         C.POINTER(Diag)]
        L.orc_limiter.argtypes = [pp, dp, C.POINTER(Diag)]
        L.orc_rk3_step.argtypes = [pp, dp, C.c_double, C.c_int, C.POINTER(Diag)]
        L.orc_rk3_step.restype = C.c_int
        L.orc_stable_dt.argtypes = [pp, dp, C.c_double]
        L.orc_stable_dt.restype = C.c_double
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---- one-dimensional operators ------------------------------------------------

def gauss_legendre(n: int):
    x, w = np.zeros(n), np.zeros(n)
    lib().orc_gauss_legendre(n, _p(x), _p(w))
    return x, w


def lagrange_ops(xi: np.ndarray):
    n = len(xi)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    D, lL, lR = np.zeros((n, n)), np.zeros(n), np.zeros(n)
    lib().orc_lagrange(n, _p(xi), _p(D), _p(lL), _p(lR))
    return D, lL, lR


def dg_correction(p: int, xi: np.ndarray):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    GL, GR = np.zeros(p + 1), np.zeros(p + 1)
    lib().orc_dg_correction(p, _p(xi), _p(GL), _p(GR))
    return GL, GR


# ---- problem-level operations -------------------------------------------------

def velocity_grid(pr: Problem):
    u, w = np.zeros((pr.nv, 3)), np.zeros(pr.nv)
    s = pr.cstruct()
    lib().orc_velocity_grid(C.byref(s), _p(u), _p(w))
    return u, w


def node_coords(pr: Problem):
    x = np.zeros((pr.nx, pr.dim))
    s = pr.cstruct()
    lib().orc_node_coords(C.byref(s), _p(x))
    return x


def maxwellian(pr: Problem, prim: np.ndarray) -> np.ndarray:
    """prim [nx,5] = (rho, Ux, Uy, Uz, theta) -> f [ne, ns, nv]."""
    prim = np.ascontiguousarray(prim, dtype=np.float64).reshape(pr.nx, 5)
    f = np.zeros((pr.ne, pr.ns, pr.nv))
    s = pr.cstruct()
    lib().orc_maxwellian(C.byref(s), _p(prim), _p(f))
    return f


def moments(pr: Problem, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    Q = np.zeros((pr.nx, 5))
    s = pr.cstruct()
    lib().orc_moments(C.byref(s), _p(f), _p(Q))
    return Q


def newton_node(pr: Problem, Q):
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    alpha = np.zeros(5)
    its = C.c_int(0)
    res = C.c_double(0)
    s = pr.cstruct()
    st = lib().orc_newton_node(C.byref(s), _p(Q), _p(alpha), C.byref(its), C.byref(res))
    return st, alpha, its.value, res.value


def transport(pr: Problem, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    T = np.zeros_like(f)
    s = pr.cstruct()
    lib().orc_transport(C.byref(s), _p(f), _p(T))
    return T


def collision(pr: Problem, f: np.ndarray):
    f = np.ascontiguousarray(f, dtype=np.float64)
    Cc = np.zeros_like(f)
    d = Diag()
    s = pr.cstruct()
    lib().orc_collision(C.byref(s), _p(f), _p(Cc), C.byref(d))
    return Cc, d.as_dict()


def residual(pr: Problem, f: np.ndarray):
    f = np.ascontiguousarray(f, dtype=np.float64)
    L = np.zeros_like(f)
    d = Diag()
    s = pr.cstruct()
    lib().orc_residual(C.byref(s), _p(f), _p(L), C.byref(d))
    return L, d.as_dict()


def residual_elems(pr: Problem, f: np.ndarray, elems):
    f = np.ascontiguousarray(f, dtype=np.float64)
    el = np.ascontiguousarray(elems, dtype=np.int64)
    out = np.zeros((len(el), pr.ns, pr.nv))
    d = Diag()
    s = pr.cstruct()
    lib().orc_residual_elems(C.byref(s), _p(f), el.ctypes.data_as(C.POINTER(C.c_int64)),
                             len(el), _p(out), C.byref(d))
    return out, d.as_dict()


def limiter(pr: Problem, f: np.ndarray):
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    d = Diag()
    s = pr.cstruct()
    lib().orc_limiter(C.byref(s), _p(f), C.byref(d))
    return f, d.as_dict()


def rk3_step(pr: Problem, f: np.ndarray, dt: float, nsteps: int = 1):
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    d = Diag()
    s = pr.cstruct()
    st = lib().orc_rk3_step(C.byref(s), _p(f), float(dt), int(nsteps), C.byref(d))
    if st:
        raise MemoryError("oracle rk3_step could not allocate its stage buffers")
    return f, d.as_dict()


def stable_dt(pr: Problem, f: np.ndarray, cfl: float) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    s = pr.cstruct()
    return float(lib().orc_stable_dt(C.byref(s), _p(f), float(cfl)))
