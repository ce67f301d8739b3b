"""Shared test helpers: oracle problem from a workload dict, error norms."""
import numpy as np

from oracle import oracle as orc

KEYS = ["dim", "order", "nelem", "xlo", "xhi", "nvel", "vlo", "vhi", "bc", "mu_ref",
        "theta_ref", "omega", "gamma", "limiter", "newton_maxit", "newton_tol"]
OPTIONAL = ["equilibrium", "wall_theta", "wall_vel", "sutherland"]


def oracle_problem(pb) -> orc.Problem:
    kw = {k: pb[k] for k in KEYS}
    kw.update({k: pb[k] for k in OPTIONAL if k in pb})
    return orc.Problem(**kw)


def initial_state(pb, kind, seed=None, amp=0.0, **prim_kw):
    """f from the oracle's Maxwellian sampler at the oracle's nodes, optionally times a
    seeded positive perturbation (the same array is fed to both sides)."""
    from paper_2308_06196_amd import workloads as wl
    pr = oracle_problem(pb)
    f = orc.maxwellian(pr, wl.PRIM[kind](orc.node_coords(pr), **prim_kw))
    if seed is not None:
        f = f * wl.perturbation(seed, f.shape, amp)
    return f


def rel_max(a, b, scale=None):
    a = np.asarray(a)
    b = np.asarray(b)
    s = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / s)


def field_errors(pb, Qa, Qb):
    """Gauss-weighted L2 relative errors of rho, rho U (normalised by ||rho||), E."""
    _, wq = orc.gauss_legendre(pb["order"] + 1)
    W = wq
    for _ in range(pb["dim"] - 1):
        W = np.outer(W, wq).ravel()
    ne = int(np.prod(pb["nelem"][: pb["dim"]]))
    Wn = np.tile(W, ne)
    n = lambda v: float(np.sqrt(np.sum(Wn * v * v)))
    rho = n(Qb[:, 0])
    return {"rho": n(Qa[:, 0] - Qb[:, 0]) / rho,
            "mom": n(np.linalg.norm(Qa[:, 1:4] - Qb[:, 1:4], axis=1)) / rho,
            "E": n(Qa[:, 4] - Qb[:, 4]) / n(Qb[:, 4])}
