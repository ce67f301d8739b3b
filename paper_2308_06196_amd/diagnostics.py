"""Taylor-Green vortex diagnostics: kinetic energy and enstrophy vs time.

The paper uses the Taylor-Green vortex to show that the Boltzmann-BGK
approach captures transition to turbulence (Sec. 3, Taylor-Green vortex), with
kinetic energy and enstrophy histories as the measures. These integrals are
taken from the macroscopic moments the library computes on the GPU
(bgk_moments): over every element, with the element's Gauss quadrature,

    K = int 1/2 rho |U|^2 dx,    Z = int 1/2 rho |curl U|^2 dx,

where curl U uses the element-local derivative of the nodal velocity
(Lagrange interpolation on the Gauss points). A history runs the workload in
FP64, FP32 and BF16-increment storage side by side; no reference data exists
for this configuration, so the FP32 and BF16 histories are compared against
the FP64 one.

Usage: python -m paper_2308_06196_amd.diagnostics [--n 16] [--steps 100] [--every 10]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import bgk
from . import workloads as wl


def _gauss_ops(n1: int):
    """Gauss points, weights and the Lagrange derivative matrix D[a, b] = l_b'(x_a)."""
    x, w = np.polynomial.legendre.leggauss(n1)
    c = np.array([1.0 / np.prod([x[b] - x[m] for m in range(n1) if m != b]) for b in range(n1)])
    D = np.zeros((n1, n1))
    for a in range(n1):
        for b in range(n1):
            if a != b:
                D[a, b] = (c[b] / c[a]) / (x[a] - x[b])
        D[a, a] = -D[a].sum()
    return x, w, D


def integrals(pb: dict, Q: np.ndarray, gamma: float = 5.0 / 3.0) -> dict:
    """Mass, kinetic energy and enstrophy of the moments Q [nx, 5] on the mesh of a
    3-D problem (library node order: element-major, a_1 fastest)."""
    d, n1 = pb["dim"], pb["order"] + 1
    if d != 3:
        raise ValueError("enstrophy needs a 3-D mesh")
    ne = [int(v) for v in pb["nelem"][:3]]
    h = [(pb["xhi"][k] - pb["xlo"][k]) / ne[k] for k in range(3)]
    _, w, D = _gauss_ops(n1)
    nel = ne[0] * ne[1] * ne[2]
    q = Q.reshape(nel, n1, n1, n1, 5)  # [e, a_z, a_y, a_x, m]
    rho = q[..., 0]
    U = q[..., 1:4] / rho[..., None]
    # derivative of U_c along axis k (array axes 3, 2, 1 = x, y, z) per element
    def ddx(f, k):
        ax = 3 - k
        return np.moveaxis(np.tensordot(D, np.moveaxis(f, ax, 0), axes=(1, 0)), 0, ax) * (2.0 / h[k])
    om = np.stack([ddx(U[..., 2], 1) - ddx(U[..., 1], 2),
                   ddx(U[..., 0], 2) - ddx(U[..., 2], 0),
                   ddx(U[..., 1], 0) - ddx(U[..., 0], 1)], axis=-1)
    W = np.einsum("i,j,k->ijk", w, w, w) * (h[0] * h[1] * h[2] / 8.0)  # [a_z, a_y, a_x]
    ke = 0.5 * rho * (U * U).sum(-1)
    ens = 0.5 * rho * (om * om).sum(-1)
    P = (gamma - 1.0) * (q[..., 4] - ke)
    return {"mass": float((W * rho).sum()), "kinetic_energy": float((W * ke).sum()),
            "enstrophy": float((W * ens).sum()), "mean_pressure": float((W * P).sum())}


def tgv_history(n: int = 16, order: int = 3, nv1: int = 16, steps: int = 100, every: int = 10,
                precisions=(bgk.FP64, bgk.FP32, bgk.BF16), cfl: float = 0.1,
                dt: float | None = None) -> list:
    """Kinetic energy and enstrophy every `every` steps of the Taylor-Green box in
    each storage precision (same time step for all: dt, or the stable step of the
    first run's initial state)."""
    pb = wl.tgv3d(n=n, order=order, nv1=nv1)
    rows = []
    for prec in precisions:
        s = bgk.Solver(pb, precision=prec)
        try:
            s.set_maxwellian(wl.prim_tgv3d(s.node_coords()))
            if dt is None:
                dt = s.stable_dt(cfl)
            for k in range(0, steps + 1, every):
                if k:
                    s.rk3_step(dt, every)
                r = integrals(pb, s.moments().cpu().numpy())
                r.update({"precision": bgk.PRECISION_NAME[prec], "step": k, "t": k * dt})
                rows.append(r)
        finally:
            s.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--order", type=int, default=3)
    ap.add_argument("--nv", type=int, default=16)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--every", type=int, default=10)
    a = ap.parse_args(argv)
    rows = tgv_history(a.n, a.order, a.nv, a.steps, a.every)
    for r in rows:
        print(json.dumps(r), flush=True)
    f64 = {r["step"]: r for r in rows if r["precision"] == "fp64"}
    print("| step | t | K (FP64) | Z (FP64) | storage | rel. diff K | rel. diff Z |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        if r["precision"] == "fp64":
            continue
        b = f64[r["step"]]
        print(f"| {r['step']} | {r['t']:.4f} | {b['kinetic_energy']:.6e} | {b['enstrophy']:.6e} | "
              f"{r['precision']} | "
              f"{abs(r['kinetic_energy'] - b['kinetic_energy']) / b['kinetic_energy']:.1e} | "
              f"{abs(r['enstrophy'] - b['enstrophy']) / b['enstrophy']:.1e} |")


if __name__ == "__main__":
    main()
