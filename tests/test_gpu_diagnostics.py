"""Taylor-Green histories on the GPU (FP64, FP32 and BF16-increment storage):
mass is conserved, kinetic energy decays in FP64, and the FP32 and BF16
histories stay within stated tolerances of the FP64 one (no reference data
exists for this configuration).

BF16 tolerance: the stored stage increments round with relative error
<= 2^-8, and an increment is at most a few 1e-3 of f per step here, so the
integrals move by <~1e-5 per step from rounding; 1e-3 relative over 20 steps
for K and Z, and 1e-4 for the mass (every rounding error of an increment
changes the discrete mass by at most 2^-8 of that increment)."""
import pytest

pytestmark = pytest.mark.gpu


def test_tgv_history_fp64_fp32_bf16():
    import torch
    assert torch.cuda.is_available()
    from paper_2308_06196_amd import diagnostics as dg
    print("[case] tgv history n=4 p=3 nv1=12 steps=20", flush=True)
    rows = dg.tgv_history(n=4, order=3, nv1=12, steps=20, every=5)
    f64 = [r for r in rows if r["precision"] == "fp64"]
    f32 = {r["step"]: r for r in rows if r["precision"] == "fp32"}
    b16 = {r["step"]: r for r in rows if r["precision"] == "bf16"}
    for r in rows:
        print(r, flush=True)
    m0 = f64[0]["mass"]
    for a, b in zip(f64, f64[1:]):
        assert b["kinetic_energy"] < a["kinetic_energy"]
        assert abs(b["mass"] - m0) < 1e-13 * m0
    for r in f64:
        s = f32[r["step"]]
        assert abs(s["kinetic_energy"] - r["kinetic_energy"]) < 1e-5 * r["kinetic_energy"]
        assert abs(s["enstrophy"] - r["enstrophy"]) < 1e-4 * r["enstrophy"]
        h = b16[r["step"]]
        assert abs(h["kinetic_energy"] - r["kinetic_energy"]) < 1e-3 * r["kinetic_energy"]
        assert abs(h["enstrophy"] - r["enstrophy"]) < 1e-3 * r["enstrophy"]
        assert abs(h["mass"] - m0) < 1e-4 * m0


def test_tgv_history_fp64_matches_oracle():
    """The FP64 Taylor-Green history (kinetic energy and enstrophy of the GPU's
    moments) against the same integrals of the oracle's moments after the same
    steps (4^3 elements, p = 3, 12^3 velocities, 20 steps): 1e-12 relative."""
    import numpy as np
    import torch
    assert torch.cuda.is_available()
    from oracle import oracle as orc
    from paper_2308_06196_amd import bgk
    from paper_2308_06196_amd import diagnostics as dg
    from paper_2308_06196_amd import workloads as wl
    from tests.helpers import oracle_problem
    pb = wl.tgv3d(n=4, order=3, nv1=12)
    pr = oracle_problem(pb)
    f = orc.maxwellian(pr, wl.prim_tgv3d(orc.node_coords(pr)))
    dt = orc.stable_dt(pr, f, 0.1)
    print("[case] tgv history vs oracle n=4 p=3 nv1=12 steps=20", flush=True)
    ref = []
    for k in range(0, 21, 5):
        if k:
            f, _ = orc.rk3_step(pr, f, dt, 5)
        ref.append(dg.integrals(pb, orc.moments(pr, f)))
    rows = dg.tgv_history(n=4, order=3, nv1=12, steps=20, every=5, precisions=(bgk.FP64,), dt=dt)
    for r, o in zip(rows, ref):
        dk = abs(r["kinetic_energy"] - o["kinetic_energy"]) / o["kinetic_energy"]
        dz = abs(r["enstrophy"] - o["enstrophy"]) / o["enstrophy"]
        print(f"  step {r['step']}: K {r['kinetic_energy']:.12e} (oracle {o['kinetic_energy']:.12e}, "
              f"rel {dk:.1e}); Z rel {dz:.1e}", flush=True)
        assert dk < 1e-12 and dz < 1e-12
