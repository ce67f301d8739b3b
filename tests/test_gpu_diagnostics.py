"""Taylor-Green histories on the GPU (FP64 and FP32 storage): mass is conserved,
kinetic energy decays in FP64, and the FP32 history stays within the stated
tolerance of the FP64 one (no reference data exists for this configuration)."""
import pytest

pytestmark = pytest.mark.gpu


def test_tgv_history_fp64_vs_fp32():
    import torch
    assert torch.cuda.is_available()
    from paper_2308_06196_amd import diagnostics as dg
    print("[case] tgv history n=4 p=3 nv1=12 steps=20", flush=True)
    rows = dg.tgv_history(n=4, order=3, nv1=12, steps=20, every=5)
    f64 = [r for r in rows if r["precision"] == "fp64"]
    f32 = {r["step"]: r for r in rows if r["precision"] == "fp32"}
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
