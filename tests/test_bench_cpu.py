"""Host logic of bench.py: the roofline entry (algorithmic bytes 8s/3 per DOF
per launch, divided by the measured average launch) and the stored HBM
traffic, which is reported only for the workload and precision it was
measured on and only while the kernel sources hash matches."""
import json

import pytest

import bench


def _res(precision, dof=1_000_000, stage_ms=2.0, launches=4):
    s = 8 if precision == 0 else 4
    alg = 8.0 * s / 3.0 if precision != 2 else 8.0
    return {"timing": {"stage_launches": launches, "stage_ms": stage_ms * launches},
            "alg_bytes_per_dof": alg, "dof": dof, "precision": precision}


def test_roofline_algorithmic_rate():
    r = bench.roofline(_res(0), 5, "box2d")
    assert r["avg_launch_ms"] == pytest.approx(2.0)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(8.0 * 8 / 3 * 1e6)
    assert r["achieved"] == pytest.approx(8.0 * 8 / 3 * 1e6 / 2e-3 / 1e9, abs=0.1)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, abs=1e-4)
    assert bench.roofline({"timing": {"stage_launches": 0, "stage_ms": 0.0}}, 5, "box2d") is None


def test_traffic_is_keyed_by_workload_precision_and_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    tf = tmp_path / "traffic.json"
    tf.write_text(json.dumps({"source_hash": h, "box2d/stage_f64": {"bytes_per_launch": 123.0},
                              "tgv3d/stage_f32": {"bytes_per_launch": 456.0}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tf))
    assert bench.roofline(_res(0), 5, "box2d")["traffic"] == 123.0
    assert bench.roofline(_res(1), 5, "tgv3d")["traffic"] == 456.0
    # no measurement for this workload or precision: null, never another one's
    assert bench.roofline(_res(1), 5, "mach2")["traffic"] is None
    assert bench.roofline(_res(1), 5, "box2d")["traffic"] is None
    # sources changed since the counters were taken: null
    tf.write_text(json.dumps({"source_hash": "0" * 16, "box2d/stage_f64": {"bytes_per_launch": 1.0}}))
    assert bench.roofline(_res(0), 5, "box2d")["traffic"] is None


def test_source_hash_ignores_comments(tmp_path):
    a = tmp_path / "a"
    b = tmp_path / "b"
    a.mkdir()
    b.mkdir()
    (a / "k.hip").write_text("int f() { return 1; }  // one\n/* block */\n")
    (b / "k.hip").write_text("int f()  {\n  return 1;\n}\n")
    assert bench.kernel_source_hash(str(a)) == bench.kernel_source_hash(str(b))
    (b / "k.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_hash(str(a)) != bench.kernel_source_hash(str(b))


def test_committed_traffic_matches_the_sources():
    """The committed counters were taken on the current kernel sources."""
    tr = json.load(open(bench.TRAFFIC_FILE))
    assert tr["source_hash"] == bench.kernel_source_hash()
    assert "box2d/stage_f64" in tr and "box2d/stage_f32" in tr
