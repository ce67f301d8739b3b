"""Throughput benchmark of the BGK phase-space hot path on one MI355X.

One step = one full SSP-RK3 step (three residual evaluations with the fused
stage kernel, three equilibrium solves) of the whole phase space, inputs
resident in HBM. Default workload: the 2-D periodic box (32x32 elements,
p=3, 24^3 velocities on [-6,6]^3, Kn=1e-3; 226,492,416 phase-space DOF), run
in FP64 and with FP32 bulk storage / FP64 collision side by side.

Prints one JSON line: value = FP64 DOF-updates/s; "mixed" holds the FP32-bulk
path, "mixed_bf16" the path with an FP32 state and BF16 stage increments;
"roofline" the dominant kernel (fused stage) against HBM peak;
"collision_conservation" the largest relative discrete moment of the collision
term of each path's final state; "workloads" the 3-D Taylor-Green box (FP32,
BF16 increments, FP64), the Mach-2 box (FP32) and the shock tube (FP64, its
100 steps), each with its roofline entry; "serving" the request mix (batched
server against the plain FP64 path); "cpu_baseline" the FP64 oracle timed on
a bounded sample on the host's cores (all of them and one), and on the whole
shock tube (100 steps, all cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "phase-space DOF-updates/s FP64 vs mixed; p50/p99 latency of batched solves"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def workload(name):
    from paper_2308_06196_amd import workloads as wl
    if name == "box2d":
        return wl.box2d(), wl.prim_box2d, ("box2d: 2-D periodic box [0,1]^2, 32x32 elements p=3, "
                                           "24^3 velocities on [-6,6]^3, Kn=1e-3, SSP-RK3, CFL 0.1")
    if name == "sod1d":
        return wl.sod1d(), wl.prim_sod, ("sod1d: shock tube, 32 elements p=2, 16^3 velocities on "
                                         "[-6,6]^3, Kn=1e-2, specular walls, SSP-RK3, CFL 0.1")
    if name == "tgv3d":
        return wl.tgv3d(), wl.prim_tgv3d, ("tgv3d: 3-D periodic Taylor-Green box, 16^3 elements "
                                           "p=3, 16^3 velocities on [-5,5]^3, Kn=1e-3")
    if name == "mach2":
        return wl.mach2(), wl.prim_mach2, ("mach2: 3-D periodic box, 32^3 elements p=2, 20^3 "
                                           "velocities on [-8,8]^3, Kn=1e-2, Mach 2")
    raise SystemExit(f"unknown workload {name}")


# host-side runtime sources: they do not change what a stage kernel reads or writes
HOST_SOURCES = ("bgk_runtime.hip", "bgk_launch.hpp")


def kernel_source_hash(csrc: str | None = None) -> str:
    """Hash of the compile flags and the kernel sources (device code and launch
    configuration; the host runtime excluded) with comments and whitespace
    removed, so that the
    stored HBM traffic (profiles/traffic.json) is used only for the kernels it
    was measured on."""
    import re
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2308_06196_amd", "csrc")
    # compile flags that shape the device code (include paths left out)
    from paper_2308_06196_amd import build as _build
    fl = _build.FLAGS
    h.update(" ".join(f for i, f in enumerate(fl)
                      if f != "-I" and not (i and fl[i - 1] == "-I")).encode() + b"\0")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".hpp")) and fn not in HOST_SOURCES:
            src = open(os.path.join(csrc, fn)).read()
            src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
            src = re.sub(r"//[^\n]*", " ", src)
            h.update(fn.encode() + b"\0" + " ".join(src.split()).encode())
    return h.hexdigest()[:16]


DTYPE = {0: "f64", 1: "f32-bulk/f64-collision",
         2: "f32-state/bf16-stage-increments/f64-collision"}


def collision_conservation(s, pb):
    """Largest relative discrete moment of the collision term of the solver's
    state (bgk_collision_moments), scaled per node by (rho, rho, rho, rho, E)/tau."""
    import numpy as np
    Q = s.moments().cpu().numpy()
    Cm = s.collision_moments().cpu().numpy()
    gamma = pb["gamma"] or 5.0 / 3.0
    rho, E = Q[:, 0], Q[:, 4]
    P = (gamma - 1.0) * (E - 0.5 * (Q[:, 1:4] ** 2).sum(1) / rho)
    th = P / rho
    mu = pb["mu_ref"] * (th / pb["theta_ref"]) ** pb["omega"]
    scale = np.column_stack([rho] * 4 + [E]) * (P / mu)[:, None]
    return float((np.abs(Cm) / scale).max())


def run_gpu(pb, prim_fn, precision, steps, warmup, conservation=False):
    import torch

    from paper_2308_06196_amd import bgk
    s = bgk.Solver(pb, precision=precision, device="cuda:0")
    s.set_maxwellian(prim_fn(s.node_coords()))
    dt = s.stable_dt(0.1)
    if warmup:
        s.rk3_step(dt, warmup)
    s.synchronize()
    s.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.rk3_step(dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = s.timing_read()
    s.timing(False)
    diag = s.diagnostics()
    cons = collision_conservation(s, pb) if conservation else None
    dof = s.nx * s.nv
    out = {"dof": dof, "elapsed_s": el, "ms_per_step": 1e3 * el / steps,
           "value": dof * steps / el, "timing": tm, "diag": diag, "dt": dt,
           "precision": precision, "collision_conservation": cons,
           # compulsory bytes per DOF per stage launch, averaged over the three
           # stages: 8s/3 for a stored state of s bytes (read input, [read f^n],
           # write output); BF16 increments: (4+2, 4+2+2, 4+2+4) B = 8 B
           "alg_bytes_per_dof": 8.0 if precision == 2 else 8.0 * (8 if precision == 0 else 4) / 3.0}
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def roofline(res, steps, workload):
    """Fused stage kernel: algorithmic bytes = compulsory f traffic, 2s (stage 1:
    read input, write output) + 3s + 3s (stages 2, 3: also read f^n) per DOF,
    i.e. 8s/3 per DOF per launch on average (BF16 increments: 8 B). The
    measured traffic is the one stored for this workload and precision."""
    tm = res["timing"]
    n = tm["stage_launches"]
    if not n:
        return None
    avg_ms = tm["stage_ms"] / n
    bytes_per_launch = res["alg_bytes_per_dof"] * res["dof"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    try:
        tr = json.load(open(TRAFFIC_FILE))
        key = workload + "/stage_" + {0: "f64", 1: "f32", 2: "bf16"}[res["precision"]]
        if tr.get("source_hash") == kernel_source_hash() and key in tr:
            traffic = tr[key]["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_stage (fused FR transport + BGK relaxation + SSP-RK combine + limiter "
                      "+ moment partials)",
            "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": bytes_per_launch}


def cpu_baseline(pb_full, prim_fn, budget_s=12.0):
    """FP64 oracle (plain, untuned) on the same workload restricted to an 8x8-element
    box (same p, velocity grid, IC and Kn); DOF-updates/s over as many steps as fit
    in about budget_s seconds."""
    import numpy as np

    from oracle import oracle as orc
    from paper_2308_06196_amd import workloads as wl  # noqa: F401
    keys = ["dim", "order", "nelem", "xlo", "xhi", "nvel", "vlo", "vhi", "bc", "mu_ref",
            "theta_ref", "omega", "gamma", "limiter", "newton_maxit", "newton_tol"]
    pb = dict(pb_full)
    d = pb["dim"]
    pb["nelem"] = [min(8, n) if k < d else 1 for k, n in enumerate(pb["nelem"])]
    pr = orc.Problem(**{k: pb[k] for k in keys})
    f = orc.maxwellian(pr, prim_fn(orc.node_coords(pr)))
    dt = orc.stable_dt(pr, f, 0.1)
    t0 = time.perf_counter()
    f, _ = orc.rk3_step(pr, f, dt, 1)
    t1 = time.perf_counter() - t0
    more = max(0, int(budget_s / max(t1, 1e-3)) - 1)
    t0 = time.perf_counter()
    if more:
        f, _ = orc.rk3_step(pr, f, dt, more)
    t2 = time.perf_counter() - t0
    steps = 1 + more
    dof = pr.nx * pr.nv
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": dof * steps / (t1 + t2), "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{'x'.join(str(n) for n in pb['nelem'][:d])} elements of the same workload "
                      f"({dof} DOF), {steps} SSP-RK3 steps, {t1 + t2:.1f} s, FP64, "
                      f"direct velocity sums"}


def cpu_full_run(pb, prim_fn, steps):
    """FP64 oracle (plain, untuned) on the whole workload for `steps` SSP-RK3
    steps (the shock tube: small enough to run in full within the bounded CPU
    budget); DOF-updates/s."""
    from oracle import oracle as orc
    keys = ["dim", "order", "nelem", "xlo", "xhi", "nvel", "vlo", "vhi", "bc", "mu_ref",
            "theta_ref", "omega", "gamma", "limiter", "newton_maxit", "newton_tol"]
    pr = orc.Problem(**{k: pb[k] for k in keys})
    f = orc.maxwellian(pr, prim_fn(orc.node_coords(pr)))
    dt = orc.stable_dt(pr, f, 0.1)
    t0 = time.perf_counter()
    f, _ = orc.rk3_step(pr, f, dt, steps)
    el = time.perf_counter() - t0
    dof = pr.nx * pr.nv
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": dof * steps / el, "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle", "sample": f"the whole workload ({dof} DOF), {steps} SSP-RK3 "
                                        f"steps, {el:.2f} s, FP64, direct velocity sums"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_in_process(workload_name, threads, budget_s, full_steps=0):
    """cpu_baseline (or, with full_steps, cpu_full_run) in a child process with
    OMP_NUM_THREADS = threads (the oracle's OpenMP team size is fixed when its
    library loads)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
           "--workload", workload_name, "--cpu-budget", str(budget_s)]
    if full_steps:
        cmd += ["--cpu-full-steps", str(full_steps)]
    out = subprocess.run(cmd, env=env, capture_output=True, text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def serving(n_requests, steps, seed=0, pool_gb=200.0, max_members=8, quantum=4,
            kinds=("sod1d", "box2d"), policy="sjf", large_dof=2.5e8):
    """Serving mix (shock tubes and periodic boxes, p in 1..3, 8^3..32^3 velocities,
    Kn log-uniform [1e-4, 1], 100 steps each). A saturating run (all requests at
    t = 0) measures the capacity; then the same requests arrive as a Poisson
    stream at 0.8 x that rate. The comparator is the plain FP64 path: the same
    kernels launched directly, one request at a time in arrival order, no
    overlap, on the same two arrival patterns, timed on the wall clock with the
    same set-up work per request (solver, initial state, time step). Both take
    the requests' workspaces from one device arena of the pool's size."""
    from paper_2308_06196_amd import serve
    from paper_2308_06196_amd import workloads as wl
    pool = int(pool_gb * (1 << 30))

    def reqs(rate):
        return serve.make_requests(wl.serving_requests(n=n_requests, seed=seed, rate=rate,
                                                       steps=steps, kinds=kinds))

    def batched(rate):
        ex = serve.BatchExecutor(max_members=max_members, arena_bytes=pool)
        m = serve.Server(ex, pool, max_members=max_members, quantum=quantum,
                         policy=policy, large_dof=large_dof).run(reqs(rate))
        ex.close()
        return m

    def say(what, m):
        print(f"[bench] serving {what}: {m['completed']} of {m['requests']} completed in "
              f"{m['span_s']:.2f} s, p50 {m['p50_s']:.3f} s", file=sys.stderr, flush=True)

    sat = batched(None)
    say("batched, all at t = 0", sat)
    cap_rate = sat["completed"] / sat["span_s"]
    pois = batched(0.8 * cap_rate)
    say("batched, Poisson", pois)
    seq_sat = serve.run_sequential(reqs(None), pool, arena=True)
    say("sequential FP64, all at t = 0", seq_sat)
    seq_pois = serve.run_sequential(reqs(0.8 * cap_rate), pool, arena=True)
    say("sequential FP64, Poisson", seq_pois)
    return {"requests": n_requests, "steps_each": steps, "kinds": list(kinds),
            "policy": policy, "max_members": max_members, "workspaces": "device arena",
            "large_dof": large_dof, "max_large": 1,
            "total_dof": int(sum(r.dof for r in reqs(None))),
            "capacity_requests_per_s": cap_rate, "poisson_rate_per_s": 0.8 * cap_rate,
            "batched_saturating": sat, "batched_poisson": pois,
            "sequential_fp64_saturating": seq_sat, "sequential_fp64_poisson": seq_pois}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="box2d")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64",
                    help="precision of the headline value")
    ap.add_argument("--serving", type=int, default=256, metavar="N",
                    help="requests in the serving mix (0: skip)")
    ap.add_argument("--serving-steps", type=int, default=100)
    ap.add_argument("--serving-policy", default="sjf", choices=["fifo", "sjf"],
                    help="admission order of the batched server")
    ap.add_argument("--serving-large-dof", type=float, default=2.5e8,
                    help="requests of this many phase-space DOF or more run one at a time "
                         "beside the small ones (0: no limit)")
    ap.add_argument("--serving-members", type=int, default=8,
                    help="requests resident in the batch at once")
    ap.add_argument("--serving-kinds", default="sod1d,box2d",
                    help="request kinds of the serving mix (sod1d, box2d, channel2d)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the Taylor-Green and Mach-2 lines")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only time the CPU oracle on the workload's sample and print it")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-full-steps", type=int, default=0, metavar="N",
                    help="with --cpu-baseline-only: run the whole workload for N steps")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times); "
                         "calibrates the HBM byte counters against a known traffic")
    a = ap.parse_args()
    if a.copy_probe:
        import torch
        src = torch.ones(a.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 3}))
        return
    if a.cpu_baseline_only:
        pb, prim_fn, _ = workload(a.workload)
        if a.cpu_full_steps:
            print(json.dumps(cpu_full_run(pb, prim_fn, a.cpu_full_steps)), flush=True)
        else:
            print(json.dumps(cpu_baseline(pb, prim_fn, a.cpu_budget)), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)
    pb, prim_fn, desc = workload(a.workload)
    main_prec = {"fp64": 0, "fp32": 1, "bf16": 2}[a.precision]
    res = run_gpu(pb, prim_fn, main_prec, a.steps, a.warmup, conservation=True)
    print(f"[bench] {a.workload} {a.precision}: {res['value']:.4e} DOF-updates/s, "
          f"{res['ms_per_step']:.3f} ms/step, timing {res['timing']}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": res["value"], "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[main_prec], "data": "synthetic",
        "config": {"workload": desc, "dof": res["dof"], "dt": res["dt"],
                   "newton_it_max": res["diag"]["newton_it_max"],
                   "limiter_hits": res["diag"]["limiter_hits"]},
        "roofline": roofline(res, a.steps, a.workload),
    }
    cons = {DTYPE[main_prec]: res["collision_conservation"]}
    if not a.no_mixed and main_prec == 0:
        for key, prec, label in (("mixed", 1, "fp32-bulk"), ("mixed_bf16", 2, "bf16-increments")):
            mx = run_gpu(pb, prim_fn, prec, a.steps, a.warmup, conservation=True)
            print(f"[bench] {a.workload} {label}: {mx['value']:.4e} DOF-updates/s, "
                  f"{mx['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
            line[key] = {"dtype": DTYPE[prec], "value": mx["value"],
                         "ms_per_step": mx["ms_per_step"],
                         "roofline": roofline(mx, a.steps, a.workload)}
            cons[DTYPE[prec]] = mx["collision_conservation"]
    # discrete moments of the collision term of the final state, relative
    # (the benchmark spec target 1e-13), per storage precision
    line["collision_conservation"] = cons
    if not a.no_workloads and a.workload == "box2d":
        # the 3-D Taylor-Green box (FP32, BF16 increments, FP64) and the Mach-2 box
        # (FP32), each with the roofline entry of its stage kernel
        line["workloads"] = {}
        for name, prec, steps in (("tgv3d", 1, 5), ("tgv3d", 2, 5), ("tgv3d", 0, 3),
                                  ("mach2", 1, 3), ("sod1d", 0, 100)):
            wpb, wprim, wdesc = workload(name)
            r = run_gpu(wpb, wprim, prec, steps, 1)
            key = f"{name}_{['fp64', 'fp32', 'bf16'][prec]}"
            line["workloads"][key] = {
                "workload": wdesc, "dtype": DTYPE[prec], "dof": r["dof"], "steps": steps,
                "value": r["value"], "unit": "DOF-updates/s", "ms_per_step": r["ms_per_step"],
                "roofline": roofline(r, steps, name)}
            print(f"[bench] {key}: {r['value']:.4e} DOF-updates/s, {r['ms_per_step']:.3f} ms/step, "
                  f"stage frac {line['workloads'][key]['roofline']['frac']}",
                  file=sys.stderr, flush=True)
    if a.serving:
        sv = serving(a.serving, a.serving_steps, kinds=tuple(a.serving_kinds.split(",")),
                     policy=a.serving_policy, max_members=a.serving_members,
                     large_dof=a.serving_large_dof or None)
        line["serving"] = sv
        p, q = sv["batched_poisson"], sv["sequential_fp64_poisson"]
        print(f"[bench] serving {a.serving} requests: batched p50 {p['p50_s']:.3f} s, p99 "
              f"{p['p99_s']:.3f} s (sequential FP64 p50 {q['p50_s']:.3f} s, p99 {q['p99_s']:.3f} s);"
              f" saturating {sv['batched_saturating']['dof_updates_per_s']:.3e} vs "
              f"{sv['sequential_fp64_saturating']['dof_updates_per_s']:.3e} DOF-updates/s",
              file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cb = cpu_baseline_in_process(a.workload, threads, a.cpu_budget)
        one = cpu_baseline_in_process(a.workload, 1, a.cpu_budget)
        cb["cpu_model"] = cpu_model()
        cb["single_core"] = {"value": one["value"], "cores": one["cores"], "sample": one["sample"]}
        if a.workload == "box2d":
            # the shock tube (32 elements, p = 2, 16^3 velocities) in full, 100 steps
            c1 = cpu_baseline_in_process("sod1d", threads, a.cpu_budget, full_steps=100)
            cb["sod1d_full"] = {"value": c1["value"], "cores": c1["cores"], "sample": c1["sample"]}
        line["cpu_baseline"] = cb
        print(f"[bench] cpu baseline {line['cpu_baseline']}", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
