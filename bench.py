#!/usr/bin/env python3
"""Benchmark: boundary-element matvec pair-interactions per second inside
full polarisable solvation solves, and solve time mixed vs FP64, on one
MI355X.

One step = one complete pbmp_solve of the workload: vacuum and dissolved
induced-dipole loops, every GMRES solve with its operator products, the
right-hand sides, the site readouts, the Coulomb/Thole fields and the
energy.  value = (operator products in the timed steps x panels x far-field
nodes) / wall time of the timed steps (direct-equivalent pair interactions
per second).  Inputs are resident on the device before timing starts.

Prints one JSON line.  Use --gpus 1 (the only supported count).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20

# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch, mean over the dispatches
# of one solve) scaled by what the counters read for a 256 MiB copy
# (FETCH_SIZE reads 0.5001 of the bytes read, WRITE_SIZE 1.0 of the bytes
# written).  Keyed by (mode, kernel); valid only for the workload and precision measured
# and while the sources of the kernel hash to the recorded value (otherwise
# traffic is reported null).
TRAFFIC = {
    ("treecode", "p2p"): {"workload": "sphere_81920", "precision": "mixed", "fetch_kib": 5843.61, "fetch_scale": 0.50006,
                          "write_kib": 51638.60, "write_scale": 1.0, "sha": "486e9fb11d200fa2"},
    ("direct", "p2p"): {"workload": "sphere_81920", "precision": "mixed", "fetch_kib": 20980.51, "fetch_scale": 0.50006,
                        "write_kib": 33280.0, "write_scale": 1.0, "sha": "614bbeac61608d8e"},
}
TRAFFIC_SOURCES = {
    ("treecode", "p2p"): ["k_tree.hip", "pair.hpp", "tree.hpp", "k_treebuild.hip"],
    ("direct", "p2p"): ["k_p2p.hip", "pair.hpp"],
}


def _sources_hash(files):
    import hashlib
    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1810_03698_amd", "csrc")
    for f in files:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(mode, kernel, workload, precision):
    rec = TRAFFIC.get((mode, kernel))
    if rec is None or rec["workload"] != workload or rec["precision"] != precision:
        return None
    if rec["sha"] != _sources_hash(TRAFFIC_SOURCES[(mode, kernel)]):
        return None
    return rec["fetch_kib"] * 1024 / rec["fetch_scale"] + rec["write_kib"] * 1024 / rec["write_scale"]
ALG_FLOP_PER_PAIR = 33  # four kernels per (target, far-field node) pair
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X published (packed FP32)
PEAK_FP32_NONPACKED = 78.6  # nominal: 256 CU x 64 lanes x 2 FLOP x 2.4 GHz
PEAK_FP64_VECTOR = 78.6  # TFLOP/s, MI355X published


def _m2p_flops(order):
    """FLOP per (target, box) pair of the implemented M2P evaluation, not
    counting products with 1, terms with 0 or additions to 0.  Per
    coefficient k != 0 of the Laplace/Yukawa recurrences (n1, n2 = number of
    k_i >= 1, >= 2): 6 n1 - 3 for the three sums over the first-lower
    coefficients, 3 (n2 - 1) for the three over the second-lower ones, and 5
    (|k| = 1), 7 (no k_i >= 2) or 13 to combine them; 8 per coefficient for
    the four moment dot products; 14 for the pair set-up.  P = 4: 955,
    P = 5: 1630."""
    total = 14
    for s in range(order + 1):
        for i in range(s, -1, -1):
            for j in range(s - i, -1, -1):
                k = (i, j, s - i - j)
                total += 8
                if not s:
                    continue
                n1 = sum(e >= 1 for e in k)
                n2 = sum(e >= 2 for e in k)
                total += 6 * n1 - 3 + (3 * (n2 - 1) if n2 else 0)
                total += 5 if s == 1 else (7 if n2 == 0 else 13)
    return total


def cpu_baseline(w, target_seconds):
    """Time the FP64 CPU oracle's direct operator sums on a bounded sample of
    target rows of the same workload; returns pair-interactions per second."""
    import numpy as np
    from oracle import bie
    m = bie.Mesh(w["verts"], w["tris"], w["params"]["kappa"])
    N = m.N
    rng = np.random.default_rng(0)
    x = rng.normal(size=2 * N)
    m.operator_sums(x[:N], x[N:], rows=(0, 8))  # thread pool start-up
    rows = 256
    t0 = time.perf_counter()
    m.operator_sums(x[:N], x[N:], rows=(0, rows))
    dt = time.perf_counter() - t0
    rows = int(min(N, max(rows, rows * target_seconds / max(dt, 1e-6))))
    t0 = time.perf_counter()
    m.operator_sums(x[:N], x[N:], rows=(0, rows))
    dt = time.perf_counter() - t0
    pairs = rows * N * 3.0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    one = _one_core_rate(w, max(1.0, target_seconds / 4))
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": cores,
            "kind": "oracle",
            "sample": "FP64 oracle direct operator sums (all four kernels, "
                      "near/self rules included) for target rows 0..%d of the "
                      "%d-panel workload: %.3e pairs in %.1f s" % (rows, N, pairs, dt),
            "one_core_value": one}


_ONE_CORE = """
import sys, time, numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import bie
z = np.load(sys.argv[2])
m = bie.Mesh(z["verts"], z["tris"], float(z["kappa"]))
x = np.random.default_rng(0).normal(size=2 * m.N)
rows, dt = 8, 0.0
while dt < float(sys.argv[3]) and rows < m.N:
    rows = min(m.N, rows * 4)
    t0 = time.perf_counter()
    m.operator_sums(x[:m.N], x[m.N:], rows=(0, rows))
    dt = time.perf_counter() - t0
print(rows * m.N * 3.0 / dt)
"""


def _one_core_rate(w, seconds):
    """The same oracle sums on one thread (a child process with
    OMP_NUM_THREADS=1), pair-interactions per second."""
    import subprocess
    import tempfile
    import numpy as np
    root = os.path.dirname(os.path.abspath(__file__))
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "mesh.npz")
        np.savez(f, verts=w["verts"], tris=w["tris"], kappa=w["params"]["kappa"])
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", _ONE_CORE, root, f, str(seconds)],
                           env=env, capture_output=True, text=True, timeout=600)
    try:
        return float(r.stdout.strip().splitlines()[-1])
    except (ValueError, IndexError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_81920")
    ap.add_argument("--mode", default=None, help="direct | treecode (default: workload's)")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="FP64 solves timed for the mixed-vs-FP64 comparison (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device copy first (the reference "
                         "dispatch for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU "
              "path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    from paper_1810_03698_amd import Solver
    from synth import workload

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = workload(args.workload)
    p = w["params"]
    mode = args.mode or p["mode"]

    def make(precision):
        s = Solver(eps_in=p["eps_in"], eps_out=p["eps_out"], kappa=p["kappa"],
                   gauss_far=int(p["gauss_far"]), near_eta=p["near_eta"],
                   mode=mode, theta=p.get("theta", 0.5),
                   order_P=int(p.get("order_P", 4)),
                   leaf_panels=int(p.get("leaf_panels", 300)),
                   gmres_restart=int(p["gmres_restart"]), gmres_tol=p["gmres_tol"],
                   scf_tol_debye=p["scf_tol_debye"], scf_omega=p["scf_omega"],
                   thole_a=p["thole_a"], precision=precision,
                   stream=stream.cuda_stream)
        t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
        s.set_mesh(t(w["verts"]), t(w["tris"], torch.int32))
        s.set_sites(t(w["xyz"]), t(w["q"]), t(w["d"]), t(w["Q9"]), t(w["alpha"]))
        return s

    if args.copy_calibration:
        a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    N = len(w["tris"])
    G = int(p["gauss_far"]) * N
    s = make(args.precision)
    for _ in range(args.warmup):
        s.solve(outputs=False)
    s.kernel_stats(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs = 0
    res = None
    for _ in range(args.steps):
        res = s.solve(outputs=False)
        matvecs += res["matvecs"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.kernel_stats(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = matvecs * float(N) * G / elapsed

    # dominant kernel: the one with the larger accumulated device time
    p2p_avg = st["p2p_ms"] / max(1, st["p2p_launches"])
    m2p_avg = st["m2p_ms"] / max(1, st["m2p_launches"])
    if st["p2p_ms"] >= st["m2p_ms"]:
        name, avg_ms = "p2p", p2p_avg
        per_launch = ALG_FLOP_PER_PAIR * st["p2p_pairs"] / max(1, st["p2p_launches"])
    else:
        name, avg_ms = "m2p", m2p_avg
        per_launch = _m2p_flops(int(p.get("order_P", 4))) * st["m2p_pairs"] / max(1, st["m2p_launches"])
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    # the far field runs in FP32 in mixed precision and in FP64 otherwise
    peak = PEAK_FP32_VECTOR if args.precision == "mixed" else PEAK_FP64_VECTOR
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic_bytes(mode, name, args.workload, args.precision), "traffic_unit": "bytes per launch",
                "kernel": name, "avg_launch_ms": avg_ms,
                "frac_of_nonpacked_fp32": (achieved / PEAK_FP32_NONPACKED
                                           if args.precision == "mixed" else None),
                "p2p_ms_total": st["p2p_ms"], "m2p_ms_total": st["m2p_ms"],
                "p2m_ms_total": st["p2m_ms"],
                "p2p_avg_ms": p2p_avg, "m2p_avg_ms": m2p_avg,
                "p2p_pairs_per_launch": st["p2p_pairs"] / max(1, st["p2p_launches"]),
                "m2p_pairs_per_launch": st["m2p_pairs"] / max(1, st["m2p_launches"]),
                "p2p_tflops_alg": ALG_FLOP_PER_PAIR * st["p2p_pairs"] / max(1e-30, st["p2p_ms"]) / 1e9,
                "m2p_tflops_alg": _m2p_flops(int(p.get("order_P", 4))) * st["m2p_pairs"]
                / max(1e-30, st["m2p_ms"]) / 1e9}

    solve_cmp = None
    if args.fp64_steps > 0:
        s64 = make("fp64")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = None
        for _ in range(args.fp64_steps):
            r64 = s64.solve(outputs=False)
        torch.cuda.synchronize()
        fp64_ms = 1e3 * (time.perf_counter() - t1) / args.fp64_steps
        solve_cmp = {"mixed_ms": ms_per_step, "fp64_ms": fp64_ms,
                     "speedup_mixed_over_fp64": fp64_ms / ms_per_step,
                     "dG_mixed": res["dG"], "dG_fp64": r64["dG"],
                     "dG_rel_diff": abs(res["dG"] - r64["dG"]) / abs(r64["dG"]),
                     "scf_iters": res["scf_iters"], "gmres_iters": res["gmres_iters"],
                     "fp64_gmres_iters": r64["gmres_iters"]}
        s64.close()

    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": "BEM matvec pair-interactions/s; solve time at 1e-4 dG error, mixed vs FP64",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "panels": N, "far_nodes": G,
                   "sites": len(w["q"]), "mode": mode, "precision": args.precision,
                   "theta": p.get("theta"), "order_P": p.get("order_P"),
                   "leaf_panels": p.get("leaf_panels"),
                   "gmres_restart": p["gmres_restart"], "gmres_tol": p["gmres_tol"],
                   "scf_tol_debye": p["scf_tol_debye"],
                   "matvecs_per_step": matvecs / args.steps,
                   "dG_kcal": res["dG"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "solve_mixed_vs_fp64": solve_cmp,
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
