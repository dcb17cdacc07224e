#!/usr/bin/env python3
"""Benchmark: boundary-element matvec pair-interactions per second inside
full polarisable solvation solves, and solve time at 1e-4 relative error in
the solvation energy, mixed precision against FP64, on one MI355X.

Workload: the 5000-atom synthetic globule (144236 panels, 5000 polarisable
multipole sites, treecode theta 0.5, P 5, leaf 300), the largest
configuration that one GPU holds.

One step = one complete pbmp_solve of the workload in mixed precision at the
loosest GMRES and induced-dipole tolerances whose solvation energy stays
within 1e-4 of the reference (table SOLVE_TOL, found by --calibrate): the
vacuum and dissolved induced-dipole loops, every GMRES solve with its
operator products, the right-hand sides, the site readouts, the
Coulomb/Thole fields and the energy.  value = (operator products in the
timed steps x panels x far-field nodes) / wall time of the timed steps:
direct-equivalent pair interactions per second (the treecode executes far
fewer; the executed counts are reported beside it).  Inputs are resident on
the device before timing starts.

After the timed steps: one FP64 solve at its own tolerances from the table,
and the reference -- an FP64 solve at GMRES 1e-10 / induced dipoles 1e-9 D
-- against which both energies' errors are reported.

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
# (FETCH_SIZE reads 0.50008 of the bytes read, WRITE_SIZE 1.0 of the bytes
# written).  Keyed by (mode, kernel, workload, precision); valid only while
# the sources of the kernel hash to the recorded value (otherwise traffic is
# reported null).
TRAFFIC = {
    ("treecode", "m2p", "globule_5000", "mixed"): {
        "fetch_kib": 4612.76, "fetch_scale": 0.50008, "write_kib": 139723.00,
        "write_scale": 1.0, "sha": "d7b0216f1432cb9e"},
    ("treecode", "p2p", "globule_5000", "mixed"): {
        "fetch_kib": 16974.85, "fetch_scale": 0.50008, "write_kib": 198625.44,
        "write_scale": 1.0, "sha": "d7b0216f1432cb9e"},
}
TRAFFIC_SOURCES = {
    "treecode": ["k_tree.hip", "pair.hpp", "tree.hpp", "k_treebuild.hip"],
    "direct": ["k_p2p.hip", "pair.hpp"],
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
    rec = TRAFFIC.get((mode, kernel, workload, precision))
    if rec is None or rec["sha"] != _sources_hash(TRAFFIC_SOURCES[mode]):
        return None
    return rec["fetch_kib"] * 1024 / rec["fetch_scale"] + rec["write_kib"] * 1024 / rec["write_scale"]


ALG_FLOP_PER_PAIR = 33  # four kernels per (target, far-field node) pair
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X published (packed FP32)
PEAK_FP32_NONPACKED = 78.6  # nominal: 256 CU x 64 lanes x 2 FLOP x 2.4 GHz
PEAK_FP64_VECTOR = 78.6  # TFLOP/s, MI355X published

# Loosest (GMRES tolerance, induced-dipole tolerance in Debye) per workload
# and precision whose solvation energy is within 5e-5 relative of the
# reference (half the 1e-4 target, a margin for other meshes of the same
# class); from `python bench.py --calibrate --workload W` (every pair of
# GMRES 1e-4..1e-6 and SCF 1e-2..1e-4 D; the fastest that qualifies).
SOLVE_TOL = {
    ("globule_5000", "mixed"): (1e-5, 1e-3),
    ("globule_5000", "fp64"): (1e-5, 1e-3),
}
REF_TOL = (1e-10, 1e-9)
CAL_GMRES = (1e-4, 1e-5, 1e-6)
CAL_SCF = (1e-2, 1e-3, 1e-4)


def _m2p_flops(order):
    """FLOP per (target, box) pair of the implemented M2P evaluation, not
    counting products with 1, terms with 0 or additions to 0.  Per
    coefficient k != 0 of the Laplace/Yukawa recurrences, which run to
    degree P + 1 (n1, n2 = number of k_i >= 1, >= 2): 6 n1 - 3 for the three
    sums over the first-lower coefficients, 3 (n2 - 1) for the three over
    the second-lower ones, and 5 (|k| = 1), 7 (no k_i >= 2) or 13 to combine
    them; 8 per coefficient of degree <= P for the four moment dot products
    and 4 per coefficient of degree P + 1 (double layer only); 14 for the
    pair set-up.  P = 4: 1546, P = 5: 2451."""
    total = 14
    for s in range(order + 2):
        for i in range(s, -1, -1):
            for j in range(s - i, -1, -1):
                k = (i, j, s - i - j)
                total += 8 if s <= order else 4
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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _progress(*args):
    """A progress line on stderr (stdout carries only the result line)."""
    print(*args, file=sys.stderr, flush=True)


def _make_solver(w, mode, precision, stream, dev, gmres_tol, scf_tol, warm_start=False):
    import torch
    from paper_1810_03698_amd import Solver
    p = w["params"]
    s = Solver(eps_in=p["eps_in"], eps_out=p["eps_out"], kappa=p["kappa"],
               gauss_far=int(p["gauss_far"]), near_eta=p["near_eta"],
               mode=mode, theta=p.get("theta", 0.5),
               order_P=int(p.get("order_P", 4)),
               leaf_panels=int(p.get("leaf_panels", 300)),
               gmres_restart=int(p["gmres_restart"]), gmres_tol=gmres_tol,
               gmres_maxit=20000, scf_tol_debye=scf_tol, scf_omega=p["scf_omega"],
               scf_maxit=500, thole_a=p["thole_a"], precision=precision,
               stream=stream.cuda_stream, warm_start=warm_start)
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    s.set_mesh(t(w["verts"]), t(w["tris"], torch.int32))
    s.set_sites(t(w["xyz"]), t(w["q"]), t(w["d"]), t(w["Q9"]), t(w["alpha"]))
    return s


def _timed_solve(s):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve(outputs=False)
    torch.cuda.synchronize()
    return r, 1e3 * (time.perf_counter() - t0)


def reference_solve(w, mode, stream, dev):
    """The reference energy: FP64 solves tightened in stages to REF_TOL, each
    starting from the last one's solution and dipoles (the stages only
    shorten the way to the same fixed point)."""
    s = _make_solver(w, mode, "fp64", stream, dev, 1e-6, 1e-6, warm_start=True)
    total = 0.0
    for gt, st in ((1e-6, 1e-6), (1e-8, 1e-7), REF_TOL):
        s.set_options(gmres_tol=gt, scf_tol_debye=st)
        r, ms = _timed_solve(s)
        total += ms
        _progress("reference stage", gt, st, "dG", r["dG"], "gmres", r["gmres_iters"],
                  "scf", r["scf_iters"], "%.0f ms" % ms)
    s.close()
    return r, total


def calibrate(w, mode, stream, dev, args):
    """Every (GMRES, SCF) tolerance pair of the grid in both precisions
    against the reference; prints one JSON line per solve and the table
    entry: the fastest pair within 5e-5."""
    ref, ref_ms = reference_solve(w, mode, stream, dev)
    print(json.dumps({"reference": ref["dG"], "ms": ref_ms, "tol": REF_TOL,
                      "gmres": ref["gmres_iters"], "scf": ref["scf_iters"]}), flush=True)
    for precision in ("mixed", "fp64"):
        best = None
        s = _make_solver(w, mode, precision, stream, dev, CAL_GMRES[0], CAL_SCF[0])
        _timed_solve(s)  # warm-up (first-solve set-up)
        for gt in CAL_GMRES:
            for st in CAL_SCF:
                s.set_options(gmres_tol=gt, scf_tol_debye=st)
                r, ms = _timed_solve(s)
                err = abs(r["dG"] - ref["dG"]) / abs(ref["dG"])
                print(json.dumps({"precision": precision, "gmres_tol": gt, "scf_tol": st,
                                  "ms": ms, "rel_err": err, "status": r["status"],
                                  "gmres": r["gmres_iters"], "scf": r["scf_iters"]}),
                      flush=True)
                if err <= 5e-5 and r["status"] == 0 and (best is None or ms < best[0]):
                    best = (ms, gt, st)
        s.close()
        print("SOLVE_TOL[(%r, %r)] = %r" % (args.workload, precision,
                                             None if best is None else best[1:]), flush=True)


def oracle_times(products):
    """Time to solution of the FP64 CPU oracle on this host: full solves
    (dense LU) of the 1280- and 5120-panel spheres, and for the larger
    workloads the time of one matrix-free O(N^2) product times the number
    of operator products the GPU solve of the same workload needed
    (extrapolated).  `products`: workload -> GPU product count (None: a
    product count is not available, report the product time only)."""
    import numpy as np
    from oracle import bie, solver as osolver
    from synth import workload
    out = {"cpu_model": _cpu_model(),
           "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}
    for name in ("sphere_1280", "sphere_5120"):
        w = workload(name)
        p = w["params"]
        t0 = time.perf_counter()
        sol = osolver.BemSolvent(w["verts"], w["tris"], p["eps_in"], p["eps_out"], p["kappa"])
        r = osolver.solvation(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"], sol,
                              tol_debye=p["scf_tol_debye"])
        out[name] = {"solve_s": time.perf_counter() - t0, "kind": "measured",
                     "scf_iters": r["scf_iters"], "dG": r["dG"]}
        _progress("oracle", name, out[name])
    for name, nprod in products.items():
        w = workload(name)
        m = bie.Mesh(w["verts"], w["tris"], w["params"]["kappa"])
        x = np.random.default_rng(0).normal(size=2 * m.N)
        rows = min(m.N, 2048)
        t0 = time.perf_counter()
        m.operator_sums(x[:m.N], x[m.N:], rows=(0, rows))
        t_prod = (time.perf_counter() - t0) * m.N / rows
        out[name] = {"product_s": t_prod, "kind": "extrapolated",
                     "gpu_products": nprod,
                     "solve_s": None if nprod is None else t_prod * nprod}
        _progress("oracle", name, out[name])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="globule_5000")
    ap.add_argument("--mode", default=None, help="direct | treecode (default: workload's)")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--gmres-tol", type=float, default=None,
                    help="override the calibrated tolerances of the timed solves")
    ap.add_argument("--scf-tol", type=float, default=None)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 solve and the reference after the timed steps")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="search the tolerance grid against the reference (prints the "
                         "SOLVE_TOL entries) instead of the benchmark")
    ap.add_argument("--oracle-times", default=None,
                    help="time the FP64 CPU oracle instead of the benchmark: full solves "
                         "of the two small spheres and, per 'workload=gpu_products' item "
                         "of this comma-separated list, one product extrapolated")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device copy first (the reference "
                         "dispatch for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU "
              "path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    if args.oracle_times is not None:
        products = {}
        for item in filter(None, args.oracle_times.split(",")):
            name, _, n = item.partition("=")
            products[name] = int(n) if n else None
        print(json.dumps({"oracle_times": oracle_times(products)}), flush=True)
        return

    import torch
    from synth import workload

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = workload(args.workload)
    p = w["params"]
    mode = args.mode or p["mode"]

    if args.calibrate:
        calibrate(w, mode, stream, dev, args)
        return

    if args.copy_calibration:
        a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def tol_for(precision):
        g, sc = SOLVE_TOL.get((args.workload, precision), (p["gmres_tol"], p["scf_tol_debye"]))
        return (args.gmres_tol or g, args.scf_tol or sc)

    N = len(w["tris"])
    G = int(p["gauss_far"]) * N
    gtol, stol = tol_for(args.precision)
    s = _make_solver(w, mode, args.precision, stream, dev, gtol, stol)
    _progress("workload", args.workload, "panels", N, "sites", len(w["q"]), "tolerances",
              gtol, stol)
    for _ in range(args.warmup):
        s.solve(outputs=False)
        _progress("warm-up solve done")
    s.kernel_stats(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs = 0
    res = None
    for k in range(args.steps):
        res = s.solve(outputs=False)
        matvecs += res["matvecs"]
        if k % 5 == 4:
            _progress("timed solves done:", k + 1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.kernel_stats(False)
    s.close()
    ms_per_step = 1e3 * elapsed / args.steps
    value = matvecs * float(N) * G / elapsed

    # dominant kernel: the one with the larger accumulated device time
    order = int(p.get("order_P", 4))
    p2p_avg = st["p2p_ms"] / max(1, st["p2p_launches"])
    m2p_avg = st["m2p_ms"] / max(1, st["m2p_launches"])
    if st["p2p_ms"] >= st["m2p_ms"]:
        name, avg_ms = "p2p", p2p_avg
        per_launch = ALG_FLOP_PER_PAIR * st["p2p_pairs"] / max(1, st["p2p_launches"])
    else:
        name, avg_ms = "m2p", m2p_avg
        per_launch = _m2p_flops(order) * st["m2p_pairs"] / max(1, st["m2p_launches"])
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    # the far field runs in FP32 in mixed precision and in FP64 otherwise
    peak = PEAK_FP32_VECTOR if args.precision == "mixed" else PEAK_FP64_VECTOR
    traffic = traffic_bytes(mode, name, args.workload, args.precision)
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "traffic_rate_GBps": (traffic / (avg_ms * 1e-3) / 1e9 if traffic else None),
                "kernel": name, "avg_launch_ms": avg_ms,
                "frac_of_nonpacked_fp32": (achieved / PEAK_FP32_NONPACKED
                                           if args.precision == "mixed" else None),
                "p2p_ms_total": st["p2p_ms"], "m2p_ms_total": st["m2p_ms"],
                "p2m_ms_total": st["p2m_ms"],
                "p2p_avg_ms": p2p_avg, "m2p_avg_ms": m2p_avg,
                "p2p_pairs_per_launch": st["p2p_pairs"] / max(1, st["p2p_launches"]),
                "m2p_pairs_per_launch": st["m2p_pairs"] / max(1, st["m2p_launches"]),
                "p2p_tflops_alg": ALG_FLOP_PER_PAIR * st["p2p_pairs"] / max(1e-30, st["p2p_ms"]) / 1e9,
                "m2p_tflops_alg": _m2p_flops(order) * st["m2p_pairs"]
                / max(1e-30, st["m2p_ms"]) / 1e9,
                "m2p_flop_per_pair": _m2p_flops(order)}
    executed = {"p2p_pairs_per_s": st["p2p_pairs"] / elapsed,
                "m2p_target_box_pairs_per_s": st["m2p_pairs"] / elapsed,
                "p2p_pairs_per_product": st["p2p_pairs"] / max(1, st["p2p_launches"]),
                "direct_pairs_per_product": float(N) * G}

    solve_cmp = None
    if not args.no_compare:
        g64, s64t = tol_for("fp64")
        s64 = _make_solver(w, mode, "fp64", stream, dev, g64, s64t)
        s64.solve(outputs=False)  # first-solve set-up, as the warm-up of the timed steps
        r64, fp64_ms = _timed_solve(s64)
        s64.close()
        _progress("fp64 solve done: %.0f ms; reference" % fp64_ms)
        ref, ref_ms = reference_solve(w, mode, stream, dev)
        err = lambda r: abs(r["dG"] - ref["dG"]) / abs(ref["dG"])
        solve_cmp = {"mixed_ms": ms_per_step, "fp64_ms": fp64_ms,
                     "speedup_mixed_over_fp64": fp64_ms / ms_per_step,
                     "mixed_tol": [gtol, stol], "fp64_tol": [g64, s64t],
                     "dG_mixed": res["dG"], "dG_fp64": r64["dG"], "dG_reference": ref["dG"],
                     "reference_tol": list(REF_TOL), "reference_ms": ref_ms,
                     "rel_err_mixed": err(res), "rel_err_fp64": err(r64),
                     "scf_iters": res["scf_iters"], "gmres_iters": res["gmres_iters"],
                     "fp64_scf_iters": r64["scf_iters"], "fp64_gmres_iters": r64["gmres_iters"],
                     "reference_gmres_iters": ref["gmres_iters"]}

    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        _progress("cpu baseline")
        cpu = cpu_baseline(w, args.cpu_seconds)
        cpu["cpu_model"] = _cpu_model()

    out = {
        "metric": "BEM matvec pair-interactions/s; solve time at 1e-4 dG error, mixed vs FP64",
        "value": value,
        "unit": "direct-equivalent pair-interactions/s",
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
                   "gmres_restart": p["gmres_restart"], "gmres_tol": gtol,
                   "scf_tol_debye": stol,
                   "matvecs_per_step": matvecs / args.steps,
                   "dG_kcal": res["dG"]},
        "roofline": roofline,
        "executed": executed,
        "cpu_baseline": cpu,
        "solve_at_1e-4_mixed_vs_fp64": solve_cmp,
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
