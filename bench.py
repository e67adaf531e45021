#!/usr/bin/env python3
"""Benchmark of the dense fractional-Laplacian hot path on one MI355X.

Default workload (the paper's 2D test domain, Sec. 7, at the largest size
that one GPU holds): unit disk, seeded jittered-Delaunay quasi-uniform mesh
of 199,452 triangles, 99,205 interior DOFs (the FP64 matrix takes 80 GB),
s in {0.25, 0.75}, f = 1.  One step = mesh ingest (fl_set_mesh), then for
each s: FP64 assembly of A^s (all element pairs and element/boundary-facet
pairs; the s-independent plan -- element order, DOF map, pair classes,
tiles -- is made by the first assembly of the step and reused by the
second), load vector, Jacobi-PCG to ||r|| <= 1e-10 ||b||, energy-norm
error against the closed-form solution.
Everything runs in libfraclap.so; inputs are resident before the timed
region.  ``--workload disk8k`` runs the ~7.9k-triangle disk instead.

Prints ONE JSON line (rank 0, N = 1).  Metric: element-pair quadratures per
second over the whole step (pairs = T(T+1)/2 element pairs + T*B
element/facet pairs per assembly), plus the dense matvec bandwidth, the
roofline of the dominant kernel (and of the other one), the mixed-precision
+ surrogate form against FP64 at equal energy-norm error on the same
workload, the extra legs (7.9k-triangle disk; batched solves of the
~16k-DOF disk with 8 values of s and 64 right-hand sides; the surrogate on
the graded L-shape) and the CPU oracle baseline.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element-pair quadratures/s & matvec GB/s; mixed+surrogate vs FP64 at equal err"
HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic work per kernel evaluation |x - y|^{-2-2s} on the separated
# path: r^2 from the two mapped points (2 differences, 2 squares, 1 add),
# the power's multiply (pe * log r^2), and four FMAs of accumulation
# (8 flops) -- 14 flops -- plus two transcendentals (log, exp), which are
# counted apart.
FLOPS_PER_EVAL = 14
TRANS_PER_EVAL = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("disk200k", "disk8k"), default="disk200k",
                    help="disk200k: ~2e5 triangles, ~1e5 interior DOFs (default); disk8k: ~7.9k triangles")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FL_MIXED + surrogate leg on the benchmark workload")
    ap.add_argument("--no-c2", action="store_true", help="skip the 7.9k-triangle disk leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64, help="DOF rows of the all-core oracle sample")
    ap.add_argument("--cpu-rows-1core", type=int, default=2, help="DOF rows of the one-core oracle sample")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched leg (disk ~16k DOFs, 8 values of s, 64 right-hand sides)")
    ap.add_argument("--batch-cells", type=int, default=32000)
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the batched leg and print its object (profiling)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate leg (graded L-shape, ~37.7k triangles, s = 0.5)")
    ap.add_argument("--only-surrogate", action="store_true",
                    help="run only the surrogate leg and print its object (profiling)")
    ap.add_argument("--sur-train", type=int, default=65536, help="training pairs of the surrogate")
    ap.add_argument("--sur-steps", type=int, default=20000, help="Adam steps of the surrogate")
    ap.add_argument("--sur-tol", type=float, default=0.02, help="certified bound for the surrogate")
    ap.add_argument("--no-cluster", action="store_true",
                    help="skip the cluster-method leg (disks of ~3.2e4, ~2e5 and ~4e5 triangles)")
    ap.add_argument("--all-legs", action="store_true",
                    help="also run the multigrid, a posteriori and symmetry legs")
    ap.add_argument("--only-mg", action="store_true", help="run only the multigrid leg and print its object")
    ap.add_argument("--only-indicators", action="store_true",
                    help="run only the a posteriori leg and print its object")
    ap.add_argument("--only-cluster", action="store_true", help="run only the cluster leg and print its object")
    ap.add_argument("--only-symmetry", action="store_true", help="run only the symmetry leg and print its object")
    ap.add_argument("--only-mixed-assembly", action="store_true",
                    help="run only the FL_MIXED assembly of the benchmark disk (both s; the FP32 counter runs) "
                         "and print its object")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 launches) and exit: the "
                         "reference for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of the benchmark workload (scaled by a plain copy's
    counters), per kernel group; a group's figure is dropped (None) when the
    source file of its kernels changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic_disk200k.json")) as f:
            t = json.load(f)
    except OSError:
        return {}
    out = {}
    for key in ("cg_iteration", "separated_pairs"):
        ent = t.get(key) or {}
        try:
            with open(os.path.join(ROOT, "paper_1708_03912_amd", "csrc", ent["source"]), "rb") as f:
                sha = hashlib.sha256(f.read()).hexdigest()
        except (OSError, KeyError):
            continue
        if sha == ent.get("source_sha256"):
            out[key] = ent["bytes_per_launch"]
    return out


def copy_calib(mib):
    """Plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE of one launch
    should read mib * 1024 KiB each; the ratio scales the kernels' counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calib_KiB_per_launch": mib * 1024, "launches": 3}), flush=True)


def ball_fu(s):
    """(f, u) for f = 1 on the unit disk (Sec. 7 closed form
    u = c (1 - |x|^2)^s, c = 2^{-2s} Gamma(1) / Gamma(1 + s)^2 in 2D):
    c pi / (s + 1)."""
    c = 2.0 ** (-2 * s) / (math.gamma(1 + s) * math.gamma(1 + s))
    return c * math.pi / (s + 1.0)


def dense_leg(args, mesh, svals, dof_mode, rtol, steps, warmup):
    """The dense FP64 path, timed over whole steps.  One step = mesh ingest
    (fl_set_mesh), then for each s: FP64 assembly (planned once per step),
    load vector (f = 1),
    Jacobi-PCG to ||r|| <= rtol ||b||, energy-norm error against the
    closed form.  Returns the timing, per-s results, the roofline inputs
    and the handle (holding A for the last s) with the solutions."""
    import torch
    from paper_1708_03912_amd import fraclap as F
    T, B = len(mesh["cells"]), len(mesh["bfacets"])
    opts = F.make_opts(dof_mode=dof_mode)
    h = F.Handle(0)
    bufs, result = {}, {}

    def step():
        h.set_mesh(mesh)
        for s in svals:
            n = h.assemble(s, opts)
            if s not in bufs or bufs[s][0].numel() != n:
                bufs[s] = (torch.empty(n, dtype=torch.float64, device="cuda"),
                           torch.empty(n, dtype=torch.float64, device="cuda"))
            b, u = bufs[s]
            h.load_vector_one(b)
            it, rel, rc = h.solve(b, u, rtol=rtol, maxit=20000)
            e2 = h.energy_error2(ball_fu(s), b, u)
            st = h.stats()
            result[s] = dict(n=n, iters=it, relres=rel, e2=e2, t_asm=st.t_assemble_ms, t_far=st.t_far_ms,
                             t_self=st.t_self_ms, t_touch=st.t_touch_ms, t_scatter=st.t_scatter_ms,
                             t_solve=st.t_solve_ms, t_cgk=st.t_cg_kernels_ms, cg_launched=st.cg_launched,
                             t_plan=st.t_plan_ms,
                             pairs_far=list(st.pairs_far)[:opts.n_classes + 1],
                             far_evals=sum(st.pairs_far[m] * (opts.k_far[m] ** 2) ** 2
                                           for m in range(opts.n_classes + 1)))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    acc = {k: [] for k in ("t_far", "t_asm", "t_solve", "t_cgk", "cg_launched")}
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        for k in acc:
            acc[k].append(sum(result[s][k] for s in svals))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    pairs_per_step = len(svals) * (T * (T + 1) // 2 + T * B)
    mean = {k: sum(v) / len(v) for k, v in acc.items()}
    return dict(h=h, bufs=bufs, result=result, ms_per_step=ms_per_step, pairs_per_step=pairs_per_step,
                mean=mean, T=T, B=B, opts=opts)


def repeatable_assembly(h, mesh, svals, dof_mode):
    """fl_opts.deterministic = 1 on the same workload, after the timed
    steps (not part of `value`): assembly time per s, twice, and whether the
    two matrices agree bit for bit (compared on the device through a 64-bit
    sum of the words of the upper triangle and a second sum weighted by a
    fixed pattern)."""
    import torch
    from paper_1708_03912_amd import fraclap as F
    out = {}
    od = F.make_opts(dof_mode=dof_mode, deterministic=1)
    for s in svals:
        sums, ts = [], []
        for _ in range(2):
            h.set_mesh(mesh)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.assemble(s, od)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
            A = h.matrix_view()
            acc = [0, 0]
            for r0 in range(0, h.n, 4096):
                w = A[r0:r0 + 4096].contiguous().view(torch.int64)
                acc[0] += int(w.sum())
                acc[1] += int((w * (torch.arange(w.shape[1], device=w.device, dtype=torch.int64) % 7 + 1)).sum())
            sums.append(tuple(acc))
        st = h.stats()
        out[str(s)] = {"assemble_ms": [round(t, 2) for t in ts], "device_ms": round(st.t_assemble_ms, 2),
                       "separated_ms": round(st.t_far_ms, 2), "bitwise_equal": sums[0] == sums[1]}
    return out


def matvec_rate(h, reps=10):
    """fl_matvec (symmetric FP64 product from the upper triangle) timed with
    events on the library's stream (torch's current stream)."""
    import torch
    n = h.n
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        h.matvec(x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.matvec(x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tri = n * (n + 1) // 2 * 8 + 2 * n * 8
    return {"ms": round(ms, 4), "GBps": round(tri / (ms * 1e-3) / 1e9, 1),
            "bytes": tri, "full_matrix_equiv_GBps": round((n * n * 8 + 2 * n * 8) / (ms * 1e-3) / 1e9, 1)}


def rooflines(D, svals, cache_resident):
    """Roofline objects of the two kernels that share the step: the
    separated-pair assembly kernels (FP64 VALU) and the CG iteration
    (symmetric product, HBM).  Algorithmic work: 14 FP64 flops per kernel
    evaluation (r^2 from the mapped points 5, the power's multiply 1, four
    FMAs of accumulation 8) plus 2 transcendentals (log, exp) counted apart;
    the product reads the upper triangle of A, n (n + 1) / 2 * 8 bytes, plus
    the CG vectors."""
    res, mean = D["result"], D["mean"]
    nsv = len(svals)
    far_evals = sum(res[s]["far_evals"] for s in svals)
    far_ms = mean["t_far"]
    evals_per_s = far_evals / (far_ms * 1e-3)
    far_tflops = evals_per_s * FLOPS_PER_EVAL / 1e12
    traffic = measured_traffic() if cache_resident is False else {}
    rf_far = {"kernel": "far2_kernel<2,0,0,0,0> + near_kernel<2,0,0,0> (separated element pairs, FP64)",
              "bound": "alu", "achieved": round(far_tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
              "frac": round(far_tflops / FP64_PEAK_TFLOPS, 4),
              "traffic": traffic.get("separated_pairs"),
              "per_launch_ms": round(far_ms / nsv, 4), "evals_per_launch": far_evals // nsv,
              "evals_per_s": round(evals_per_s, 1), "flops_per_eval": FLOPS_PER_EVAL,
              "transcendentals_per_eval": TRANS_PER_EVAL,
              "note": "per launch = one assembly's separated pairs (near + far tiles); achieved = algorithmic "
                      "flops (14 per kernel evaluation) / measured time, transcendentals not counted"}
    # CG iteration: cg_symv + cg_update, device time of the launched
    # iterations (events around each chunk)
    n = res[svals[-1]]["n"]
    launched = mean["cg_launched"]
    cg_ms_it = mean["t_cgk"] / launched if launched else float("nan")
    vec_bytes = 12 * n * 8  # p, z, r, x, b, d and the slots' reads and writes, about
    cg_bytes = n * (n + 1) // 2 * 8 + vec_bytes
    cg_gbps = cg_bytes / (cg_ms_it * 1e-3) / 1e9
    rf_cg = {"kernel": "cg_symv_kernel + cg_update_kernel + cg_scalar_kernel (one Jacobi-PCG iteration, FP64 "
                       "symmetric product from the upper triangle)",
             "bound": "hbm", "achieved": round(cg_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
             "frac": round(cg_gbps / HBM_PEAK_GBPS, 4),
             "traffic": traffic.get("cg_iteration"),
             "per_launch_ms": round(cg_ms_it, 4), "bytes_per_launch": cg_bytes,
             "iterations_launched_per_step": launched}
    if cache_resident:
        rf_cg["note"] = ("A is %.0f MB (upper triangle %.0f MB), below the 256 MB Infinity Cache: "
                         "cache-resident rate" % (n * n * 8 / 1e6, n * (n + 1) / 2 * 8 / 1e6))
    cg_total = mean["t_cgk"]
    if far_ms >= cg_total:
        return rf_far, rf_cg
    return rf_cg, rf_far


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-GPU sharding of the dense path is not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calib(args.copy_calib)
        return
    only = {"batch": (args.only_batch, batch_leg), "surrogate": (args.only_surrogate, surrogate_leg),
            "indicators": (args.only_indicators, indicators_leg), "symmetry": (args.only_symmetry, symmetry_leg),
            "cluster": (args.only_cluster, cluster_leg), "multigrid": (args.only_mg, mg_leg),
            "mixed_assembly": (args.only_mixed_assembly, mixed_assembly_leg)}
    for key, (flag, fn) in only.items():
        if flag:
            import torch
            torch.cuda.set_device(0)
            print(json.dumps({key: fn(args)}), flush=True)
            return
    import torch
    from paper_1708_03912_amd import meshgen as M

    torch.cuda.set_device(0)
    big = args.workload == "disk200k"
    mesh = M.disk_for_cells(200000 if big else 8000, seed=2)
    svals = (0.25, 0.75)
    dof_mode = "interior" if big else "paper"
    rtol = 1e-10 if big else 1e-12
    D = dense_leg(args, mesh, svals, dof_mode, rtol, args.steps, args.warmup)
    T, B, res = D["T"], D["B"], D["result"]
    value = D["pairs_per_step"] / (D["ms_per_step"] * 1e-3)
    n = res[svals[-1]]["n"]
    roof, other = rooflines(D, svals, cache_resident=n * n * 8 < 256e6)
    mv = matvec_rate(D["h"])
    det = repeatable_assembly(D["h"], mesh, svals, dof_mode)
    wl = ("d=2 unit disk, seeded jittered-Delaunay quasi-uniform mesh T=%d B=%d, %s DOFs (n=%d), s in "
          "{0.25,0.75}, f=1: mesh ingest and the s-independent assembly plan once per step, then per s: FP64 "
          "assembly (all element pairs, boundary term) + load vector + Jacobi-PCG to %g + energy error" % (T, B, dof_mode, n, rtol))
    out = {"metric": METRIC, "value": round(value, 1), "unit": "element-pair quadratures/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(D["ms_per_step"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": wl, "cells": T, "bfacets": B,
                      "n_dofs": {str(s): res[s]["n"] for s in svals}, "s": list(svals),
                      "orders": "k_touch=6 theta=(1.5,3,6) k_far=(4,3,2,2)",
                      "pairs_per_step": D["pairs_per_step"]},
           "matvec_GBps": mv["GBps"], "matvec": mv,
           "assemble_ms": round(D["mean"]["t_asm"], 3), "solve_ms": round(D["mean"]["t_solve"], 3),
           "cg_kernels_ms": round(D["mean"]["t_cgk"], 3),
           "cg_iters": {str(s): res[s]["iters"] for s in svals},
           "energy_error": {str(s): math.sqrt(max(res[s]["e2"], 0.0)) for s in svals},
           "phase_ms": {str(s): {k: round(res[s][k], 4) for k in ("t_plan", "t_far", "t_self", "t_touch",
                                                                  "t_scatter", "t_solve", "t_cgk")}
                        for s in svals},
           "roofline": roof, "roofline_other": other, "repeatable_assembly": det}
    print(json.dumps({"progress": "dense step timed", "ms_per_step": out["ms_per_step"]}), file=sys.stderr,
          flush=True)
    if not args.no_mixed:
        out["mixed_surrogate"] = mixed_surrogate_leg(args, mesh, svals, dof_mode, rtol, D)
        print(json.dumps({"progress": "mixed leg done"}), file=sys.stderr, flush=True)
    D["h"].close()
    del D
    torch.cuda.empty_cache()
    if big and not args.no_c2:
        m2 = M.disk_for_cells(8000, seed=2)
        D2 = dense_leg(args, m2, svals, "paper", 1e-12, max(1, min(args.steps, 5)), 1)
        out["disk8k"] = {"ms_per_step": round(D2["ms_per_step"], 3),
                         "value": round(D2["pairs_per_step"] / (D2["ms_per_step"] * 1e-3), 1),
                         "cells": D2["T"], "assemble_ms": round(D2["mean"]["t_asm"], 3),
                         "separated_ms": round(D2["mean"]["t_far"], 3),
                         "solve_ms": round(D2["mean"]["t_solve"], 3),
                         "cg_iters": {str(s): D2["result"][s]["iters"] for s in svals},
                         "matvec": matvec_rate(D2["h"], reps=50),
                         "roofline": rooflines(D2, svals, cache_resident=True)[0]}
        D2["h"].close()
        del D2
    legs = [("batch", not args.no_batch, batch_leg), ("surrogate", not args.no_surrogate, surrogate_leg),
            ("cluster", big and not args.no_cluster, cluster_leg),
            ("multigrid", args.all_legs, mg_leg), ("indicators", args.all_legs, indicators_leg),
            ("symmetry", args.all_legs, symmetry_leg)]
    for key, on, fn in legs:
        if on:
            out[key] = fn(args)
            print(json.dumps({"progress": key + " leg done"}), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_rows(args, mesh, svals, dof_mode, D_pairs=out["config"]["pairs_per_step"],
                                                big=big)
    print(json.dumps(out), flush=True)


def mixed_surrogate_leg(args, mesh, svals, dof_mode, rtol, D):
    """The same workload with FL_MIXED (FP32 separated pairs, FP32 inner CG
    inside FP64 iterative refinement) and the learned surrogate in distance
    classes 0-1 (trained on this mesh's band pairs, exact fallback where not
    certified), one step per s after one untimed one.  Equal error: the gap
    ||u_X - u_64||_A in the FP64 matrix against the FP64 energy error E."""
    import torch
    from paper_1708_03912_amd import fraclap as F
    h64 = D["h"]
    hs = F.Handle(0)
    hs.set_mesh(mesh)
    out = {"surrogate_training": train_surrogate_for(mesh, args, hs)}
    om = F.make_opts(dof_mode=dof_mode, precision="mixed", surrogate=2, sur_tol=args.sur_tol)
    o64 = D["opts"]
    tot_m = tot_64 = 0.0
    for s in svals:
        r = {}
        # the FP64 reference solution of this s (the dense leg keeps only the
        # last s's matrix)
        h64.set_mesh(mesh)
        n = h64.assemble(s, o64)
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        u64 = torch.zeros_like(b)
        h64.load_vector_one(b)
        h64.solve(b, u64, rtol=rtol, maxit=20000)
        st64 = h64.stats()
        r["fp64"] = {"assemble_ms": round(st64.t_assemble_ms, 2), "separated_ms": round(st64.t_far_ms, 2),
                     "solve_ms": round(st64.t_solve_ms, 2), "cg_iters": st64.last_iters}
        um = torch.zeros_like(b)
        for rep in range(2):                      # first pass untimed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hs.set_mesh(mesh)
            nm = hs.assemble(s, om)
            bm = torch.empty(nm, dtype=torch.float64, device="cuda")
            hs.load_vector_one(bm)
            itm, relm, rcm = hs.solve(bm, um, rtol=rtol, maxit=20000)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
        st = hs.stats()
        r["mixed_surrogate"] = {"wall_ms": round(wall, 2), "assemble_ms": round(st.t_assemble_ms, 2),
                                "separated_ms": round(st.t_far_ms, 2), "solve_ms": round(st.t_solve_ms, 2),
                                "inner_iters": itm, "refinements": st.last_outer, "relres": relm,
                                "pairs_surrogate": int(st.pairs_surrogate),
                                "pairs_fallback": int(st.pairs_fallback)}
        E = math.sqrt(max(h64.energy_error2(ball_fu(s), b, u64), 0.0))
        du = um - u64
        y = torch.empty_like(du)
        h64.matvec(du, y)
        gap = math.sqrt(max(float(torch.dot(du, y)), 0.0))
        r["energy_error_fp64"] = E
        r["energy_error_mixed_surrogate"] = math.sqrt(max(h64.energy_error2(ball_fu(s), b, um), 0.0))
        r["gap_over_E"] = gap / E if E > 0 else None
        r["equal_error"] = bool(E > 0 and gap <= 0.1 * E)
        t64 = st64.t_assemble_ms + st64.t_solve_ms
        tm = st.t_assemble_ms + st.t_solve_ms
        r["speedup_assembly"] = round(st64.t_assemble_ms / st.t_assemble_ms, 3)
        r["speedup_solve"] = round(st64.t_solve_ms / st.t_solve_ms, 3)
        r["speedup_assembly_plus_solve"] = round(t64 / tm, 3)
        tot_64 += t64
        tot_m += tm
        out[str(s)] = r
    out["speedup_assembly_plus_solve_both_s"] = round(tot_64 / tot_m, 3)
    hs.close()
    return out


def cpu_baseline_rows(args, mesh, svals, dof_mode, D_pairs, big):
    """The oracle as it stands (plain C, FP64, OpenMP) on the host cores.
    Large workload: a row sample -- the rows of randomly chosen DOFs of A^0.75
    (every element pair touching them, separated, touching and boundary),
    once on all cores and once on one core; rate = element pairs integrated
    per second; the full step would take pairs_per_step / rate (an
    extrapolation, assembly only).  Small workload: one full step (assembly,
    PCG, energy error).  Also the host's dense FP64 matrix-vector rate
    (numpy / OpenBLAS dgemv on a 1 GiB matrix)."""
    import numpy as np
    from oracle import oracle as O
    ncores = len(os.sched_getaffinity(0))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    O.lib()
    ords = O.Orders(k_touch=6, k_touch_bnd=6, theta=[1.5, 3.0, 6.0], k_far=[4, 3, 2, 2], k_far_bnd=[4, 3, 2, 2])
    out = {"unit": "element-pair quadratures/s", "kind": "oracle", "nproc": ncores, "cpu_model": model}
    if not big:
        os.environ["OMP_NUM_THREADS"] = str(ncores)
        t0 = time.perf_counter()
        for s in svals:
            A, dofs, _ = O.assemble(mesh, s, ords)
            b = O.load_vector_one(mesh, dofs)
            u, it, rel = O.pcg(A, b, rtol=1e-12)
            O.energy_error(O.ball_fu(2, s), b, u, A)
        dt = time.perf_counter() - t0
        out.update({"value": round(D_pairs / dt, 1), "cores": ncores, "seconds": round(dt, 2),
                    "sample": "one full step of the same workload (both s: assembly + Jacobi-PCG + energy error)"})
        return out
    nv = len(mesh["verts"])
    cells = np.asarray(mesh["cells"])
    T, B = len(cells), len(mesh["bfacets"])
    s = svals[-1]
    dofs = O.dof_nodes(nv, mesh["bfacets"], s, dof_mode)
    rng = np.random.default_rng(77)

    def run(nrows, threads):
        rows = np.sort(rng.choice(dofs, nrows, replace=False))
        hit = np.isin(cells, rows).any(axis=1)
        nh = int(hit.sum())
        pairs = nh * T - nh * (nh - 1) // 2 + nh * B   # pairs (K, Kt) with K or Kt hit, plus facets
        t0 = time.perf_counter()
        O.assemble_full(mesh, s, ords, rows=rows, compact=True, threads=threads)
        dt = time.perf_counter() - t0
        return {"rows": nrows, "cells_hit": nh, "pairs": pairs, "seconds": round(dt, 2),
                "value": round(pairs / dt, 1), "threads": threads}

    allc = run(args.cpu_rows, ncores)
    one = run(args.cpu_rows_1core, 1)
    os.environ["OMP_NUM_THREADS"] = str(ncores)
    # host dense matvec rate (the CPU library reference for a8)
    M_ = np.random.default_rng(3).standard_normal((8192, 16384))
    x = np.ones(16384)
    M_ @ x
    t0 = time.perf_counter()
    for _ in range(5):
        M_ @ x
    mv_s = (time.perf_counter() - t0) / 5
    out.update({"value": allc["value"], "cores": ncores, "seconds": allc["seconds"] + one["seconds"],
                "sample": "rows of %d (all cores) / %d (one core) random DOFs of A^%g on the same mesh: every "
                          "element pair touching them (separated, touching, boundary); value = pairs integrated "
                          "per second on all cores" % (args.cpu_rows, args.cpu_rows_1core, s),
                "all_cores": allc, "one_core": one,
                "extrapolated_step_assembly_s": round(D_pairs / allc["value"], 1),
                "host_dgemv_GBps": round(M_.nbytes / mv_s / 1e9, 2)})
    return out


def batch_leg(args):
    """Many right-hand sides and several s (unit disk, ~32k triangles, ~16k
    interior DOFs; s = linspace(0.1, 0.9, 8); 64 right-hand sides f =
    sum of 16 cosine modes with N(0,1) coefficients, seeds 1000..1063).
    One step: batched FP64 assembly of the 8 matrices, then the batched
    Jacobi-PCG to ||r|| <= 1e-10 ||b|| for all 512 systems, plain FP64 and
    FP64 refinement around an FP32-arithmetic inner CG on FP32 / bf16 hi+lo /
    bf16 matrix storage.  The gap of each low-precision solution to the FP64
    one is measured in the FP64 energy norm."""
    import numpy as np
    import torch
    from paper_1708_03912_amd import fraclap as F, meshgen as M
    mesh = M.disk_for_cells(args.batch_cells, seed=2)
    T, Bf = len(mesh["cells"]), len(mesh["bfacets"])
    svals = np.linspace(0.1, 0.9, 8)
    ns = len(svals)
    nrhs = 64
    coef = np.stack([np.random.default_rng(1000 + m).standard_normal(16) for m in range(nrhs)])
    h = F.Handle(0)
    h.set_mesh(mesh)
    opts = F.make_opts(dof_mode="interior")
    n = h.assemble_batch(svals, opts)
    tune = {}
    for dt in ("f64", "f32", "bf16x2", "bf16"):
        rows, best = h.autotune(dt)
        tune[dt] = dict(best=rows[best], configs=len(rows))
    b = torch.zeros(nrhs, n, dtype=torch.float64, device="cuda")
    h.load_vector("fourier16", b, coef)
    inners = ("f64", "f32", "bf16x2", "bf16")
    U = {k: torch.zeros(ns, nrhs, n, dtype=torch.float64, device="cuda") for k in inners}
    rtol = 1e-10
    res = {}
    steps = max(1, min(args.steps, 2))
    for rep in range(steps + 1):           # first pass untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.assemble_batch(svals, opts)
        torch.cuda.synchronize()
        t_asm = (time.perf_counter() - t0) * 1e3
        st = h.stats()
        res["assemble_ms"] = t_asm
        res["assemble_device_ms"] = st.t_assemble_ms
        res["far_ms"] = st.t_far_ms
        h.load_vector("fourier16", b, coef)
        for k in inners:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, rel, rc = h.solve_batch(b, U[k], rtol=rtol, maxit=20000, inner=k)
            torch.cuda.synchronize()
            res[k] = dict(ms=(time.perf_counter() - t0) * 1e3, rc=rc, iters=it, rel=rel,
                          outer=h.stats().last_outer)
    # energy-norm gaps to the FP64 solutions (FP64 matrices)
    Y = torch.empty_like(U["f64"])
    h.matmul(U["f64"], Y, "f64")
    norm2 = (U["f64"] * Y).sum(dim=2)
    gaps = {}
    for k in inners[1:]:
        D = U[k] - U["f64"]
        h.matmul(D, Y, "f64")
        g2 = (D * Y).sum(dim=2).clamp(min=0)
        gaps[k] = float((g2 / norm2).sqrt().max())
    pairs = ns * (T * (T + 1) // 2 + T * Bf)
    out = {"workload": f"d=2 unit disk T={T} B={Bf} n={n} (interior DOFs), s=linspace(0.1,0.9,8), "
                       f"64 right-hand sides (16 cosine modes, N(0,1) coefficients), CG to 1e-10",
           "cells": T, "n": n, "ns": ns, "nrhs": nrhs,
           "assemble_ms": round(res["assemble_ms"], 2), "assemble_device_ms": round(res["assemble_device_ms"], 2),
           "far_ms": round(res["far_ms"], 2),
           "assembly_pairs_per_s": round(pairs / (res["assemble_ms"] * 1e-3), 1),
           "gemm_tuned": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v["best"].items()}
                          for k, v in tune.items()}}
    for k in inners:
        r = res[k]
        it = r["iters"]
        out["solve_" + k] = {"ms": round(r["ms"], 2), "converged": bool(np.all(r["rel"] <= rtol)),
                             "iters_mean_per_s": [round(float(x), 1) for x in it.mean(axis=1)],
                             "iters_max": int(it.max()), "refinements": r["outer"],
                             "max_relres": float(r["rel"].max())}
        if k != "f64":
            out["solve_" + k]["energy_gap_rel_max"] = gaps[k]
    h.close()
    return out


def surrogate_leg(args):
    """Learned surrogate on the graded L-shape ((-1,1)^2 minus [0,1)x(-1,0],
    newest-vertex bisection graded 1:64 toward the re-entrant corner and the
    boundary, 37,692 triangles), s = 0.5, f = 1.

    Training set: separated element pairs of this mesh drawn from the two
    closest distance classes (centroid distance < 3 larger longest edges),
    s uniform in [0.05, 0.95]; targets by the library's order-8 rule.  The
    network (9-64-64-21, FP16 matrix cores) is trained on the GPU with Adam
    and certified on held-out pairs of the same kind.  Then four FP64-matrix
    assemblies of A^0.5 are compared: exact orders (4,3,2,2) (the plain
    path), the surrogate in classes 0-1 (exact fallback where not
    certified), the surrogate with FP32 separated pairs (FL_MIXED), and the
    plain order-2 rule in classes 0-1 (and FL_MIXED alone).  Each is solved
    by Jacobi-PCG to 1e-10; energy-norm distances ||u_X - u_ref||_A /
    ||u_ref||_A are measured against a reference assembled with orders 8 / 6
    in classes 0-1."""
    import numpy as np
    import torch
    from paper_1708_03912_amd import fraclap as F, meshgen as M, pairgen as G
    mesh = M.lshape_config3()
    T, Bf = len(mesh["cells"]), len(mesh["bfacets"])
    s = 0.5
    pairs = T * (T + 1) // 2 + T * Bf
    out = {"workload": f"d=2 graded L-shape T={T} B={Bf} (size ratio 1:64), s=0.5, f=1: exact-order FP64 "
                       f"assembly vs learned surrogate (classes 0-1) + Jacobi-PCG to 1e-10",
           "cells": T, "bfacets": Bf, "s": s}
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    h = F.Handle(0)
    Xt, Yt, st_ = G.mesh_band_pairs(mesh, 101, args.sur_train)  # same draws as train_surrogate_for
    Xv, Yv, sv = G.mesh_band_pairs(mesh, 102, 16384)
    ft = torch.zeros(len(st_), 9, dtype=torch.float64, device="cuda")
    tt = torch.zeros(len(st_), 21, dtype=torch.float64, device="cuda")
    fv = torch.zeros(len(sv), 9, dtype=torch.float64, device="cuda")
    tv = torch.zeros(len(sv), 21, dtype=torch.float64, device="cuda")
    Xt, Yt, st_, Xv, Yv, sv = (dev(a) for a in (Xt, Yt, st_, Xv, Yv, sv))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.surrogate_dataset(Xt, Yt, st_, ft, tt, k_exact=8)
    h.surrogate_dataset(Xv, Yv, sv, fv, tv, k_exact=8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.surrogate_init(7)
    h.surrogate_fit_scaling(ft, tt)
    topt = F.default_train_opts(steps=args.sur_steps, batch=1024)
    hist = h.surrogate_train(ft, tt, topt)
    t2 = time.perf_counter()
    bound = h.surrogate_certify(fv, tv)
    pred = torch.zeros_like(tv)
    h.surrogate_predict(fv, pred)
    err = (pred - tv).abs()
    t3 = time.perf_counter()
    # network throughput on the matrix cores: inference over 2^20 feature
    # rows (held-out rows repeated), timed with events on the stream
    big = fv.repeat((1 << 20) // fv.shape[0] + 1, 1)[:1 << 20].contiguous()
    outp = torch.empty(big.shape[0], 21, dtype=torch.float64, device="cuda")
    h.surrogate_predict(big, outp)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        h.surrogate_predict(big, outp)
    ev1.record()
    torch.cuda.synchronize()
    inf_ms = ev0.elapsed_time(ev1) / 5
    flops_pair = 2 * (32 * 64 + 64 * 64 + 64 * 32)  # padded layers, as executed
    out["network_inference"] = {"pairs": int(big.shape[0]), "ms": round(inf_ms, 4),
                                "pairs_per_s": round(big.shape[0] / (inf_ms * 1e-3), 1),
                                "mfma_tflops": round(big.shape[0] * flops_pair / (inf_ms * 1e-3) / 1e12, 2),
                                "peak_tflops": 2500.0, "flops_per_pair": flops_pair,
                                "note": "includes reading 72 B of FP64 features and writing 168 B of FP64 targets per pair"}
    out["train"] = {"pairs": int(ft.shape[0]), "heldout_pairs": int(fv.shape[0]), "steps": topt.steps,
                    "batch": topt.batch, "dataset_ms": round((t1 - t0) * 1e3, 2),
                    "train_ms": round((t2 - t1) * 1e3, 2), "certify_ms": round((t3 - t2) * 1e3, 2),
                    "loss_first": float(np.mean(hist[:20])), "loss_last": float(np.mean(hist[-200:])),
                    "heldout_abs_err": {"median": float(err.median()), "p99": float(torch.quantile(err.flatten()[:1 << 20], 0.99)),
                                        "max": float(err.max())},
                    "heldout_order2_rel_err": {"median": float(tv.abs().median()), "max": float(tv.abs().max())},
                    "bound_at_s": [float(b) for b in bound[:, 2]], "sur_tol": args.sur_tol}
    legs = {"plain": F.make_opts(),
            "surrogate": F.make_opts(surrogate=2, sur_tol=args.sur_tol),
            "mixed": F.make_opts(precision="mixed"),
            "surrogate_mixed": F.make_opts(surrogate=2, sur_tol=args.sur_tol, precision="mixed"),
            "order2_band": F.make_opts(k_far=[2, 2, 2, 2]),
            "reference": F.make_opts(k_far=[8, 6, 2, 2])}
    hs = {"plain": F.Handle(0)}
    for k in legs:
        if k != "plain":
            hs[k] = h if k == "surrogate" else F.Handle(0)
    # the mixed leg needs the same network: copy the parameters over
    blob = h.surrogate_get_params()
    hs["surrogate_mixed"].surrogate_set_params(blob)
    sol = {}
    for k, o in legs.items():
        hk = hs[k]
        hk.set_mesh(mesh)
        for rep in range(2):                     # first assembly untimed
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            n = hk.assemble(s, o)
            torch.cuda.synchronize()
            a_ms = (time.perf_counter() - a0) * 1e3
        stt = hk.stats()
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        u = torch.zeros(n, dtype=torch.float64, device="cuda")
        hk.load_vector_one(b)
        it, rel, rc = hk.solve(b, u, rtol=1e-10, maxit=20000)
        t_solve = hk.stats().t_solve_ms
        sol[k] = (b, u)
        out[k] = {"assemble_ms": round(a_ms, 3), "assemble_device_ms": round(stt.t_assemble_ms, 3),
                  "separated_ms": round(stt.t_far_ms, 3), "pairs_per_s": round(pairs / (a_ms * 1e-3), 1),
                  "pairs_far": [int(x) for x in list(stt.pairs_far)[:4]],
                  "pairs_surrogate": int(stt.pairs_surrogate), "pairs_fallback": int(stt.pairs_fallback),
                  "kernel_evals": int(stt.kernel_evals), "cg_iters": it, "relres": rel,
                  "solve_ms": round(t_solve, 3)}
    # energy-norm distances in the reference matrix (band classes with
    # orders 8 / 6: quadrature error of the band far below every leg's)
    hr = hs["reference"]
    ur = sol["reference"][1]
    y = torch.empty_like(ur)
    hr.matvec(ur, y)
    unorm = math.sqrt(float(torch.dot(ur, y)))
    out["n"] = int(ur.numel())
    out["u_energy_norm"] = unorm
    for k in legs:
        if k == "reference":
            continue
        du = sol[k][1] - ur
        hr.matvec(du, y)
        out[k]["energy_gap_to_reference_rel"] = math.sqrt(max(float(torch.dot(du, y)), 0.0)) / unorm
        out[k]["speedup_vs_plain"] = round(out["plain"]["assemble_ms"] / out[k]["assemble_ms"], 3)
    for hk in set(hs.values()):
        hk.close()
    return out


def train_surrogate_for(mesh, args, h):
    """Train h's network on band pairs of mesh (library dataset, library
    kernels) and certify it on held-out pairs; returns timings."""
    import numpy as np
    import torch
    from paper_1708_03912_amd import fraclap as F, pairgen as G
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    Xt, Yt, st_ = (dev(a) for a in G.mesh_band_pairs(mesh, 101, args.sur_train))
    Xv, Yv, sv = (dev(a) for a in G.mesh_band_pairs(mesh, 102, 16384))
    ft = torch.zeros(Xt.shape[0], 9, dtype=torch.float64, device="cuda")
    tt = torch.zeros(Xt.shape[0], 21, dtype=torch.float64, device="cuda")
    fv = torch.zeros(Xv.shape[0], 9, dtype=torch.float64, device="cuda")
    tv = torch.zeros(Xv.shape[0], 21, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.surrogate_dataset(Xt, Yt, st_, ft, tt, k_exact=8)
    h.surrogate_dataset(Xv, Yv, sv, fv, tv, k_exact=8)
    h.surrogate_init(7)
    h.surrogate_fit_scaling(ft, tt)
    hist = h.surrogate_train(ft, tt, F.default_train_opts(steps=args.sur_steps, batch=1024))
    bound = h.surrogate_certify(fv, tv)
    torch.cuda.synchronize()
    return {"train_total_ms": round((time.perf_counter() - t0) * 1e3, 1), "loss_last": float(np.mean(hist[-200:])),
            "bound_at_s": {"0.25": [float(b) for b in bound[:, 1]], "0.75": [float(b) for b in bound[:, 3]]}}


def mixed_assembly_leg(args):
    """FL_MIXED assembly (FP32 separated pairs) of the benchmark disk,
    interior DOFs, s in {0.25, 0.75}, once each (after one untimed
    assembly): the workload of the FP32 counter summary."""
    from paper_1708_03912_amd import fraclap as F, meshgen as M
    mesh = M.disk_for_cells(200000, seed=2)
    h = F.Handle(0)
    h.set_mesh(mesh)
    om = F.make_opts(dof_mode="interior", precision="mixed")
    h.assemble(0.75, om)
    out = {"workload": "unit disk T=%d, interior DOFs, FL_MIXED assembly" % len(mesh["cells"])}
    for s in (0.25, 0.75):
        n = h.assemble(s, om)
        st = h.stats()
        out[str(s)] = {"n": n, "assemble_ms": round(st.t_assemble_ms, 3), "separated_ms": round(st.t_far_ms, 3)}
    h.close()
    return out


def mg_leg(args):
    """Nested uniform refinements of a disk mesh (~500 triangles, 3 and 4
    levels: ~8k and ~32k triangles, s in {0.25, 0.75}; 5 levels: ~128k
    triangles, s = 0.75), f = 1: Jacobi-PCG against CG preconditioned by one
    multigrid V(2,2) cycle (Sec. 5), both to 1e-10; iterations, solve times,
    the hierarchy's setup time and the energy-norm distance of the two
    solutions.  Then the same multigrid CG with the cluster approximation
    (Sec. 6: m = 6, eta = 2, leaves of 32) as the operator of CG and of the
    finest level of the cycle."""
    import torch
    from paper_1708_03912_amd import fraclap as F, meshgen as M
    base = M.disk_for_cells(500, seed=2)
    out = {"workload": "unit disk, ~500-triangle base mesh refined uniformly (nested), f=1, CG to 1e-10: "
                       "Jacobi-PCG vs multigrid V(2,2)-preconditioned CG"}
    for levels, svals in ((3, (0.25, 0.75)), (4, (0.25, 0.75)), (5, (0.75,))):
        meshes, parents = M.hierarchy(base, levels)
        nv = [len(m["verts"]) for m in meshes]
        for s in svals:
            h = F.Handle(0)
            h.set_mesh(meshes[-1])
            n = h.assemble(s)
            b = torch.empty(n, dtype=torch.float64, device="cuda")
            h.load_vector_one(b)
            uj, um = torch.zeros_like(b), torch.zeros_like(b)
            h.solve(b, uj, rtol=1e-10, maxit=20000)  # warm-up (workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            itj, relj, _ = h.solve(b, uj, rtol=1e-10, maxit=20000)
            torch.cuda.synchronize()
            tj = (time.perf_counter() - t0) * 1e3
            t0 = time.perf_counter()
            h.mg_setup(nv, parents)
            torch.cuda.synchronize()
            tset = (time.perf_counter() - t0) * 1e3
            h.solve_mg(b, um, rtol=1e-10)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            itm, relm, _ = h.solve_mg(b, um, rtol=1e-10)
            torch.cuda.synchronize()
            tm = (time.perf_counter() - t0) * 1e3
            du = um - uj
            y = torch.empty_like(du)
            h.matvec(du, y)
            gap = float(torch.dot(du, y)) ** 0.5
            h.matvec(uj, y)
            unorm = float(torch.dot(uj, y)) ** 0.5
            # the cluster approximation as the fine operator
            t0 = time.perf_counter()
            h.cluster_build(m=6, eta=2.0, leaf=32)
            torch.cuda.synchronize()
            tcb = (time.perf_counter() - t0) * 1e3
            uh = torch.zeros_like(b)
            h.solve_cluster_mg(b, uh, rtol=1e-10)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ith, relh, _ = h.solve_cluster_mg(b, uh, rtol=1e-10)
            torch.cuda.synchronize()
            th = (time.perf_counter() - t0) * 1e3
            du = uh - um
            h.matvec(du, y)
            gaph = float(torch.dot(du, y)) ** 0.5
            out[f"levels{levels}_s{s}"] = {"cells": len(meshes[-1]["cells"]), "n": n, "jacobi_iters": itj,
                                           "jacobi_ms": round(tj, 3), "mg_setup_ms": round(tset, 3),
                                           "mg_iters": itm, "mg_ms": round(tm, 3),
                                           "speedup": round(tj / tm, 3) if tm > 0 else None,
                                           "relres": [relj, relm], "gap_rel": gap / unorm if unorm > 0 else None,
                                           "cluster_build_ms": round(tcb, 3), "cluster_mg_iters": ith,
                                           "cluster_mg_ms": round(th, 3), "cluster_mg_relres": relh,
                                           "cluster_gap_rel": gaph / unorm if unorm > 0 else None}
            h.close()
    return out


def indicators_leg(args):
    """A posteriori path (Sec. 4): the strong form of the discrete solution
    at the 4 collapsed Gauss points of every cell (edge rules 2 / 12
    points) and the BR indicators, on the disk mesh of the headline
    (~8k triangles), s in {0.25, 0.75}, timed against the assembly of the
    same matrix; then the adaptive loops of Sec. 7 (d = 1: 32 steps from
    8 cells; d = 2: 8 steps from a 200-triangle disk) with the time of each
    phase and the fitted energy-error rate."""
    import numpy as np
    import torch
    from paper_1708_03912_amd import adaptive as AD, fraclap as F, meshgen as M
    from math import gamma, pi
    mesh = M.disk_for_cells(args.cells, seed=2)
    T = len(mesh["cells"])
    out = {"workload": f"unit disk, {T} triangles, f=1, u_h = the FP64 solution; strong form at 4 points "
                       f"per cell (edge rules 2 far / 12 touching) + indicators"}
    for s in (0.25, 0.75):
        h = F.Handle(0)
        h.set_mesh(mesh)
        n = h.assemble(s)                  # first call: buffers and plan
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = h.assemble(s)
        torch.cuda.synchronize()
        t_asm = (time.perf_counter() - t0) * 1e3
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        h.load_vector_one(b)
        u = torch.zeros_like(b)
        h.solve(b, u, rtol=1e-10)
        Lu = torch.empty(T * 4, dtype=torch.float64, device="cuda")
        ec = torch.empty(T, dtype=torch.float64, device="cuda")
        en = torch.empty(len(mesh["verts"]), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.strong_form(s, u, Lu)            # first call: geometry plan
        torch.cuda.synchronize()
        t_first = (time.perf_counter() - t0) * 1e3
        reps = max(3, args.steps)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            h.strong_form(s, u, Lu)
            h.indicators(s, Lu, ec, en)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        nt = T * 4
        edges = (3 * T + len(mesh["bfacets"])) // 2
        inter = nt * edges * 2
        out[f"s{s}"] = {"n": n, "targets": nt, "edge_sources": edges * 2, "ms": round(ms, 4),
                        "first_call_ms": round(t_first, 3), "assembly_ms": round(t_asm, 3),
                        "far_interactions_per_s": inter / (ms * 1e-3),
                        "estimator": float(ec.sum().item())}
        h.close()
    # adaptive loops (Sec. 7, f = 1 on the unit ball)
    def ball_fu(d, s):
        c = 2.0 ** (-2 * s) * gamma(d / 2) / (gamma(d / 2 + s) * gamma(1 + s))
        if d == 1:
            return c * gamma(0.5) * gamma(s + 1) / gamma(s + 1.5)
        return c * pi / (s + 1.0)
    o = F.make_opts(k_touch=8, k_touch_bnd=8, k_far=[6, 5, 4, 3], k_far_bnd=[6, 5, 4, 3])
    loops = {}
    for name, m0, s, nst, proj in (("1d_s0.25", M.interval(8), 0.25, 32, None),
                                   ("1d_s0.75", M.interval(8), 0.75, 32, None),
                                   ("2d_s0.75", M.disk_for_cells(200, seed=2), 0.75, 8, M.project_disk)):
        t0 = time.perf_counter()
        steps, _ = AD.adaptive_loop(m0, s, nst, opts=o if m0["dim"] == 1 else None, fu=ball_fu(m0["dim"], s),
                                    rtol=1e-12, project=proj)
        wall = time.perf_counter() - t0
        nn = np.array([st.n for st in steps], dtype=float)
        ee = np.sqrt(np.maximum([st.e2 for st in steps], 1e-300))
        k = min(8, len(steps))
        loops[name] = {"steps": len(steps), "n_first": int(nn[0]), "n_last": int(nn[-1]),
                       "energy_err_last": float(ee[-1]),
                       "rate_last8": float(np.polyfit(np.log(nn[-k:]), np.log(ee[-k:]), 1)[0]),
                       "t_assemble_s": round(sum(st.t_assemble for st in steps), 4),
                       "t_solve_s": round(sum(st.t_solve for st in steps), 4),
                       "t_indicators_s": round(sum(st.t_indicators for st in steps), 4),
                       "wall_s": round(wall, 3)}
    out["adaptive"] = loops
    # the all-pairs part by the cluster method (m = 6, eta = 2, leaves of 16
    # cells) against the direct sum, growing meshes, s = 0.75
    cl = {}
    for cells in (8000, 32000, 128000):
        mesh = M.disk_for_cells(cells, seed=2)
        T = len(mesh["cells"])
        h = F.Handle(0)
        h.set_mesh(mesh)
        n = h.assemble(0.75)
        u = torch.tensor(np.random.default_rng(3).standard_normal(n), device="cuda")
        Ld, Lc = torch.empty(T * 4, dtype=torch.float64, device="cuda"), torch.empty(T * 4, dtype=torch.float64,
                                                                                     device="cuda")
        h.strong_form(0.75, u, Ld)
        h.strong_form_cluster(0.75, u, Lc, m=6, eta=2.0, leaf=16)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        h.strong_form(0.75, u, Ld)
        ev[1].record()
        h.strong_form_cluster(0.75, u, Lc, m=6, eta=2.0, leaf=16)
        ev[2].record()
        torch.cuda.synchronize()
        cl[f"cells{T}"] = {"direct_ms": round(ev[0].elapsed_time(ev[1]), 3),
                           "cluster_ms": round(ev[1].elapsed_time(ev[2]), 3),
                           "rel_gap": float((Lc - Ld).abs().max() / Ld.abs().max())}
        h.close()
    out["cluster_strong_form"] = cl
    return out


def cluster_leg(args):
    """Cluster method (Sec. 6) assembled from the mesh alone
    (fl_cluster_assemble: near field from the pair kernels, far field by
    Chebyshev interpolation, no dense matrix) on unit disks, s = 0.75,
    f = 1, interior DOFs, eta = 2, leaves of 32 DOFs, m = 6 and 8: assembly
    and Jacobi-PCG (to 1e-10) times, device bytes, product time and energy
    error against the closed form; m = 6 also with the blocks kept in FP32
    (precision FL_MIXED: assembled in FP64, rounded once, products and sums
    in FP64).  On the disks of ~3.2e4 and ~2e5
    triangles the dense FP64 path runs beside it; the ~4e5-triangle disk
    (n ~ 2e5) has a dense matrix larger than the device memory."""
    import torch
    from paper_1708_03912_amd import fraclap as F, meshgen as M
    s = 0.75
    fu = ball_fu(s)
    out = {"workload": "unit disk, s=0.75, f=1, interior DOFs; cluster method assembled from the mesh, eta=2, "
                       "leaf 32, m in {6, 8}, m = 6 also with FP32 blocks; dense FP64 path beside it where its matrix fits",
           "device_bytes": torch.cuda.mem_get_info()[1]}
    o = F.make_opts(dof_mode="interior")

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    for cells in (32000, 200000, 400000):
        mesh = M.disk_for_cells(cells, seed=2)
        r = {}
        h = F.Handle(0)
        h.set_mesh(mesh)
        n = None
        if cells <= 200000:
            n, t_asm = timed(lambda: h.assemble(s, o))
            b = torch.empty(n, dtype=torch.float64, device="cuda")
            h.load_vector_one(b)
            u = torch.zeros_like(b)
            (it, rel, rc), t_sol = timed(lambda: h.solve(b, u, rtol=1e-10, maxit=20000))
            x = torch.ones(n, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            h.matvec(x, y)
            _, t_mv = timed(lambda: [h.matvec(x, y) for _ in range(10)])
            r["dense"] = {"assemble_ms": round(t_asm, 2), "cg_iters": it, "cg_ms": round(t_sol, 2),
                          "matvec_ms": round(t_mv / 10, 4), "bytes": n * h.ld * 8,
                          "energy_error": math.sqrt(max(fu - float(torch.dot(b, u)), 0.0))}
            del b, u, x, y
        om = F.make_opts(dof_mode="interior", precision="mixed")
        for m, oc, name in ((6, o, "cluster_m6"), (8, o, "cluster_m8"), (6, om, "cluster_m6_fp32")):
            n2, t_asm = timed(lambda: h.cluster_assemble(s, oc, m=m, eta=2.0, leaf=32))
            n = n2
            info = h.cluster_info()
            st = h.stats()
            b = torch.empty(n, dtype=torch.float64, device="cuda")
            h.load_vector_one(b)
            u = torch.zeros_like(b)
            (it, rel, rc), t_sol = timed(lambda: h.solve_cluster(b, u, rtol=1e-10, maxit=20000))
            x = torch.ones(n, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            h.cluster_matvec(x, y)
            _, t_mv = timed(lambda: [h.cluster_matvec(x, y) for _ in range(10)])
            r[name] = {
                "assemble_ms": round(t_asm, 2), "near_field_kernels_ms": round(st.t_assemble_ms, 2),
                "cg_iters": it, "cg_ms": round(t_sol, 2), "matvec_ms": round(t_mv / 10, 4),
                "bytes": info["bytes"], "near_entries": info["near_entries"], "far_pairs": info["far_pairs"],
                "energy_error": math.sqrt(max(fu - float(torch.dot(b, u)), 0.0))}
            del b, u, x, y
        r["n"] = n
        r["cells"] = len(mesh["cells"])
        r["dense_fp64_bytes"] = n * n * 8
        out["cells%d" % len(mesh["cells"])] = r
        h.close()
        torch.cuda.empty_cache()
        print(json.dumps({"progress": "cluster leg", "cells": len(mesh["cells"])}), file=sys.stderr, flush=True)
    return out


def symmetry_leg(args):
    """Symmetry reduction (Sec. 7): a unit disk invariant under rotations by
    2 pi / 8 (~32k triangles), s = 0.75, f = 1: the full system against the
    reduced one (sector against all images): DOFs, separated pairs,
    assembly and CG times, and the largest gap between the two solutions
    at the representatives."""
    import numpy as np
    import torch
    from paper_1708_03912_amd import fraclap as F, meshgen as M
    K = 8
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.0152, K, seed=2)
    out = {"workload": f"unit disk, {len(mesh['cells'])} triangles invariant under rotation by 2pi/{K} "
                       f"(sector of {Tw}), s=0.75, f=1, CG to 1e-10"}
    res = {}
    for name, sym in (("full", False), ("reduced", True)):
        h = F.Handle(0)
        h.set_mesh(mesh)
        if sym:
            h.set_symmetry(K, Tw, vfold, pre, rot)
        n = h.assemble(0.75)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = h.assemble(0.75)
        torch.cuda.synchronize()
        t_asm = (time.perf_counter() - t0) * 1e3
        st = h.stats()
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        h.load_vector_one(b)
        u = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, _, _ = h.solve(b, u, rtol=1e-10)
        torch.cuda.synchronize()
        t_cg = (time.perf_counter() - t0) * 1e3
        res[name] = (h.dofs(), u.cpu().numpy())
        out[name] = {"n": n, "separated_pairs": int(sum(st.pairs_far)), "assembly_ms": round(t_asm, 2),
                     "cg_iters": it, "cg_ms": round(t_cg, 2)}
        h.close()
    dof_f, uf = res["full"]
    dof_r, ur = res["reduced"]
    pos = np.searchsorted(dof_f, dof_r)
    out["max_gap_rel"] = float(np.abs(ur - uf[pos]).max() / np.abs(uf).max())
    out["assembly_speedup"] = round(out["full"]["assembly_ms"] / out["reduced"]["assembly_ms"], 2)
    return out


if __name__ == "__main__":
    main()
