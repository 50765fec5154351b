#!/usr/bin/env python
"""Benchmark of the block-preconditioned FGMRES solve on one MI355X.

Workload (default): the 80^3 Q1 hex mesh with three orthogonal full
fractures, 30% slip faces, one right-hand side (n_u 1,654,104, n_t 57,600,
n_p 19,200).  One step is one pass of the whole path on device-resident
inputs: preconditioner construction (H~, S1 = A + C1 H~^-1 C2, pressure
block inverse, smoothed-aggregation hierarchy with its Galerkin products)
followed by the FGMRES(50) solve to a true relative residual of 1e-8.

Printed: one JSON line.  ``value`` is the FGMRES time-to-1e-8 in seconds of
the plain FP64 path (mean over the timed steps); the FP32-preconditioned
solve time and its speedup, the V-cycle bandwidth, the roofline of the
dominant kernel (level-0 residual SpMV of the V-cycle, timed with HIP events
inside the timed region), the production forms on their own workloads
(``forms``) and the CPU oracle baseline are added as objects.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = ("FGMRES time-to-1e-8 residual (s), FP32-precond vs FP64; "
          "V-cycle HBM GB/s")
WORKLOADS = {
    "c1": "10^3 Q1 hex, one full fracture plane (100 faces), all stick",
    "c2": "80^3 Q1 hex, three orthogonal full fractures (19,200 faces), "
          "Bernoulli(0.3) slip, single right-hand side",
    "c3": "128x128x64 Q1 hex, 12 random fractures, layered modulus",
    "c4": "64^3 Q1 hex, 6 random fractures",
    "c5": "48^3 Q1 hex, 4 full x-normal fractures (9,216 faces)",
}


def spmv_bytes(nnz, nrows, ncols, sv=8, si=4, nv=1, extra_vec=0):
    """Algorithmic bytes of y = M x: values + column indices of the true
    nonzeros, row pointers, one read of x and one write of y per column,
    plus ``extra_vec`` further row-length vector streams per column."""
    return (nnz * (sv + si) + 4 * (nrows + 1)
            + nv * (nrows + ncols + extra_vec * nrows) * sv)


def vcycle_bytes(levels, nv=1, sv=8):
    """Algorithmic bytes of one V-cycle: per level the four fused smoother /
    residual products with A_l (their vector streams beyond one read and
    one write: 3 + 1 + 4 + 3), restriction, prolongation; the coarsest level
    reads its dense inverse once."""
    total = 0
    for i, d in enumerate(levels):
        n = d["n_nodes"] * d["block"]
        if d["n_agg"] == 0:                       # coarsest
            total += n * n * 8 + 2 * nv * n * sv
            break
        nxt = levels[i + 1]
        nc = nxt["n_nodes"] * nxt["block"]
        nnzP = d["p_nnzb"] * d["block"] * nxt["block"]
        total += 4 * spmv_bytes(d["nnz_scalar"], n, n, sv, nv=nv)
        total += nv * 11 * n * sv
        total += spmv_bytes(nnzP, nc, n, sv, nv=nv)          # R = P^T
        total += spmv_bytes(nnzP, n, nc, sv, nv=nv)          # P
    return total


COUNTERS = os.path.join(ROOT, "profiles",
                        "level0_residual_spmv_c2_fp64_counters.json")


def counter_traffic():
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, each scaled by what the counter
    reads for a plain 2 GiB copy; None once the kernel source differs from
    the one the counters were taken on."""
    import hashlib
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
        with open(os.path.join(ROOT, c["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if sha != c["source_sha256"]:
        return None
    return 1024.0 * (c["fetch_kib_per_launch"] * c["fetch_scale"]
                     + c["write_kib_per_launch"] * c["write_scale"])


def device_blocks(torch, s):
    out = {}
    for k, M in s.blocks().items():
        out[k] = (torch.tensor(M.indptr.astype(np.int64), device="cuda"),
                  torch.tensor(M.indices.astype(np.int32), device="cuda"),
                  torch.tensor(M.data.astype(np.float64), device="cuda"))
    return out


def cpu_baseline(s, gpu_iters, sample_its, v_gpu=None):
    """The CPU oracle on the same workload, one thread: preconditioner setup
    (untimed for the value), then ``sample_its`` FGMRES iterations, scaled to
    the GPU's iteration count.  With ``v_gpu`` (the GPU's M^-1 b) the oracle's
    application to the same b is compared with it."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pc = oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p,
                                 coords=s.coords)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, info = oracle.fgmres(pc.matvec, pc.apply, s.b, rtol=1e-8,
                                maxit=sample_its)
        t_its = time.perf_counter() - t0
        apply_diff = None
        if v_gpu is not None:
            vo = pc.apply(s.b)
            apply_diff = float(np.linalg.norm(v_gpu - vo) / np.linalg.norm(vo))
    per_it = t_its / max(info.iterations, 1)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": per_it * gpu_iters, "unit": "s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{info.iterations} FGMRES iterations of the NumPy/SciPy "
                       f"FP64 oracle on this workload after its setup "
                       f"({t_setup:.1f} s, not in value), scaled to the GPU "
                       f"iteration count {gpu_iters}"),
            "per_iteration_s": per_it, "setup_s": t_setup,
            "gpu_vs_oracle_apply_rel_diff": apply_diff,
            "cpu_model": cpu, "host": platform.node()}


def stream_triad(torch, sol, n=1 << 29, reps=10):
    """a = b + s c over three n-double arrays (4 GiB each by default) with the
    library's triad kernel; HIP events on the current stream, best of
    ``reps`` after a warm-up, 24 bytes per element."""
    b = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    sol.stream_triad(b, c, 3.0, a)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sol.stream_triad(b, c, 3.0, a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    ok = bool((a == 7.0).all())
    del a, b, c
    torch.cuda.empty_cache()
    gbs = 24.0 * n / best / 1e9
    return {"GBps": gbs, "frac": gbs / HBM_PEAK_GBS, "seconds": best,
            "array_bytes": 8 * n, "check": ok}


def _timed(torch, fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def forms(torch, s2, blocks2, coords2, b2, fp64_solve_s):
    """The production forms on their own workloads, each after one untimed
    warm-up call: t-p-u and M2* on the 80^3 system, the 32-right-hand-side batch
    (64^3, FP32 preconditioner) against the same columns solved one by one,
    the FP32 hierarchy on the 128x128x64 layered system, and the adjoint
    solve with the transmissibility gradient on the 48^3 system."""
    import fracgen
    from fracgen.configs import observations, rhs_batch
    from paper_2112_12397_amd import Solver, solver_from_system
    out = {}
    # t-p-u (Alg 3.2): one AMG call per application
    sol = Solver(blocks2, s2.n_u, s2.n_t, s2.n_p, coords=coords2, mode="tpu")
    x = torch.empty_like(b2)
    sol.solve(b2, out=x)
    t, (_, inf) = _timed(torch, lambda: sol.solve(b2, out=x), 2)
    out["tpu_80cube"] = {"solve_s": t, "iterations": inf["iterations"],
                         "true_rel_residual": inf["true_rel_residual"],
                         "speedup_vs_tup": fp64_solve_s / t}
    del sol
    # M2* = D2^-1 L2^-1 (remark after Prop 3.2): one AMG call, no U2 factor
    sol = Solver(blocks2, s2.n_u, s2.n_t, s2.n_p, coords=coords2,
                 mode="tup_star")
    sol.solve(b2, out=x)
    t, (_, inf) = _timed(torch, lambda: sol.solve(b2, out=x), 2)
    out["tup_star_80cube"] = {"solve_s": t, "iterations": inf["iterations"],
                              "true_rel_residual": inf["true_rel_residual"],
                              "speedup_vs_tup": fp64_solve_s / t}
    del sol
    # batch of 32 right-hand sides
    s4 = fracgen.make_config("c4")
    sol = solver_from_system(s4, precision="fp32")
    B = torch.tensor(np.ascontiguousarray(rhs_batch(s4, k=32).T), device="cuda")
    X = torch.empty_like(B)
    sol.solve_batch(B, out=X)
    tb, (_, infs, st) = _timed(torch, lambda: sol.solve_batch(B, out=X))
    xs = torch.empty_like(B[0])
    sol.solve(B[0].contiguous(), out=xs)

    def seq():
        its = []
        for c in range(32):
            _, i1 = sol.solve(B[c].contiguous(), out=xs)
            its.append(i1["iterations"])
        return its
    tq, its1 = _timed(torch, seq)
    out["batch32_64cube_fp32prec"] = {
        "workload": "64^3 Q1 hex, 6 random fractures, 32 RHS (norms 1e-2..1e2)",
        "batch_s": tb, "per_rhs_s": tb / 32, "sequential_s": tq,
        "speedup_vs_sequential": tq / tb, "status": st,
        "iterations_max": max(i["iterations"] for i in infs),
        "iterations_mean": float(np.mean([i["iterations"] for i in infs])),
        "sequential_iterations_mean": float(np.mean(its1)),
        "worst_true_rel_residual": max(i["true_rel_residual"] for i in infs),
        "n_u": s4.n_u, "n_t": s4.n_t, "n_p": s4.n_p}
    del sol, s4
    # FP32 hierarchy on the layered 128x128x64 system
    s3 = fracgen.make_config("c3")
    b3 = torch.tensor(s3.b, device="cuda")
    res = {"workload": "128x128x64 Q1 hex, 12 random fractures, layered E",
           "n_u": s3.n_u, "n_t": s3.n_t, "n_p": s3.n_p}
    xx = {}
    for prec in ("fp64", "fp32"):
        sol = solver_from_system(s3, precision=prec)
        x3 = torch.empty_like(b3)
        sol.solve(b3, out=x3)
        t, (_, inf) = _timed(torch, lambda: sol.solve(b3, out=x3), 2)
        res[prec] = {"solve_s": t, "iterations": inf["iterations"],
                     "true_rel_residual": inf["true_rel_residual"]}
        xx[prec] = x3.clone()
        del sol
    res["fp32_speedup"] = res["fp64"]["solve_s"] / res["fp32"]["solve_s"]
    res["rel_diff_fp32_vs_fp64"] = float(
        (xx["fp32"] - xx["fp64"]).norm() / xx["fp64"].norm())
    out["precision_128x128x64"] = res
    del s3, b3, xx
    # adjoint solve and transmissibility gradient
    s5 = fracgen.make_config("c5")
    _, p_obs = observations(s5)
    sol = solver_from_system(s5)
    b5 = torch.tensor(s5.b, device="cuda")
    x5, _ = sol.solve(b5)
    off = s5.n_u + s5.n_t
    g = torch.zeros_like(b5)
    g[off:] = x5[off:] - torch.tensor(p_obs, device="cuda")
    sol.solve_T(g, rtol=1e-11)
    tf, (_, inff) = _timed(torch, lambda: sol.solve(b5, rtol=1e-11))
    ta, (lam, infa) = _timed(torch, lambda: sol.solve_T(g, rtol=1e-11))
    pairs = torch.tensor(s5.flow_pairs)
    ndir = torch.tensor(s5.flow_ndir)
    ups = torch.tensor(s5.upsilon)
    tg, _ = _timed(torch, lambda: sol.grad_log_trans(pairs, ndir, ups,
                                                     lam[off:], x5[off:]))
    out["adjoint_48cube"] = {
        "workload": "48^3 Q1 hex, 4 full fractures (9,216 faces), rtol 1e-11",
        "forward_s": tf, "forward_iterations": inff["iterations"],
        "adjoint_s": ta, "adjoint_iterations": infa["iterations"],
        "gradient_s": tg}
    del sol, s5
    # open faces (Q2 != 0): sequential AMG calls (t-u-p) or S~ (t-p-u)
    so = fracgen.make_config("c2o")
    bo = torch.tensor(so.b, device="cuda")
    res = {"workload": "80^3 Q1 hex, three intersecting fractures, 30% slip, "
                       "10% open faces (Q2 != 0)",
           "faces_stick_slip_open": [int(c) for c in
                                     np.bincount(so.face_state, minlength=3)],
           "q2_nnz": int(so.Q2.nnz)}
    for mode in ("tup", "tpu", "tup_star"):
        t0 = time.perf_counter()
        sol = solver_from_system(so, mode=mode)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        xo = torch.empty_like(bo)
        sol.solve(bo, out=xo)
        t, (_, inf) = _timed(torch, lambda: sol.solve(bo, out=xo), 2)
        res[mode] = {"solve_s": t, "iterations": inf["iterations"],
                     "true_rel_residual": inf["true_rel_residual"],
                     "setup_s_incl_upload": ts}
        del sol
    out["open_faces_80cube"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-sample-its", type=int, default=2)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batch / precision / adjoint / t-p-u runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on exactly one GPU; multi-GPU runs "
              "are not supported (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import fracgen
    from paper_2112_12397_amd import Solver

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    s = fracgen.make_config(args.config)
    blocks = device_blocks(torch, s)
    coords = torch.tensor(s.coords, device="cuda")
    b = torch.tensor(s.b, device="cuda")
    x = torch.empty_like(b)

    sol = Solver(blocks, s.n_u, s.n_t, s.n_p, coords=coords)
    for _ in range(args.warmup):
        sol.setup(blocks, coords)
        sol.solve(b, out=x)
    torch.cuda.synchronize()

    sol.kernel_timer(enable=True, reset=True)
    t_setup, t_solve, infos = 0.0, 0.0, []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        sol.setup(blocks, coords)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = sol.solve(b, out=x)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_setup += t1 - t0
        t_solve += t2 - t1
        infos.append(info)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t_all
    launches, kernel_ms = sol.kernel_timer(enable=False, reset=True)
    K = args.steps
    iters = infos[-1]["iterations"]
    for inf in infos:
        if not inf["converged"] or inf["true_rel_residual"] > 1e-8:
            raise SystemExit(f"solve did not converge: {inf}")

    levels = [sol.level_info(l) for l in range(sol.num_levels())]
    setup_parts = sol.setup_times()

    # numeric re-setup (next Newton iteration, same patterns): reuses the
    # aggregates, tentative prolongators and apply layouts
    t_upd = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.update_values(blocks)
        torch.cuda.synchronize()
        t_upd.append(time.perf_counter() - t0)
    resetup = {"update_values_s": min(t_upd), "setup_s": t_setup / K,
               "hierarchy_reused": sol.hierarchy_reused(),
               "parts_s": sol.setup_times()}

    # dominant kernel: level-0 residual SpMV of the V-cycle (one column)
    d0 = levels[0]
    nv = 1
    k_bytes = spmv_bytes(d0["nnz_scalar"], s.n_u, s.n_u, nv=nv, extra_vec=1)
    k_avg_s = kernel_ms / max(launches, 1) / 1e3
    achieved = k_bytes / k_avg_s / 1e9

    # V-cycle bandwidth (one FP64 column), HIP events on the library stream
    vb = torch.randn(s.n_u, dtype=torch.float64, device="cuda")
    vx = torch.empty_like(vb)
    for _ in range(3):
        sol.vcycle(vb, out=vx)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
        enable_timing=True)
    nrep = 20
    ev0.record()
    for _ in range(nrep):
        sol.vcycle(vb, out=vx)
    ev1.record()
    torch.cuda.synchronize()
    vc_s = ev0.elapsed_time(ev1) / nrep / 1e3
    vc_bytes = vcycle_bytes(levels)

    # pressure-block solve alone (one per application in t-u-p with Q2 = 0)
    wp = torch.randn(s.n_p, dtype=torch.float64, device="cuda")
    vp = torch.empty_like(wp)
    for _ in range(3):
        sol.psolve(wp, out=vp)
    ev0.record()
    for _ in range(nrep):
        sol.psolve(wp, out=vp)
    ev1.record()
    torch.cuda.synchronize()
    ps_s = ev0.elapsed_time(ev1) / nrep / 1e3
    del wp, vp

    # measured STREAM triad (three 4 GiB arrays) as the achievable HBM rate
    triad = stream_triad(torch, sol)

    out = {
        "metric": METRIC,
        "value": t_solve / K,
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_all / K,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}",
                   "n_u": s.n_u, "n_t": s.n_t, "n_p": s.n_p, "N": s.N,
                   "mode": "t-u-p", "restart": 50, "rtol": 1e-8,
                   "seed": s.seed},
        "iterations": iters,
        "true_rel_residual": infos[-1]["true_rel_residual"],
        "setup_s": t_setup / K,
        "setup_parts_s": setup_parts,
        "resetup": resetup,
        "amg_levels": [{"dofs": d["n_dofs"], "nnz": d["nnz_scalar"],
                        "layout_A_P_R": d["layout"],
                        "tuned_us_A_P_R": [round(t, 1) for t in d["tune_us"]]}
                       for d in levels],
        "vcycle": {"seconds": vc_s, "vcycles_per_s": 1.0 / vc_s,
                   "algorithmic_bytes": vc_bytes,
                   "GBps": vc_bytes / vc_s / 1e9,
                   "frac": vc_bytes / vc_s / 1e9 / HBM_PEAK_GBS,
                   "frac_of_triad": vc_bytes / vc_s / 1e9 / triad["GBps"],
                   "columns": 1, "dtype": "f64"},
        "psolve": {"seconds": ps_s,
                   "share_of_iteration": ps_s / (t_solve / K / max(iters, 1)),
                   "note": "exact pressure-block solve, one per "
                           "preconditioner application"},
        "stream_triad": triad,
        "roofline": {"bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "frac_of_triad": achieved / triad["GBps"],
                     "traffic": counter_traffic(),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 "
                                     "FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "level-0 residual SpMV (sliced-ELL 3x3 blocks, "
                               "1 column, FP64)",
                     "bytes_per_launch": k_bytes,
                     "avg_launch_us": k_avg_s * 1e6,
                     "launches": launches},
    }

    if not args.no_fp32:
        sol32 = Solver(blocks, s.n_u, s.n_t, s.n_p, coords=coords,
                       precision="fp32")
        for _ in range(args.warmup):
            sol32.solve(b, out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            x32, i32 = sol32.solve(b, out=x)
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - t0) / K
        out["fp32_prec"] = {"solve_s": t32, "iterations": i32["iterations"],
                            "true_rel_residual": i32["true_rel_residual"],
                            "converged": bool(i32["converged"]),
                            "speedup_vs_fp64": (t_solve / K) / t32}
        del sol32

    if not args.no_forms and args.config == "c2":
        out["forms"] = forms(torch, s, blocks, coords, b, t_solve / K)

    if not args.no_cpu_baseline:
        v_gpu = sol.apply_prec(b).cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(s, iters, args.cpu_sample_its,
                                           v_gpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
