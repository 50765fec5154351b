#!/usr/bin/env python
"""Benchmark of the block-preconditioned FGMRES solve on one MI355X.

Workload (default): the precision form, a 128x128x64 Q1 hex mesh with 12
mesh-aligned fractures of random extent and a layered modulus (n_u
3,351,615, n_t 110,601, n_p 36,867).  One step is one pass of the whole path
on device-resident inputs: preconditioner construction (H~, S1 = A + C1
H~^-1 C2, the nested-dissection factorization of the pressure block, the
smoothed-aggregation hierarchy with its Galerkin products) followed by the
FGMRES(50) solve to a true relative residual of 1e-8.  The steps run twice:
with the AMG hierarchy stored and applied in FP32 (the production form) and
all in FP64.

Printed: one JSON line.  ``value`` is the FGMRES time-to-1e-8 in seconds with
the FP32 hierarchy (mean over the timed steps); ``fp64`` holds the plain FP64
path and ``fp32_speedup_vs_fp64`` the ratio.  Added: the V-cycle bandwidth,
the pressure solve, the roofline of the dominant kernel (level-0 residual
SpMV of the V-cycle, timed with HIP events on the library's stream inside
the timed region), the error against the FP64 oracle, the other workloads
(``forms``: the 10^3 latency case, the 80^3 plain FP64 case with its own
roofline, the 32-column batch with its SpMM bandwidth, the adjoint, open
faces) and the CPU oracle baseline.
"""
import argparse
import hashlib
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
    "c3": "128x128x64 Q1 hex, 12 random mesh-aligned fractures, layered "
          "modulus (8 layers, contrast 1e3), FP32 hierarchy vs all-FP64",
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
    residual products with A_l (their vector streams beyond the gathered
    input and one output, D^-1 included: pre 4 (b, D^-1, d, R), residual 1
    (R), post 2 + 2 (b, D^-1; D^-1, x)), restriction, prolongation; the
    coarsest level reads its dense FP64 inverse once."""
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
        total += nv * 9 * n * sv
        total += spmv_bytes(nnzP, nc, n, sv, nv=nv)          # R = P^T
        total += spmv_bytes(nnzP, n, nc, sv, nv=nv)          # P
    return total


def counter_traffic(name):
    """HBM bytes per launch of a kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (profiles/<name>.json), each scaled by what
    the counter reads for a plain copy of known size; None once the kernel
    source differs from the one the counters were taken on."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    try:
        with open(path) as f:
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


def progress(msg):
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def _events(torch, sol, fn, reps):
    """Mean device time of fn() over reps calls, HIP events on the library's
    stream (the current stream when the solver was made)."""
    for _ in range(3):
        fn()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(sol.stream)
    for _ in range(reps):
        fn()
    ev1.record(sol.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps / 1e3


def run_steps(torch, sol, blocks, coords, b, x, warmup, steps, timer=False):
    """warmup + timed steps of setup + solve; returns per-step means."""
    for _ in range(warmup):
        sol.setup(blocks, coords)
        sol.solve(b, out=x)
    torch.cuda.synchronize()
    if timer:
        sol.kernel_timer(enable=True, reset=True)
    t_setup = t_solve = 0.0
    infos = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        sol.setup(blocks, coords)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = sol.solve(b, out=x)
        torch.cuda.synchronize()
        t_setup += t1 - t0
        t_solve += time.perf_counter() - t1
        infos.append(info)
    t_all = time.perf_counter() - t_all
    launches, kernel_ms = (sol.kernel_timer(enable=False, reset=True)
                           if timer else (0, 0.0))
    for inf in infos:
        if not inf["converged"] or inf["true_rel_residual"] > 1e-8:
            raise SystemExit(f"solve did not converge: {inf}")
    return {"solve_s": t_solve / steps, "setup_s": t_setup / steps,
            "step_s": t_all / steps, "iterations": infos[-1]["iterations"],
            "true_rel_residual": infos[-1]["true_rel_residual"],
            "setup_parts_s": sol.setup_times(),
            "timer": (launches, kernel_ms)}


def path_report(torch, sol, s, res, sv, nrep=20):
    """V-cycle and pressure-solve figures of a set-up solver, the level-0
    residual SpMV (timed launches in res['timer']) as roofline."""
    levels = [sol.level_info(l) for l in range(sol.num_levels())]
    vb = torch.randn(s.n_u, dtype=torch.float64, device="cuda")
    vx = torch.empty_like(vb)
    vc_s = _events(torch, sol, lambda: sol.vcycle(vb, out=vx), nrep)
    vc_bytes = vcycle_bytes(levels, sv=sv)
    wp = torch.randn(s.n_p, dtype=torch.float64, device="cuda")
    vp = torch.empty_like(wp)
    ps_s = _events(torch, sol, lambda: sol.psolve(wp, out=vp), nrep)
    pinfo = sol.pressure_info()
    it_s = res["solve_s"] / max(res["iterations"], 1)
    launches, kernel_ms = res["timer"]
    d0 = levels[0]
    k_bytes = spmv_bytes(d0["nnz_scalar"], s.n_u, s.n_u, sv=sv, extra_vec=1)
    k_avg_s = kernel_ms / max(launches, 1) / 1e3
    out = {
        "amg_levels": [dict({"dofs": d["n_dofs"], "nnz": d["nnz_scalar"],
                             "layout_A_P_R": d["layout"]},
                            **({"tuned_us_A_P_R": [round(t, 1)
                                                   for t in d["tune_us"]]}
                               if any(d["tune_us"]) else {}))
                       for d in levels],
        "vcycle": {"seconds": vc_s, "vcycles_per_s": 1.0 / vc_s,
                   "algorithmic_bytes": vc_bytes,
                   "GBps": vc_bytes / vc_s / 1e9,
                   "frac": vc_bytes / vc_s / 1e9 / HBM_PEAK_GBS,
                   "columns": 1, "dtype": "f32" if sv == 4 else "f64"},
        "psolve": {"seconds": ps_s, "share_of_iteration": ps_s / it_s,
                   "algorithmic_bytes": pinfo["solve_bytes"],
                   "GBps": pinfo["solve_bytes"] / ps_s / 1e9,
                   "levels": pinfo["n_levels"], "fronts": pinfo["n_fronts"],
                   "factor_entries": pinfo["factor_entries"],
                   "max_pivots": pinfo["max_pivots"],
                   "max_boundary": pinfo["max_boundary"],
                   "note": "nested-dissection multifrontal solve, FP64, one "
                           "per preconditioner application"},
        "level0_residual_spmv": {
            "bytes_per_launch": k_bytes, "avg_launch_us": k_avg_s * 1e6,
            "launches": launches,
            "GBps": k_bytes / k_avg_s / 1e9 if launches else None},
    }
    return out


def stream_triad(torch, sol, n=1 << 29, reps=10):
    """a = b + s c over three n-double arrays (4 GiB each by default) with the
    library's triad kernel; HIP events on the library's stream, best of
    ``reps`` after a warm-up, 24 bytes per element."""
    b = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    sol.stream_triad(b, c, 3.0, a)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sol.stream)
        sol.stream_triad(b, c, 3.0, a)
        e1.record(sol.stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    ok = bool((a == 7.0).all())
    del a, b, c
    torch.cuda.empty_cache()
    gbs = 24.0 * n / best / 1e9
    return {"GBps": gbs, "frac": gbs / HBM_PEAK_GBS, "seconds": best,
            "array_bytes": 8 * n, "check": ok}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, gpu_iters, sample_its, v_gpu):
    """The CPU FP64 oracle on the same workload, one thread: its
    preconditioner setup (reported, not in value), then ``sample_its``
    FGMRES(50) iterations (CGS2) from x0 = 0 with every iteration timed; the
    iteration time is fitted as a + b j (j = position in the Arnoldi cycle,
    the orthogonalization cost grows with it) and summed over the GPU's
    iteration count.  ``v_gpu`` maps labels to the GPU's M^-1 b, compared
    with the oracle's."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pc = oracle.BlockPrecond(s.blocks(), s.n_u, s.n_t, s.n_p,
                                 coords=s.coords)
        t_setup = time.perf_counter() - t0
        stamps = []
        apply = pc.apply

        def stamped(w):
            stamps.append(time.perf_counter())
            return apply(w)
        t0 = time.perf_counter()
        _, info = oracle.fgmres(pc.matvec, stamped, s.b, rtol=1e-8,
                                maxit=sample_its, ortho="cgs2")
        stamps.append(time.perf_counter())
        t_its = time.perf_counter() - t0
        vo = pc.apply(s.b)
    per = np.diff(stamps)                      # iteration j = 1 .. k
    j = np.arange(1, per.size + 1, dtype=float)
    if per.size >= 2:
        b1, a0 = np.polyfit(j, per, 1)
    else:
        b1, a0 = 0.0, float(per.mean())
    jj = (np.arange(gpu_iters) % 50) + 1
    value = float(np.sum(a0 + b1 * jj))
    diffs = {k: float(np.linalg.norm(v - vo) / np.linalg.norm(vo))
             for k, v in v_gpu.items()}
    return {"value": value, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"{per.size} FGMRES(50) iterations (CGS2) of the "
                       f"NumPy/SciPy FP64 oracle on this workload after its "
                       f"setup ({t_setup:.1f} s, not in value); iteration "
                       f"time fitted as {a0:.3f} + {b1:.4f} j s (j = step in "
                       f"the Arnoldi cycle) and summed over the GPU's "
                       f"{gpu_iters} iterations"),
            "setup_s": t_setup, "sampled_iteration_s": [float(p) for p in per],
            "sample_wall_s": t_its,
            "gpu_vs_oracle_apply_rel_diff": diffs,
            "cpu_model": cpu_model(), "host": platform.node()}


FORM_NAMES = ("latency", "plain", "batch", "adjoint", "open")


def forms(torch, only=None):
    """The other workloads, each after one untimed warm-up call; ``only``
    restricts the run to one of FORM_NAMES."""
    out = {}

    def want(name):
        return only is None or only == name
    if want("latency"):
        out.update(form_latency(torch))
    if want("plain"):
        out.update(form_plain(torch))
    if want("batch"):
        out.update(form_batch(torch))
    if want("adjoint"):
        out.update(form_adjoint(torch))
    if want("open"):
        out.update(form_open(torch))
    return out


def form_latency(torch):
    """10^3: the launch-bound end, time to solution with setup, and the
    oracle's iteration count and solution."""
    import fracgen
    import oracle
    from paper_2112_12397_amd import Solver
    out = {}
    progress("forms: 10^3")
    s1 = fracgen.make_config("c1")
    b1 = torch.tensor(s1.b, device="cuda")
    blocks1 = device_blocks(torch, s1)
    c1c = torch.tensor(s1.coords, device="cuda")
    sol = Solver(blocks1, s1.n_u, s1.n_t, s1.n_p, coords=c1c)
    x1 = torch.empty_like(b1)
    r1 = run_steps(torch, sol, blocks1, c1c, b1, x1, 2, 10)
    pc1 = oracle.BlockPrecond(s1.blocks(), s1.n_u, s1.n_t, s1.n_p,
                              coords=s1.coords)
    xo1, io1 = oracle.fgmres(pc1.matvec, pc1.apply, s1.b, rtol=1e-8,
                             ortho="cgs2")
    del r1["timer"]
    r1.update({"workload": WORKLOADS["c1"], "N": s1.N,
               "oracle_iterations": io1.iterations,
               "x_rel_diff_vs_oracle": float(np.linalg.norm(
                   x1.cpu().numpy() - xo1) / np.linalg.norm(xo1))})
    out["latency_10cube_fp64"] = r1
    return out


def form_plain(torch):
    """80^3 plain FP64: its own roofline, V-cycle and pressure solve."""
    import fracgen
    from paper_2112_12397_amd import Solver
    out = {}
    progress("forms: 80^3 plain FP64")
    s2 = fracgen.make_config("c2")
    b2 = torch.tensor(s2.b, device="cuda")
    blocks2 = device_blocks(torch, s2)
    c2c = torch.tensor(s2.coords, device="cuda")
    sol = Solver(blocks2, s2.n_u, s2.n_t, s2.n_p, coords=c2c)
    x2 = torch.empty_like(b2)
    r2 = run_steps(torch, sol, blocks2, c2c, b2, x2, 1, 3, timer=True)
    rep = path_report(torch, sol, s2, r2, 8)
    t_upd = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.update_values(blocks2)
        torch.cuda.synchronize()
        t_upd.append(time.perf_counter() - t0)
    k = rep["level0_residual_spmv"]
    tr2 = counter_traffic("level0_residual_spmv_c2_fp64_counters")
    res2 = {"workload": WORKLOADS["c2"], "N": s2.N,
            "solve_s": r2["solve_s"], "setup_s": r2["setup_s"],
            "iterations": r2["iterations"],
            "true_rel_residual": r2["true_rel_residual"],
            "setup_parts_s": r2["setup_parts_s"],
            "update_values_s": min(t_upd),
            "update_parts_s": sol.setup_times(),
            "hierarchy_reused": sol.hierarchy_reused(),
            "roofline": {"bound": "hbm", "achieved": k["GBps"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": k["GBps"] / HBM_PEAK_GBS,
                         "traffic": tr2,
                         "traffic_GBps": (tr2 / (k["avg_launch_us"] * 1e-6)
                                          / 1e9 if tr2 and k["launches"]
                                          else None),
                         "kernel": "level-0 residual SpMV, FP64",
                         **k}}
    res2.update({kk: rep[kk] for kk in ("vcycle", "psolve", "amg_levels")})
    for mode in ("tpu", "tup_star"):
        solm = Solver(blocks2, s2.n_u, s2.n_t, s2.n_p, coords=c2c, mode=mode)
        solm.solve(b2, out=x2)
        t, (_, inf) = _timed(torch, lambda: solm.solve(b2, out=x2), 2)
        res2[mode] = {"solve_s": t, "iterations": inf["iterations"],
                      "true_rel_residual": inf["true_rel_residual"],
                      "speedup_vs_tup": r2["solve_s"] / t}
        del solm
    out["plain_fp64_80cube"] = res2
    return out


def form_batch(torch):
    """32 right-hand sides sharing one Jacobian, FP32 hierarchy."""
    import fracgen
    from fracgen.configs import rhs_batch
    from paper_2112_12397_amd import solver_from_system
    out = {}
    progress("forms: 64^3 batch")
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
    # the batched level-0 residual SpMM, timed launch by launch (eager cycle)
    sol.kernel_timer(enable=True, reset=True)
    sol.solve_batch(B, out=X)
    nl, ms = sol.kernel_timer(enable=False, reset=True)
    d0 = sol.level_info(0)
    kb = spmv_bytes(d0["nnz_scalar"], s4.n_u, s4.n_u, sv=4, nv=32,
                    extra_vec=1)
    avg = ms / max(nl, 1) / 1e3
    trb = counter_traffic("batch_spmm_c4_fp32x32_counters")
    out["batch32_64cube_fp32prec"] = {
        "workload": "64^3 Q1 hex, 6 random fractures, 32 RHS (norms 1e-2..1e2)",
        "batch_s": tb, "per_rhs_s": tb / 32, "sequential_s": tq,
        "speedup_vs_sequential": tq / tb, "status": st,
        "iterations_max": max(i["iterations"] for i in infs),
        "iterations_mean": float(np.mean([i["iterations"] for i in infs])),
        "sequential_iterations_mean": float(np.mean(its1)),
        "worst_true_rel_residual": max(i["true_rel_residual"] for i in infs),
        "level0_residual_spmm": {
            "columns": 32, "dtype": "f32", "bytes_per_launch": kb,
            "avg_launch_us": avg * 1e6, "launches": nl,
            "GBps": kb / avg / 1e9 if nl else None,
            "frac": kb / avg / 1e9 / HBM_PEAK_GBS if nl else None,
            "traffic": trb,
            "traffic_GBps": trb / avg / 1e9 if trb and nl else None},
        "n_u": s4.n_u, "n_t": s4.n_t, "n_p": s4.n_p}
    return out


def form_adjoint(torch):
    """Adjoint solve and transmissibility gradient."""
    import fracgen
    from fracgen.configs import observations
    from paper_2112_12397_amd import solver_from_system
    out = {}
    progress("forms: 48^3 adjoint")
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
    return out


def form_open(torch):
    """Open faces (Q2 != 0): sequential AMG calls (t-u-p) or S~ (t-p-u)."""
    import fracgen
    from paper_2112_12397_amd import solver_from_system
    out = {}
    progress("forms: 80^3 open faces")
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
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-its", type=int, default=4)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other workloads (forms)")
    ap.add_argument("--only-form", choices=FORM_NAMES,
                    help="run only this one of the other workloads and print "
                         "its JSON (profiling aid)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; runs on several GPUs "
              "are not supported (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import fracgen
    from paper_2112_12397_amd import Solver

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.only_form:
        print(json.dumps(forms(torch, only=args.only_form)), flush=True)
        return
    progress(f"generating {args.config}")
    s = fracgen.make_config(args.config)
    blocks = device_blocks(torch, s)
    coords = torch.tensor(s.coords, device="cuda")
    b = torch.tensor(s.b, device="cuda")
    x = torch.empty_like(b)
    K = args.steps

    paths, reports, v_gpu = {}, {}, {}
    for prec, sv in (("fp32", 4), ("fp64", 8)):
        progress(f"{args.config} {prec}: {args.warmup} + {K} steps")
        sol = Solver(blocks, s.n_u, s.n_t, s.n_p, coords=coords,
                     precision=prec)
        res = run_steps(torch, sol, blocks, coords, b, x, args.warmup, K,
                        timer=True)
        reports[prec] = path_report(torch, sol, s, res, sv)
        paths[prec] = res
        v_gpu[prec] = sol.apply_prec(b).cpu().numpy()
        if prec == "fp64":
            triad = stream_triad(torch, sol)
        del sol
        torch.cuda.empty_cache()

    r32, r64 = paths["fp32"], paths["fp64"]
    k = reports["fp32"]["level0_residual_spmv"]
    traffic = counter_traffic("level0_residual_spmv_c3_fp32_counters")
    k_s = k["avg_launch_us"] * 1e-6
    out = {
        "metric": METRIC,
        "value": r32["solve_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["step_s"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "dtype_note": "AMG hierarchy and V-cycle in FP32; Jacobian product, "
                      "Arnoldi, true residual, coarsest solve and pressure "
                      "factor in FP64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}",
                   "n_u": s.n_u, "n_t": s.n_t, "n_p": s.n_p, "N": s.N,
                   "mode": "t-u-p", "restart": 50, "rtol": 1e-8,
                   "seed": s.seed, "step": "setup + solve on "
                                           "device-resident inputs"},
        "iterations": r32["iterations"],
        "true_rel_residual": r32["true_rel_residual"],
        "setup_s": r32["setup_s"],
        "setup_parts_s": r32["setup_parts_s"],
        "fp64": {kk: r64[kk] for kk in ("solve_s", "setup_s", "step_s",
                                        "iterations", "true_rel_residual",
                                        "setup_parts_s")},
        "fp32_speedup_vs_fp64": r64["solve_s"] / r32["solve_s"],
        "vcycle": {"fp32": reports["fp32"]["vcycle"],
                   "fp64": reports["fp64"]["vcycle"]},
        "psolve": reports["fp32"]["psolve"],
        "amg_levels": reports["fp32"]["amg_levels"],
        "level0_residual_spmv_fp64": reports["fp64"]["level0_residual_spmv"],
        "stream_triad": triad,
        "roofline": {"bound": "hbm", "achieved": k["GBps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": k["GBps"] / HBM_PEAK_GBS,
                     "frac_of_triad": k["GBps"] / triad["GBps"],
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 "
                                     "FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "traffic_GBps": (traffic / k_s / 1e9
                                      if traffic and k["launches"] else None),
                     "traffic_frac": (traffic / k_s / 1e9 / HBM_PEAK_GBS
                                      if traffic and k["launches"] else None),
                     "bytes_model": "survey CSR model: value + 4-byte "
                                    "column per true nonzero, vectors; the "
                                    "blocked slots move fewer bytes, so "
                                    "frac can exceed 1 while traffic_frac "
                                    "stays below",
                     "kernel": "level-0 residual SpMV of the V-cycle "
                               "(sliced-ELL 3x3 blocks, 1 column, FP32)",
                     "bytes_per_launch": k["bytes_per_launch"],
                     "avg_launch_us": k["avg_launch_us"],
                     "launches": k["launches"]},
    }
    if not args.no_forms:
        out["forms"] = forms(torch)
    if not args.no_cpu_baseline:
        progress("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(s, r32["iterations"],
                                           args.cpu_sample_its, v_gpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
