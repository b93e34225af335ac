"""Benchmark: space-time multigrid V-cycles on one MI355X.

Workload (default): 2-D heat equation on the unit square, Q1 with 127 x 127
interior nodes, N = 256 DG(p_t=1) slabs on (0,1) (mu = tau/h^2 = 64),
f = sum of 8 seeded Gaussian bumps, u0 = sin(pi x) sin(pi y); FP64.
A step is one V-cycle of the whole hot path (residual, damped block-Jacobi
smoothing by fast diagonalisation, restriction, prolongation, coarsest solve)
plus the fine residual norm used by the stopping test.  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line.  Besides DoF*V-cycles/s it reports the time to a 1e-10
relative residual for the FP64 solve and for the mixed-precision solve (FP32
inner V-cycle inside FP64 iterative refinement), the roofline position of the
dominant kernel (per-launch durations from HIP events recorded by the library
around each launch during a profiled pass of the same steps), and the CPU
oracle timed on a bounded sample of the same workload family.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6    # MI355X dense FP64 matrix
FP32_MFMA_PEAK_TFS = 157.3   # MI355X dense FP32 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=2, help="workload index (1..5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels eagerly instead of replaying a hipGraph")
    ap.add_argument("--only-timed", action="store_true", help="timed V-cycles only (for profiler runs)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel families")
    ap.add_argument("--no-inexact", action="store_true", help="skip the spatial-multigrid smoother measurement")
    ap.add_argument("--no-mesh", action="store_true", help="skip the P1 tetrahedral-mesh measurement")
    ap.add_argument("--only-mesh", action="store_true", help="only the P1 tetrahedral-mesh measurement (for profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (calibrates HBM byte counters) and exit")
    return ap.parse_args()


def measure_inexact(stmg, torch, d, n, N, pt, b, F, u_ref, dev, args):
    """The paper's smoother (one spatial multigrid V-cycle per slab, nu_x = 2,
    omega_x = 2/3, block Jacobi in space) on the same workload: V-cycle
    throughput, time to 1e-10 and the HBM rate of its stencil kernels."""
    X = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev, smoother="spatial_mg")
    steps = max(args.steps // 2, 5)
    u = torch.zeros_like(F)
    if not args.no_graph:
        X.set_graph(True)
    X.solve(F, u=u, rtol=0.0, maxit=2, raise_on_noconv=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X.solve(F, u=u, rtol=0.0, maxit=steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ux, itsx, histx = X.solve(F, u=u, rtol=1e-10, maxit=100)
    torch.cuda.synchronize()
    tx = time.perf_counter() - t0
    err = (torch.linalg.vector_norm(ux - u_ref) / torch.linalg.vector_norm(u_ref)).item()
    X.set_graph(False)
    u2 = torch.zeros_like(F)
    X.solve(F, u=u2, rtol=0.0, maxit=1, raise_on_noconv=False)
    X.profile_start()
    X.solve(F, u=u2, rtol=0.0, maxit=steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    kinds = ["residual", "jacobi", "xfer_x", "restrict", "prolong", "fused", "pass_fwd", "pass_inv", "other"]
    prof = {k: X.profile_read(k, level=-1) for k in kinds}
    jac0_ms, jac0_cnt = X.profile_read("jacobi", level=0)
    X.profile_stop()
    nu = X.params["nu1"] + X.params["nu2"]
    jac_bytes = spatial_cycle_bytes([X.levels[0]], d, X.nt, b)[0] * nu * steps
    gbs = jac_bytes / (jac0_ms * 1e-3) / 1e9
    dof = X.level_dof(0)
    X.close()
    return {"value": dof * steps / el, "unit": "DoF*V-cycles/s", "ms_per_step": 1e3 * el / steps,
            "steps": steps, "time_to_1e-10_s": tx, "cycles_to_1e-10": itsx, "final_relres": histx[-1][0],
            "rel_error_vs_exact_smoother_solution": err,
            "jacobi_kernels_fine_level": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": gbs / HBM_PEAK_GBS, "launches": jac0_cnt,
                                          "avg_launch_ms": jac0_ms / max(jac0_cnt, 1),
                                          "bytes_total": jac_bytes},
            "kernel_breakdown_ms_per_step": {k: v[0] / steps for k, v in prof.items()}}


def measure_p1(stmg, torch, dev, args):
    """The parallel example's setting on a P1 mesh: the unit cube of 49,152
    tetrahedra (12 refined four times), p_t = 3, tau = 0.1, nu1 = nu2 = 1,
    omega_t = 1, one spatial cycle per slab (node-block Jacobi, nu_x = 2,
    omega_x = 2/3) on N = 1024 slabs.  V-cycle throughput, time to the
    examples' reduction 1e-8 and the HBM rate of the CSR residual kernel."""
    from paper_1411_0519_amd import workloads
    coarse = workloads.coarse_mesh("cube12")
    R, N, pt = 4, 1024, 3
    X = stmg.Solver(3, R, N, pt=pt, T=0.1 * N, omega=1.0, nu1=1, nu2=1, smoother="spatial_mg", mesh=coarse,
                    device=dev)
    lv = stmg.mesh_level(*coarse, R)
    f, u0 = workloads.mesh_data(lv["points"], N, seed=21)
    F = X.rhs(torch.from_numpy(f.ravel()).to(dev), torch.from_numpy(u0.ravel()).to(dev))
    steps = max(args.steps // 2, 5)
    u = torch.zeros_like(F)
    if not args.no_graph:
        X.set_graph(True)
    X.solve(F, u=u, rtol=0.0, maxit=2, raise_on_noconv=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X.solve(F, u=u, rtol=0.0, maxit=steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, hist = X.solve(F, u=u, rtol=1e-8, maxit=100)
    torch.cuda.synchronize()
    tsolve = time.perf_counter() - t0
    # the same solve with FP64 refinement around an FP32 inner cycle
    Xm = stmg.Solver(3, R, N, pt=pt, T=0.1 * N, omega=1.0, nu1=1, nu2=1, smoother="spatial_mg", mesh=coarse,
                     device=dev, precision="mixed")
    if not args.no_graph:
        Xm.set_graph(True)
    um = torch.zeros_like(F)
    Xm.solve(F, u=um, rtol=0.0, maxit=2, raise_on_noconv=False)
    um.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    um, itsm, histm = Xm.solve(F, u=um, rtol=1e-8, maxit=100)
    torch.cuda.synchronize()
    tmixed = time.perf_counter() - t0
    Xm.close()
    X.set_graph(False)
    u2 = torch.zeros_like(F)
    X.solve(F, u=u2, rtol=0.0, maxit=1, raise_on_noconv=False)
    X.profile_start()
    X.solve(F, u=u2, rtol=0.0, maxit=steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    kinds = ["residual", "jacobi", "xfer_x", "restrict", "prolong", "other"]
    prof = {k: X.profile_read(k, level=-1) for k in kinds}
    res_ms, res_cnt = X.profile_read("residual", level=0)
    X.profile_stop()
    dof = X.level_dof(0)
    nnz = len(lv["col"])
    # u and F read once, r written once, the CSR pattern and both value arrays
    res_bytes = 24.0 * dof + 20.0 * nnz + 4.0 * (len(lv["rowptr"]))
    gbs = res_bytes * res_cnt / (res_ms * 1e-3) / 1e9
    out = {"workload": "heat3d_p1_cube12_R4_N1024_p3: unit cube of 49,152 P1 tetrahedra (12 refined 4 times, "
                       f"{X.levels[0]['nx']} interior nodes), N=1024 slabs, tau=0.1, DG p_t=3, FP64, "
                       "nu1=nu2=1, omega_t=1, spatial cycle nu_x=2 omega_x=2/3, schedule " + X.schedule,
           "dof": dof, "value": dof * steps / el, "unit": "DoF*V-cycles/s", "ms_per_step": 1e3 * el / steps,
           "steps": steps, "time_to_1e-8_s": tsolve, "cycles_to_1e-8": its, "final_relres": hist[-1][0],
           "mixed_time_to_1e-8_s": tmixed, "mixed_cycles_to_1e-8": itsm, "mixed_final_relres": histm[-1][0],
           "mixed_rel_diff_vs_fp64": (torch.linalg.vector_norm(um - u) / torch.linalg.vector_norm(u)).item(),
           "residual_kernel_fine_level": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": gbs / HBM_PEAK_GBS, "launches": res_cnt,
                                          "avg_launch_ms": res_ms / max(res_cnt, 1), "bytes_per_launch": res_bytes},
           "kernel_breakdown_ms_per_step": {k: v[0] / steps for k, v in prof.items()}}
    X.close()
    return out


def cpu_baseline(budget_s=20.0):
    """Oracle V-cycles on a reduced member of the same family (same mu, p_t)."""
    import numpy as np

    from oracle import multigrid, spacetime
    from paper_1411_0519_amd import workloads

    d, n, N, pt = 2, 63, 64, 1      # mu = (1/64) * 64^2 = 64, like the 127^2 x 256 workload
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(d, n, N, pt)
    f, u0 = workloads.make(d, n, N, batch=1, seed=2, f="bumps", u0="sine1")
    F = spacetime.rhs(H.fine, f, u0)
    setup = time.perf_counter() - t0
    k = len(H.levels) - 1
    u = np.zeros_like(F)
    H.vcycle(k, u, F)                 # factorisations happen on first use
    cycles = 0
    t0 = time.perf_counter()
    while True:
        u = H.vcycle(k, u, F)
        _ = np.linalg.norm(H.residual(k, u, F))
        cycles += 1
        el = time.perf_counter() - t0
        if el > budget_s or cycles >= 50:
            break
    rate = H.fine.dof * cycles / el
    return {"value": rate, "unit": "DoF*V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"2-D n={n} N={N} p_t={pt} (mu=64, {H.fine.dof} DoF), {cycles} V-cycles + residual "
                      f"norm each, {el:.1f} s; setup {setup:.1f} s excluded; scipy CSR SpMV and SuperLU "
                      f"solves run on one thread",
            "host_cpus_available": len(os.sched_getaffinity(0))}


TRANSFORM_NAMES = ["default", "lds", "register", "register_twice_folded", "slab_resident",
                   "twice_folded_residual_fused"]


def tuned_levels(S, tuning):
    """Per-level kernel families the autotuner picked (all but the coarsest level)."""
    if tuning is None:
        return None
    return [{"level": k, "n": S.levels[k]["n"], "N": S.levels[k]["N"], "small_step": bool(t[0]),
             "transform": TRANSFORM_NAMES[t[1]], "step_ms": round(t[2], 4)}
            for k, t in enumerate(tuning[:-1])]


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE / WRITE_SIZE runs, scaled by a device copy of known
    size), or None when there is no record or the kernel's source changed
    since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    src = os.path.join(ROOT, rec["source"])
    if rec.get("kernel") != kernel or not os.path.exists(src):
        return None
    with open(src, "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec


def spatial_cycle_bytes(levels, d, nt, b, nu1x=2, nu2x=2, elem=8):
    """Algorithmic HBM bytes of the block-Jacobi/defect launches of one spatial
    cycle per time level (reads of x, f and, for the fused update, u; one
    write): first pre-smoothing step reads f only; the last post-smoothing
    step of the top sub-level also reads u; a one-node sub-level reads f and
    writes x."""
    out = []
    for L in levels:
        n, N = L["n"], L["N"]
        tot = 0.0
        j = 0
        m = n
        while True:
            nvals = b * N * nt * m ** d
            if m == 1:
                tot += 2 * nvals
                break
            arrays = (2 + 3 * (nu1x - 1)) if nu1x > 0 else 0
            arrays += 3                                    # defect
            arrays += 3 * nu2x + (1 if j == 0 else 0)      # post-smoothing (+ u read)
            tot += arrays * nvals
            m = (m - 1) // 2
            j += 1
        out.append(tot * elem)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (one process, one device); multi-GPU runs are not supported, use --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1411_0519_amd import stmg, workloads

    dev = "cuda:0"
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "copies": 5}))
        return
    if args.only_mesh:
        with torch.cuda.stream(torch.cuda.Stream(device=dev)):
            print(json.dumps({"p1_mesh": measure_p1(stmg, torch, dev, args)}))
        return
    w = workloads.WORKLOADS[args.workload]
    d, n, N, pt, b = w["dim"], w["n"], w["N"], w["pt"], w["batch"]
    _, f, u0 = workloads.workload(args.workload)
    stream = torch.cuda.Stream(device=dev)
    result = {}
    with torch.cuda.stream(stream):
        S = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev)
        fg = torch.from_numpy(f.ravel()).to(dev)
        ug0 = torch.from_numpy(u0.ravel()).to(dev)
        F = S.rhs(fg, ug0)
        dof = S.level_dof(0)
        u = torch.zeros(dof, dtype=torch.float64, device=dev)
        tuning = None if args.no_autotune else S.autotune()
        if not args.no_graph:
            S.set_graph(True)
        # warmup (also records the graph)
        S.solve(F, u=u, rtol=0.0, maxit=max(args.warmup, 1), raise_on_noconv=False)
        torch.cuda.synchronize()
        u.zero_()
        t0 = time.perf_counter()
        _, its, _ = S.solve(F, u=u, rtol=0.0, maxit=args.steps, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert its == args.steps
        ms = 1e3 * el / args.steps
        value = dof * args.steps / el
        if args.only_timed:
            print(json.dumps({"metric": "space-time DoF*V-cycles/s", "value": value, "ms_per_step": ms}))
            return

        # time to a 1e-10 relative residual, FP64 (setup excluded)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u64, its64, hist64 = S.solve(F, u=u, rtol=1e-10, maxit=100)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0

        # profiled pass (eager, HIP events around every launch)
        S.set_graph(False)
        u2 = torch.zeros_like(u)
        S.solve(F, u=u2, rtol=0.0, maxit=2, raise_on_noconv=False)
        S.profile_start()
        S.solve(F, u=u2, rtol=0.0, maxit=args.steps, raise_on_noconv=False)
        torch.cuda.synchronize()
        kinds = ["residual", "resid_x", "pass_fwd", "pass_inv", "fused", "small", "restrict", "prolong", "other"]
        prof = {}
        for k in kinds:
            tot, cnt = S.profile_read(k, level=-1)
            tot0, cnt0 = S.profile_read(k, level=0)
            prof[k] = {"ms_total": tot, "launches": cnt, "fine_ms_total": tot0, "fine_launches": cnt0}
        S.profile_stop()
        if not args.no_graph:
            S.set_graph(True)

        # mixed precision: FP32 inner V-cycle, FP64 refinement
        M = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev, precision="mixed")
        tuning_mixed = None if args.no_autotune else M.autotune()
        if not args.no_graph:
            M.set_graph(True)
        um = torch.zeros_like(u)
        M.solve(F, u=um, rtol=0.0, maxit=2, raise_on_noconv=False)   # warm + record graph
        um.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        um, itsm, histm = M.solve(F, u=um, rtol=1e-10, maxit=100)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        err_mixed = (torch.linalg.vector_norm(um - u64) / torch.linalg.vector_norm(u64)).item()
        M.close()

        # mixed precision with the inner cycle's transforms on the bf16 matrix cores
        B = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev, precision="mixed_bf16")
        if not args.no_autotune:
            B.autotune()
        if not args.no_graph:
            B.set_graph(True)
        ub = torch.zeros_like(u)
        B.solve(F, u=ub, rtol=0.0, maxit=2, raise_on_noconv=False)
        ub.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ub, itsb, histb = B.solve(F, u=ub, rtol=1e-10, maxit=100)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        err_bf16 = (torch.linalg.vector_norm(ub - u64) / torch.linalg.vector_norm(u64)).item()
        B.close()

        inexact = None
        if not args.no_inexact:
            inexact = measure_inexact(stmg, torch, d, n, N, pt, b, F, u64, dev, args)
        p1_mesh = None
        if not args.no_mesh:
            p1_mesh = measure_p1(stmg, torch, dev, args)

    # roofline of the dominant transform kernel on the fine level.  Algorithmic
    # work is the dense sine transform's: a length-n dot product (2n flop) per
    # value per transform; the folded kernels execute about half of that on the
    # matrix cores.  The fused kernel does a forward and an inverse transform.
    L0 = S.levels[0]
    nvals = b * L0["N"] * S.nt * L0["n"] ** d
    cand = {k: v for k, v in prof.items() if k in ("pass_fwd", "pass_inv", "fused") and v["fine_launches"] > 0}
    dom = max(cand, key=lambda k: cand[k]["fine_ms_total"])
    avg_ms = cand[dom]["fine_ms_total"] / cand[dom]["fine_launches"]
    transforms = 2 if dom == "fused" else 1
    flops = transforms * 2.0 * L0["n"] * nvals
    hbm_bytes = (24 if dom == "pass_inv" else 16) * nvals
    achieved = flops / (avg_ms * 1e-3) / 1e12
    impl0 = 0 if tuning is None else tuning[0][1]
    # the default FP64 family at n = 63, 127 is twice folded (5: the same with the residual fused in)
    twice = impl0 in (0, 3, 5) and L0["n"] in (63, 127)
    if twice:
        names = {"pass_fwd": "forward x pass (k_pass_reg2<double,2,false,true,false>, twice folded)",
                 "pass_inv": "inverse x pass + update (k_pass_reg2<double,2,true,true,false>, twice folded)",
                 "fused": "fused y pass: forward + time solve + inverse (k_fused_pair2<double,2,2,false>, twice folded, one wave per time component)"}
        kernel_ids = {"pass_fwd": "k_pass_reg2<double, 2, false, true, false>",
                      "pass_inv": "k_pass_reg2<double, 2, true, true, false>", "fused": "k_fused_pair2<double, 2, 2, false>"}
        executed = flops * (L0["n"] + 1) / (4.0 * L0["n"])     # four (h/2)^2 products per column
    else:
        names = {"pass_fwd": "forward x pass (k_pass_reg<double,4,false>)", "pass_inv": "inverse x pass + update (k_pass_reg<double,4,true>)",
                 "fused": "fused y pass: forward + time solve + inverse (k_fused_pair<double,4,2>: one wave per time component)"}
        kernel_ids = {"pass_fwd": "k_pass_reg<double, 4, false, 2, true>", "pass_inv": "k_pass_reg<double, 4, true, 2, true>",
                      "fused": "k_fused_pair<double, 4, 2>"}
        executed = flops * (L0["n"] + 1) / (2.0 * L0["n"])     # two h^2 products per column
    rec = measured_traffic(w["name"], kernel_ids[dom])
    traffic = None if rec is None else rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    roof = {"kernel": names[dom] + ", fine level", "bound": "mfma", "achieved": achieved,
            "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": achieved / FP64_MFMA_PEAK_TFS, "traffic": traffic,
            "traffic_read_write_bytes": None if rec is None else [rec["fetch_bytes_per_launch"],
                                                                  rec["write_bytes_per_launch"]],
            "avg_launch_ms": avg_ms, "launches": cand[dom]["fine_launches"], "flops_per_launch": flops,
            "executed_mfma_flops_per_launch": executed,
            "hbm_bytes_per_launch": hbm_bytes, "hbm_gbs": hbm_bytes / (avg_ms * 1e-3) / 1e9}
    r0 = prof["residual"]
    res_avg = r0["fine_ms_total"] / max(r0["fine_launches"], 1)
    res_bytes = 3 * 8 * nvals                           # read u, F; write r
    res_gbs = res_bytes / (res_avg * 1e-3) / 1e9
    rx0 = prof["resid_x"]                               # read u, F; write the x-transformed residual
    rx_avg = rx0["fine_ms_total"] / rx0["fine_launches"] if rx0["fine_launches"] > 0 else None
    total_prof = sum(v["ms_total"] for v in prof.values())
    out = {
        "metric": "space-time DoF*V-cycles/s (+ time-to-1e-10, mixed vs FP64)",
        "value": value,
        "unit": "DoF*V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: {d}-D Q1 {n}^{d} interior, N={N} slabs, DG p_t={pt}, "
                               f"batch {b}, FP64, omega=1/2, nu1=nu2=2, schedule {S.schedule}",
                   "dof": dof, "levels": S.nlev, "graph": not args.no_graph,
                   "autotuned_levels": tuned_levels(S, tuning)},
        "time_to_1e-10": {"fp64_s": t64, "fp64_cycles": its64, "mixed_s": tm, "mixed_cycles": itsm,
                          "mixed_inner_levels": tuned_levels(S, tuning_mixed),
                          "speedup_mixed_vs_fp64": t64 / tm,
                          "mixed_rel_error_vs_fp64": err_mixed,
                          "fp64_final_relres": hist64[-1][0], "mixed_final_relres": histm[-1][0],
                          "mixed_bf16_s": tb, "mixed_bf16_cycles": itsb, "speedup_mixed_bf16_vs_fp64": t64 / tb,
                          "mixed_bf16_rel_error_vs_fp64": err_bf16, "mixed_bf16_final_relres": histb[-1][0]},
        "roofline": roof,
        "residual_kernel": {"kernel": "k_residual_tile2d (fine level: residual norms and restriction)",
                            "bound": "hbm", "achieved": res_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": res_gbs / HBM_PEAK_GBS, "avg_launch_ms": res_avg,
                            "launches": r0["fine_launches"], "bytes_per_launch": res_bytes},
        "residual_xfwd_kernel": None if rx_avg is None else {
            "kernel": "k_resid_xfwd (fine level: residual fused with the forward x pass, smoothing steps)",
            "bound": "hbm", "achieved": res_bytes / (rx_avg * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": res_bytes / (rx_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": rx_avg,
            "launches": prof["resid_x"]["fine_launches"], "bytes_per_launch": res_bytes},
        "kernel_breakdown_ms_per_step": {k: v["ms_total"] / args.steps for k, v in prof.items()},
        "profiled_ms_per_step": total_prof / args.steps,
    }
    if inexact is not None:
        out["inexact_smoother"] = inexact
    if p1_mesh is not None:
        out["p1_mesh"] = p1_mesh
    if not args.no_cpu_baseline:
        cb = cpu_baseline()
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = value / cb["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
