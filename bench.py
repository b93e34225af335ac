"""Benchmark: space-time multigrid V-cycles on one MI355X.

Headline workload: 3-D heat equation on the unit cube, Q1 with 63^3 interior
nodes, N = 1024 DG(p_t=1) slabs on (0,1) (mu = tau/h^2 = 4, 512,096,256
space-time DoF), f ~ U[-1,1] per node and slab (seed 3), u0 = 0; FP64.
A step is one V-cycle of the whole hot path (residual, damped block-Jacobi
smoothing by fast diagonalisation, restriction, prolongation, coarsest solve)
plus the fine residual norm used by the stopping test.  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line.  Besides DoF*V-cycles/s it reports the time to a 1e-10
relative residual for the FP64 solve and for the two mixed-precision solves
(FP32 inner V-cycle inside FP64 iterative refinement, with FP32 or BF16
matrix-core transforms) with their errors against the FP64 solution, the
roofline position of the dominant fine-level kernel (algorithmic bytes per
launch over the average launch duration, from HIP events the library records
around each launch on its stream during a profiled pass of the same steps),
the CPU oracle timed on a bounded sample of the same workload family, and
secondary lines: the 2-D 127^2 x 256 workload, the paper's inexact smoother
there, and the parallel example's P1 tetrahedral mesh.
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


def progress(msg):
    """One line per finished stage on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3, help="headline workload index (1..5)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 2-D 127^2 x 256 secondary line")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 255^2 x 512 x 64-RHS FP32 line")
    ap.add_argument("--only-batched", action="store_true", help="only the batched line (for profiler runs)")
    ap.add_argument("--cpu-full-w2", action="store_true",
                    help="also time the CPU oracle on the whole 127^2 x 256 workload (about 2 minutes, 12 GB of host memory)")
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
    """Oracle V-cycles on a reduced member of the headline family (3-D, same
    mu = 4 and p_t = 1, seeded f ~ U[-1,1], u0 = 0)."""
    import numpy as np

    from oracle import multigrid, spacetime
    from paper_1411_0519_amd import workloads

    d, n, N, pt = 3, 15, 64, 1      # mu = (1/64) * 16^2 = 4, like the 63^3 x 1024 workload
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(d, n, N, pt)
    f, u0 = workloads.make(d, n, N, batch=1, seed=3, f="uniform", u0="zero")
    F = spacetime.rhs(H.fine, f, u0)
    k = len(H.levels) - 1
    u = np.zeros_like(F)
    H.vcycle(k, u, F)                 # factorisations happen on first use
    setup = time.perf_counter() - t0
    u = np.zeros_like(F)
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
            "sample": f"3-D n={n} N={N} p_t={pt} (mu=4 like the headline, schedule {H.schedule}, {H.fine.dof} DoF), "
                      f"{cycles} V-cycles + residual norm each, {el:.1f} s; hierarchy, assembly and LU "
                      f"factorisations ({setup:.1f} s) excluded; scipy CSR SpMV and SuperLU solves run on one thread",
            "host_cpus_available": len(os.sched_getaffinity(0))}


def cpu_full_w2(budget_s=30.0):
    """The oracle on the whole 127^2 x 256 workload (8.26 M DoF, about 294 M
    nonzeros of the assembled space-time matrix): hierarchy, assembly and LU
    factorisations timed apart, then V-cycles with the residual norm each for
    about budget_s seconds (at least two)."""
    import numpy as np

    from oracle import multigrid, spacetime
    from paper_1411_0519_amd import workloads

    d, n, N, pt = 2, 127, 256, 1
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(d, n, N, pt)
    f, u0 = workloads.make(d, n, N, batch=1, seed=2, f="bumps", u0="sine1")
    F = spacetime.rhs(H.fine, f, u0)
    k = len(H.levels) - 1
    H.vcycle(k, np.zeros_like(F), F)           # factorisations happen on first use
    setup = time.perf_counter() - t0
    progress(f"CPU oracle, whole 127^2 x 256 workload: set up in {setup:.1f} s")
    u = np.zeros_like(F)
    cycles = 0
    t0 = time.perf_counter()
    while True:
        u = H.vcycle(k, u, F)
        _ = np.linalg.norm(H.residual(k, u, F))
        cycles += 1
        el = time.perf_counter() - t0
        progress(f"CPU oracle, whole 127^2 x 256 workload: {cycles} V-cycles in {el:.1f} s")
        if (el > budget_s and cycles >= 2) or cycles >= 20:
            break
    return {"value": H.fine.dof * cycles / el, "unit": "DoF*V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole 2-D n={n} N={N} p_t={pt} workload ({H.fine.dof} DoF, {H.fine.L.nnz} nonzeros), "
                      f"{cycles} V-cycles + residual norm each, {el:.1f} s; hierarchy, assembly and LU "
                      f"factorisations {setup:.1f} s excluded; one thread",
            "host_cpus_available": len(os.sched_getaffinity(0))}


TRANSFORM_NAMES = ["default", "lds", "register", "register_twice_folded", "slab_resident",
                   "twice_folded_residual_fused", "x_mode_slab_resident", "x_mode_slab_resident_residual_fused"]


def tuned_levels(S, tuning):
    """Per-level kernel families the autotuner picked (all but the coarsest level)."""
    if tuning is None:
        return None
    return [{"level": k, "n": S.levels[k]["n"], "N": S.levels[k]["N"], "small_step": bool(t[0]),
             "transform": TRANSFORM_NAMES[t[1]], "step_ms": round(t[2], 4)}
            for k, t in enumerate(tuning[:-1])]


def measured_traffic(workload_name, kind):
    """HBM bytes per fine-level launch of the kernel of `kind` from the
    committed rocprofv3 counter record of the workload (FETCH_SIZE /
    WRITE_SIZE runs, scaled by a device copy of known size), or None when
    the record has no entry for that kind or the kernel's source file changed
    since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    for ent in rec.get("kernels", []):
        if ent.get("kind") != kind:
            continue
        src = os.path.join(ROOT, ent["source"])
        if not os.path.exists(src):
            return None
        with open(src, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != ent["source_sha256"]:
                return None
        return ent
    return None


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


# Algorithmic HBM bytes per value of each fine-level kernel kind (element size
# e): the residual reads u and F and writes r (the neighbour slab's values come
# from cache); a transform pass reads and writes one vector; the last inverse
# pass of a smoothing step also reads the old iterate (u += omega x); the
# residual + restriction reads u and F and writes the coarse vector, 2^-(d+1)
# values per fine value (added in kernel_bytes).
KIND_BYTES = {"residual": 3, "resid_x": 3, "pass_fwd": 2, "pass_fwd_y": 2, "fused": 2, "pass_inv_y": 2,
              "pass_inv": 3, "resid_restrict": 2}
KIND_NAMES = {"residual": "residual r = F - L u", "resid_x": "residual fused with the forward x pass",
              "resid_restrict": "residual + full restriction F_c = P^T (F - L u)",
              "pass_fwd": "forward sine pass along x", "pass_fwd_y": "forward sine pass along y",
              "fused": "forward pass + per-mode time solve + inverse pass along the slowest axis",
              "pass_inv_y": "inverse sine pass along y", "pass_inv": "inverse sine pass along x + update u += omega x"}
TRANSFORM_KINDS = ("pass_fwd", "pass_fwd_y", "fused", "pass_inv_y", "pass_inv", "resid_x")


def kind_passes(kind, xslab):
    """Transform passes per value of a kernel kind: the fused kind runs a
    forward and an inverse pass along the slowest axis, or, for the
    x-mode-major slab solve of a 3-D level, forward and inverse passes along y
    and z; the residual fused with the x pass runs one."""
    if kind == "fused":
        return 4 if xslab else 2
    return 1


def executed_flops_per_value(kind, n, twice, xslab=False):
    """Matrix-core flops the folded kernels execute per value: a twice-folded
    pass runs four (h/2) x (h/2) products per line of n values (h = (n+1)/2),
    a once-folded one two h x h products.  The dense sine transform would need
    2 n per pass."""
    per_pass = 2.0 * ((n + 1) / 2) ** 2 / n if twice else 2.0 * 2 * ((n + 1) / 2) ** 2 / n
    return per_pass * kind_passes(kind, xslab)


def kernel_bytes(kind, d):
    """Algorithmic bytes per fine value and element byte of a kernel kind."""
    return KIND_BYTES[kind] + (0.5 ** (d + 1) if kind == "resid_restrict" else 0.0)


def kernel_table(prof, steps, nvals, n, elem, twice, mfma_peak, d, xslab=False):
    """Per-kind fine-level rows: average launch, algorithmic HBM bytes and rate,
    and for the transform kinds the executed matrix-core rate (and, apart, the
    dense-equivalent rate)."""
    table = {}
    for k in KIND_BYTES:
        v = prof.get(k)
        if not v or not v["fine_launches"]:
            continue
        avg = v["fine_ms_total"] / v["fine_launches"]
        by = kernel_bytes(k, d) * elem * nvals
        row = {"kernel": KIND_NAMES[k], "avg_launch_ms": avg, "launches": v["fine_launches"],
               "ms_per_step": v["fine_ms_total"] / steps, "bytes_per_launch": by,
               "hbm_gbs": by / (avg * 1e-3) / 1e9}
        row["hbm_frac"] = row["hbm_gbs"] / HBM_PEAK_GBS
        if k in TRANSFORM_KINDS:
            ex = executed_flops_per_value(k, n, twice, xslab) * nvals
            dense = 2.0 * n * nvals * kind_passes(k, xslab)
            row["executed_mfma_tflops"] = ex / (avg * 1e-3) / 1e12
            row["executed_mfma_frac"] = row["executed_mfma_tflops"] / mfma_peak
            row["dense_equivalent_tflops"] = dense / (avg * 1e-3) / 1e12
        table[k] = row
    return table


def profile_kinds(stmg, S, run):
    """run() under the library's per-launch event profiling; per-kind totals (all
    levels) and fine-level totals."""
    S.profile_start()
    run()
    import torch
    torch.cuda.synchronize()
    prof = {}
    for k in stmg.PROF_KINDS:
        tot, cnt = S.profile_read(k, level=-1)
        tot0, cnt0 = S.profile_read(k, level=0)
        prof[k] = {"ms_total": tot, "launches": cnt, "fine_ms_total": tot0, "fine_launches": cnt0}
    S.profile_stop()
    return prof


def measure_batched(stmg, torch, args, dev):
    """The batched workload: 2-D Q1 255^2 x 512 slabs, p_t = 2, 64 right-hand
    sides (f ~ U[-1,1], u0 = 16-mode sine series each) through one V-cycle in
    FP32 with hipGraph replay; kernel families and launch shapes per level from
    the autotuner.  Throughput, cycles and time to a 1e-4 relative residual
    for every right-hand side (FP32 residuals of this operator stall near
    1e-5), the tuned shapes and the fine-level kernel table with 4-byte
    values."""
    import numpy as np

    from paper_1411_0519_amd import workloads
    w = workloads.WORKLOADS[4]
    d, n, N, pt, b = w["dim"], w["n"], w["N"], w["pt"], w["batch"]
    nx = n ** d
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev, precision="fp32")
    fdev = torch.empty(b * N * nx, dtype=torch.float32, device=dev)
    it, u0_fn = workloads.make_streamed(**w)
    for i, fb in enumerate(it):
        fdev[i * N * nx:(i + 1) * N * nx].copy_(torch.from_numpy(fb.astype(np.float32).ravel()))
    u0 = torch.from_numpy(u0_fn().astype(np.float32).ravel()).to(dev)
    F = S.rhs(fdev, u0)
    del fdev, u0
    progress(f"{w['name']}: data ready")
    tuning = None if args.no_autotune else S.autotune()
    progress(f"{w['name']}: autotuned")
    shapes = [dict(level=k, **S.level_shape(k)) for k in range(S.nlev - 1)]
    dof = S.level_dof(0)
    steps = max(3, args.steps // 4)
    u = torch.zeros_like(F)
    if not args.no_graph:
        S.set_graph(True)
    S.solve(F, u=u, rtol=0.0, maxit=1, raise_on_noconv=False)
    torch.cuda.synchronize()
    u.zero_()
    t0 = time.perf_counter()
    S.solve(F, u=u, rtol=0.0, maxit=steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    progress(f"{w['name']}: {steps} timed V-cycles, {1e3 * el / steps:.1f} ms each")
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, hist = S.solve(F, u=u, rtol=1e-4, maxit=30, raise_on_noconv=False)
    torch.cuda.synchronize()
    tsol = time.perf_counter() - t0
    S.set_graph(False)
    u.zero_()
    prof = profile_kinds(stmg, S, lambda: S.solve(F, u=u, rtol=0.0, maxit=2, raise_on_noconv=False))
    L0 = S.levels[0]
    impl0 = 0 if tuning is None else tuning[0][1]
    twice = impl0 in (0, 3, 5, 6, 7) and L0["n"] in (63, 127, 255)
    nvals = b * L0["N"] * S.nt * L0["n"] ** d
    table = kernel_table(prof, 2, nvals, L0["n"], 4, twice, FP32_MFMA_PEAK_TFS, d)
    dom = max(table, key=lambda k: table[k]["ms_per_step"])
    row = table[dom]
    out = {"workload": f"{w['name']}: {d}-D Q1 {n}^{d} interior, N={N} slabs, DG p_t={pt}, batch {b} right-hand "
                       f"sides in one V-cycle, FP32, hipGraph replay, omega=1/2, nu1=nu2=2, schedule {S.schedule}",
           "dof": dof, "value": dof * steps / el, "unit": "DoF*V-cycles/s", "ms_per_step": 1e3 * el / steps,
           "steps": steps, "time_to_1e-4_s": tsol, "cycles_to_1e-4": its,
           "final_relres_max_over_rhs": max(hist[-1]), "autotuned_levels": tuned_levels(S, tuning),
           "autotuned_shapes": shapes,
           "roofline": {"kernel": row["kernel"] + ", fine level", "kind": dom, "bound": "hbm",
                        "achieved": row["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": row["hbm_frac"],
                        "avg_launch_ms": row["avg_launch_ms"], "bytes_per_launch": row["bytes_per_launch"]},
           "fine_level_kernels": table,
           "kernel_breakdown_ms_per_step": {k: v["ms_total"] / 2 for k, v in prof.items() if v["launches"]}}
    S.close()
    return out


def measure_workload(stmg, torch, idx, args, dev, steps, mixed=True):
    """Throughput, time to 1e-10 (FP64 and the two mixed solves) and the
    per-kind fine-level kernel table of one workload."""
    from paper_1411_0519_amd import workloads
    w = workloads.WORKLOADS[idx]
    d, n, N, pt, b = w["dim"], w["n"], w["N"], w["pt"], w["batch"]
    _, f, u0 = workloads.workload(idx)
    out = {}
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev)
    F = S.rhs(torch.from_numpy(f.ravel()).to(dev), torch.from_numpy(u0.ravel()).to(dev))
    del f, u0
    dof = S.level_dof(0)
    u = torch.zeros(dof, dtype=torch.float64, device=dev)
    tuning = None if args.no_autotune else S.autotune()
    if not args.no_graph:
        S.set_graph(True)
    S.solve(F, u=u, rtol=0.0, maxit=max(args.warmup, 1), raise_on_noconv=False)   # warmup (records the graph)
    torch.cuda.synchronize()
    u.zero_()
    t0 = time.perf_counter()
    _, its, _ = S.solve(F, u=u, rtol=0.0, maxit=steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert its == steps
    progress(f"{w['name']}: {steps} timed V-cycles, {1e3 * el / steps:.3f} ms each")
    out.update(value=dof * steps / el, ms_per_step=1e3 * el / steps, dof=dof, schedule=S.schedule, levels=S.nlev,
               autotuned_levels=tuned_levels(S, tuning), name=w["name"],
               workload=f"{w['name']}: {d}-D Q1 {n}^{d} interior, N={N} slabs, DG p_t={pt}, batch {b}, FP64, "
                        f"omega=1/2, nu1=nu2=2, schedule {S.schedule}")
    if args.only_timed:
        S.close()
        return out
    # time to a 1e-10 relative residual, FP64 (setup excluded)
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u64, its64, hist64 = S.solve(F, u=u, rtol=1e-10, maxit=100)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    ttt = {"fp64_s": t64, "fp64_cycles": its64, "fp64_final_relres": hist64[-1][0]}
    progress(f"{w['name']}: FP64 solve to 1e-10 in {its64} cycles, {t64:.3f} s")
    # profiled pass (eager, HIP events around every launch on the launch stream)
    S.set_graph(False)
    u2 = torch.zeros_like(u)
    S.solve(F, u=u2, rtol=0.0, maxit=2, raise_on_noconv=False)
    prof = profile_kinds(stmg, S, lambda: S.solve(F, u=u2, rtol=0.0, maxit=steps, raise_on_noconv=False))
    del u2
    out["kernel_breakdown_ms_per_step"] = {k: v["ms_total"] / steps for k, v in prof.items() if v["launches"]}
    out["profiled_ms_per_step"] = sum(v["ms_total"] for v in prof.values()) / steps
    L0 = S.levels[0]
    nvals = b * L0["N"] * S.nt * L0["n"] ** d
    impl0 = 0 if tuning is None else tuning[0][1]
    twice = impl0 in (0, 3, 5, 6, 7) and L0["n"] in (63, 127)
    xslab = impl0 in (6, 7)
    table = kernel_table(prof, steps, nvals, L0["n"], 8, twice, FP64_MFMA_PEAK_TFS, d, xslab)
    for k, row in table.items():   # HBM bytes by counters where the committed record covers the kernel
        rec = measured_traffic(w["name"], k)
        if rec is not None:
            row["counter_read_write_bytes"] = [rec["fetch_bytes_per_launch"], rec["write_bytes_per_launch"]]
    out["fine_level_kernels"] = table
    out["fine_level_values"] = nvals
    out["dim"] = d
    out["twice_folded"] = twice
    if not args.no_graph:
        S.set_graph(True)
    if mixed:
        for prec, key in (("mixed", "mixed"), ("mixed_bf16", "mixed_bf16")):
            M = stmg.Solver(d, n, N, pt=pt, batch=b, device=dev, precision=prec)
            tm_tuning = None if args.no_autotune else M.autotune()
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
            err = (torch.linalg.vector_norm(um - u64) / torch.linalg.vector_norm(u64)).item()
            ttt.update({f"{key}_s": tm, f"{key}_cycles": itsm, f"speedup_{key}_vs_fp64": t64 / tm,
                        f"{key}_rel_error_vs_fp64": err, f"{key}_final_relres": histm[-1][0]})
            progress(f"{w['name']}: {prec} solve to 1e-10 in {itsm} cycles, {tm:.3f} s")
            if key == "mixed":
                ttt["mixed_inner_levels"] = tuned_levels(S, tm_tuning)
            M.close()
            del um
    out["time_to_1e-10"] = ttt
    out["_solver"], out["_F"], out["_u64"] = S, F, u64
    return out


def roofline_of(m):
    """Roofline object of the fine-level kernel kind with the most time per step."""
    table = m["fine_level_kernels"]
    dom = max(table, key=lambda k: table[k]["ms_per_step"])
    row = table[dom]
    roof = {"kernel": row["kernel"] + ", fine level", "kind": dom, "bound": "hbm", "achieved": row["hbm_gbs"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": row["hbm_frac"], "traffic": None,
            "avg_launch_ms": row["avg_launch_ms"], "launches": row["launches"],
            "bytes_per_launch": row["bytes_per_launch"],
            "bytes_basis": f"{kernel_bytes(dom, m['dim']):g} x 8 B per value x {m['fine_level_values']} values"}
    if "executed_mfma_tflops" in row:
        roof["mfma_executed"] = {"achieved": row["executed_mfma_tflops"], "peak": FP64_MFMA_PEAK_TFS,
                                 "unit": "TFLOP/s", "frac": row["executed_mfma_frac"]}
        roof["dense_equivalent_tflops"] = row["dense_equivalent_tflops"]
    rec = measured_traffic(m["name"], dom)
    if rec is not None:
        roof["traffic"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
        roof["traffic_read_write_bytes"] = [rec["fetch_bytes_per_launch"], rec["write_bytes_per_launch"]]
        roof["traffic_kernel"] = rec["kernel"]
    return roof


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (one process, one device); multi-GPU runs are not supported, use --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1411_0519_amd import stmg

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
    stream = torch.cuda.Stream(device=dev)
    if args.only_batched:
        with torch.cuda.stream(stream):
            print(json.dumps({"batched": measure_batched(stmg, torch, args, dev)}))
        return
    with torch.cuda.stream(stream):
        head = measure_workload(stmg, torch, args.workload, args, dev, args.steps)
        if args.only_timed:
            print(json.dumps({"metric": "space-time DoF*V-cycles/s", "value": head["value"],
                              "ms_per_step": head["ms_per_step"], "workload": head["workload"]}))
            return
        S, F, u64 = head.pop("_solver"), head.pop("_F"), head.pop("_u64")
        S.close()
        del S, F, u64
        torch.cuda.empty_cache()
        secondary = None
        inexact = None
        if not args.no_secondary and args.workload != 2:
            sec = measure_workload(stmg, torch, 2, args, dev, max(args.steps, 20))
            S2, F2, u2 = sec.pop("_solver"), sec.pop("_F"), sec.pop("_u64")
            sec["roofline"] = roofline_of(sec)
            if not args.no_inexact:
                from paper_1411_0519_amd import workloads
                w2 = workloads.WORKLOADS[2]
                inexact = measure_inexact(stmg, torch, 2, w2["n"], w2["N"], w2["pt"], 1, F2, u2, dev, args)
            S2.close()
            del S2, F2, u2
            secondary = sec
        batched = None
        if not args.no_batched:
            batched = measure_batched(stmg, torch, args, dev)
            torch.cuda.empty_cache()
        p1_mesh = None
        if not args.no_mesh:
            p1_mesh = measure_p1(stmg, torch, dev, args)
            progress("P1 mesh workload done")

    roof = roofline_of(head)
    out = {
        "metric": "space-time DoF*V-cycles/s (+ time-to-1e-10, mixed vs FP64)",
        "value": head["value"],
        "unit": "DoF*V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "dof": head["dof"], "levels": head["levels"],
                   "graph": not args.no_graph, "autotuned_levels": head["autotuned_levels"]},
        "time_to_1e-10": head["time_to_1e-10"],
        "roofline": roof,
        "fine_level_kernels": head["fine_level_kernels"],
        "kernel_breakdown_ms_per_step": head["kernel_breakdown_ms_per_step"],
        "profiled_ms_per_step": head["profiled_ms_per_step"],
    }
    if secondary is not None:
        for k in ("autotuned_levels", "dof", "levels", "schedule", "name"):
            secondary.pop(k, None)
        out["secondary_2d_127"] = secondary
    if inexact is not None:
        out["inexact_smoother_2d_127"] = inexact
    if batched is not None:
        out["batched_2d_255_b64_fp32"] = batched
    if p1_mesh is not None:
        out["p1_mesh"] = p1_mesh
    if args.cpu_full_w2:
        progress("CPU oracle on the whole 127^2 x 256 workload")
        cf = cpu_full_w2()
        if "secondary_2d_127" in out:
            out["secondary_2d_127"]["cpu_baseline_full_size"] = cf
            out["secondary_2d_127"]["gpu_over_cpu_full_size"] = out["secondary_2d_127"]["value"] / cf["value"]
        else:
            out["cpu_baseline_full_2d_127"] = cf
    if not args.no_cpu_baseline:
        progress("CPU oracle sample")
        cb = cpu_baseline()
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = head["value"] / cb["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
