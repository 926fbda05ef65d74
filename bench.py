"""Benchmark: FGMRES + MGR time-to-1e-8 on one MI355X.

Workload: the hybrid mimetic single-phase system on a 64^3 hex grid (cell
pressures + face multipliers, 1,060,864 unknowns, 12,070,912 nonzeros,
lognormal diagonal permeability with sigma = 2), one MGR level eliminating the
cells exactly (F = cells, Jacobi), AMG V-cycle on the face system, FGMRES(50)
to a relative residual of 1e-8.  One step = MGR/AMG setup + solve, with the
matrix already resident in HBM.  The FP64 apply is the headline; the same steps
with the FP32 MGR apply are reported beside it (FP32-vs-FP64 speedup).

Prints one JSON line (stdout).  Progress goes to stderr.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(n, nnz, s=8):
    """Algorithmic bytes of one CSR SpMV y = A x: values + column indices +
    row pointers once, x once, y once."""
    return nnz * (s + 4) + 4 * (n + 1) + 2 * n * 8


def time_kernel(fn, stream, reps, flush_buf):
    """Average duration of fn() (one kernel launch) with HIP events on `stream`,
    evicting the 256 MB Infinity Cache between launches by reading a 512 MB
    buffer (a read leaves no dirty lines whose write-back would land in the
    timed launch)."""
    import torch
    ts = []
    for _ in range(reps):
        flush_buf.sum()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return statistics.mean(ts), ts


def bsr_spmv_bytes(b, nbr, nnzb, s=8):
    """Algorithmic bytes of one block-CSR SpMV: b x b value blocks + block column
    indices + block row pointers once, x once, y once."""
    n = b * nbr
    return nnzb * (b * b * s + 4) + 4 * (nbr + 1) + 2 * n * 8


def row_scaled(sysd, scale=0.05, seed=0, rows_field=None):
    """New values on the same pattern, as between two Newton solves: scalar rows
    scaled by 1 + U[-scale, scale] (only rows of field rows_field, if given)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    b, nb = sysd["b"], len(sysd["ci"])
    f = 1.0 + rng.uniform(-scale, scale, sysd["n"])
    if rows_field is not None:
        f[sysd["field"] != rows_field] = 1.0
    brow = np.repeat(np.arange(len(sysd["rp"]) - 1), np.diff(sysd["rp"]))
    rows = brow[:, None] * b + np.arange(b)[None, :]
    return (sysd["vals"].reshape(nb, b, b) * f[rows][:, :, None]).reshape(-1)


def time_reuse(solver, sysd, vals2, keep, reps=3):
    """mgr_update_values with new values (setup reuse), then a solve."""
    import torch
    v2 = torch.tensor(vals2, device="cuda")
    rhs = torch.tensor(sysd["rhs"], device="cuda")
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.update_values(v2, keep_frelax_amg=keep)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    _, [info] = solver.solve(rhs)
    torch.cuda.synchronize()
    return {"update_s": round(statistics.mean(ts), 6), "solve_s": round(time.perf_counter() - t0, 6),
            "iterations": info.iterations, "rel_res_true": info.rel_res_true,
            "kept": "F-relaxation AMG hierarchies whole" if keep else "AMG C/F splits and interpolation"}


def kernel_traffic(name):
    """HBM bytes per launch of `name` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None if the summary
    is missing or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2101_11649_amd", "csrc", "k_apply.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("k_apply.hip sha256") != sha or "traffic bytes per launch" not in fields:
        return None
    return int(float(fields["traffic bytes per launch"]))


def run_steps(P, s, vals, rhs, precision, steps, warmup, **opts):
    import torch
    solver = P.Solver(s["b"], s["rp"], s["ci"], vals, s["field"], s["levels"], precision=precision, **opts)
    stream = torch.cuda.current_stream()
    rec = []
    X = info = None
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.setup(vals)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X, [info] = solver.solve(rhs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if it >= warmup:
            rec.append((t1 - t0, t2 - t1, info.iterations, info.rel_res_true))
        log(f"  fp{precision} step {it} ({'warmup' if it < warmup else 'timed'}): setup {t1 - t0:.4f} s, "
            f"solve {t2 - t1:.4f} s, iters {info.iterations}, true rel res {info.rel_res_true:.2e}")
    return solver, rec, X, info, stream


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--grid", type=int, default=64, help="grid size per axis of the mimetic system")
    ap.add_argument("--comp-steps", type=int, default=2,
                    help="timed steps of the secondary compositional workload (0 = skip)")
    ap.add_argument("--tpfa-steps", type=int, default=2,
                    help="timed steps of the MGR_P vs MGR_Pi comparison on the TPFA mimetic system (0 = skip)")
    ap.add_argument("--interp-steps", type=int, default=2,
                    help="timed steps of the mimetic system with extended+i AMG interpolation (0 = skip)")
    ap.add_argument("--frac-steps", type=int, default=1,
                    help="timed steps of the secondary fracturing workload (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the solver runs on a single device and "
              f"has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2101_11649_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    g = args.grid
    log(f"generating hybrid mimetic {g}^3 ...")
    s = W.hybrid_mimetic(g, g, g, seed=1)
    n, nnz = s["n"], len(s["ci"])
    log(f"n = {n}, nnz = {nnz}")
    vals = torch.tensor(s["vals"], device="cuda")
    rhs = torch.tensor(s["rhs"], device="cuda")
    torch.cuda.synchronize()

    # ---- FP64 apply (headline) and FP32 apply, K timed steps each
    solver, rec64, X64, info64, stream = run_steps(P, s, vals, rhs, 64, args.steps, args.warmup)
    solver32, rec32, X32, info32, _ = run_steps(P, s, vals, rhs, 32, args.steps, args.warmup)

    reuse64 = time_reuse(solver, s, row_scaled(s, seed=11), False)
    tot64 = [a + b for a, b, _, _ in rec64]
    tot32 = [a + b for a, b, _, _ in rec32]
    value = statistics.mean(tot64)

    # ---- roofline of the dominant kernel: the FGMRES CSR SpMV on A (FP64)
    flush = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    # calibration launch for the byte counters: a plain 512 MB device copy
    calib = torch.empty_like(flush)
    calib.copy_(flush)
    xv = torch.randn(n, dtype=torch.float64, device="cuda")
    yv = torch.empty_like(xv)
    lib = P.lib()
    import ctypes
    fn = lambda: lib.mgr_matvec(solver._h, 0, ctypes.c_void_p(xv.data_ptr()), ctypes.c_void_p(yv.data_ptr()))
    fn()
    t_spmv, _ = time_kernel(fn, stream, 50, flush)
    # the library's scalar operator leaves out the exact zeros of the input
    # (diagonal kept): its entries are what the matvec reads
    rows = np.repeat(np.arange(n), np.diff(s["rp"]))
    nnz_op = int(np.count_nonzero((s["vals"] != 0.0) | (s["ci"] == rows)))
    nbytes = spmv_bytes(n, nnz_op)
    achieved = nbytes / t_spmv / 1e9

    # per-apply FP64 vs FP32 (cache flushed between launches; an apply is several kernels)
    v = torch.randn(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(v)
    ap64 = lambda: lib.mgr_apply(solver._h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(z.data_ptr()))
    ap32 = lambda: lib.mgr_apply(solver32._h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(z.data_ptr()))
    ap64(); ap32()
    t_ap64, _ = time_kernel(ap64, stream, 20, flush)
    t_ap32, _ = time_kernel(ap32, stream, 20, flush)

    def secondary(sysd, steps, mgr_desc, apply_reps, roof=None, reuse=None):
        """FP64 and FP32 apply on one more workload: time to 1e-8, per-apply time
        (cache flushed), and optionally the roofline of its FGMRES matvec."""
        vv_ = torch.tensor(sysd["vals"], device="cuda")
        bb_ = torch.tensor(sysd["rhs"], device="cuda")
        o = sysd.get("solver_opts", {})
        s64, r64, _, _, _ = run_steps(P, sysd, vv_, bb_, 64, steps, 1, **o)
        s32, r32, _, _, _ = run_steps(P, sysd, vv_, bb_, 32, steps, 1, **o)
        t64 = statistics.mean(a + b for a, b, _, _ in r64)
        t32 = statistics.mean(a + b for a, b, _, _ in r32)
        vin = torch.randn(sysd["n"], dtype=torch.float64, device="cuda")
        zout = torch.empty_like(vin)
        a64 = lambda: lib.mgr_apply(s64._h, ctypes.c_void_p(vin.data_ptr()), ctypes.c_void_p(zout.data_ptr()))
        a32 = lambda: lib.mgr_apply(s32._h, ctypes.c_void_p(vin.data_ptr()), ctypes.c_void_p(zout.data_ptr()))
        a64(); a32()
        ta64, _ = time_kernel(a64, stream, apply_reps, flush)
        ta32, _ = time_kernel(a32, stream, apply_reps, flush)
        out_ = {"workload": sysd["name"], "n": sysd["n"], "nnz": int(len(sysd["ci"]) * sysd["b"] ** 2),
                "mgr": mgr_desc}
        for key, r, ta in (("fp64", r64, ta64), ("fp32", r32, ta32)):
            out_[key] = {"time_to_tol_s": round(statistics.mean(a + b for a, b, _, _ in r), 6),
                         "setup_s": round(statistics.mean(a for a, _, _, _ in r), 6),
                         "solve_s": round(statistics.mean(b for _, b, _, _ in r), 6), "iterations": r[-1][2],
                         "rel_res_true": r[-1][3], "apply_ms": round(1e3 * ta, 4)}
        out_["speedup_time_to_tol"] = round(t64 / t32, 4)
        out_["speedup_per_apply"] = round(ta64 / ta32, 4)
        if roof:
            # the FGMRES matvec on the block-CSR input, FP64
            mv = lambda: lib.mgr_matvec(s64._h, 0, ctypes.c_void_p(vin.data_ptr()), ctypes.c_void_p(zout.data_ptr()))
            mv()
            t_mv, _ = time_kernel(mv, stream, 20, flush)
            bb = bsr_spmv_bytes(sysd["b"], len(sysd["rp"]) - 1, len(sysd["ci"]))
            out_["roofline"] = {"kernel": roof[0], "bound": "hbm", "achieved": round(bb / t_mv / 1e9, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(bb / t_mv / 1e9 / HBM_PEAK_GBS, 4), "traffic": kernel_traffic(roof[1]),
                                "bytes_per_launch": bb, "avg_launch_us": round(1e6 * t_mv, 2)}
        if reuse is not None:
            # setup reuse after a value change (rows of field reuse[0] scaled; reuse[1] = keep flag)
            out_["setup_reuse"] = time_reuse(s64, sysd, row_scaled(sysd, seed=11, rows_field=reuse[0]), reuse[1])
        s64.close()
        s32.close()
        return out_

    # ---- secondary: the compositional system with wells (128x128x64, 4 unknowns per
    # cell, 16 wells; 2-level MGR), FP64 vs FP32 apply inside FP64 FGMRES; its block
    # SpMV (about 1 GB, four times the Infinity Cache) is the HBM roofline case
    comp = comp4 = frac = None
    if args.comp_steps > 0:
        log("generating compositional 128x128x64 + 16 wells ...")
        comp = secondary(W.compositional_wells(seed=2), args.comp_steps,
                         "L1 F = components (block-Jacobi), L2 F = wells (Jacobi), coarse pressure AMG", 10,
                         ("k_bsr_spmv<4, 8> (FGMRES matvec y = A x, 4 x 4 block CSR, FP64)",
                          "k_bsr_spmv_compositional.md"))
        # the paper's own four-level order on the same grid: rho_2, rho_1, p (AMG
        # F-relaxation), then the well system (zero diagonals) as the coarse grid
        log("generating compositional 4-level 128x128x64 + 16 wells ...")
        comp4 = secondary(W.compositional_4level(seed=4), args.comp_steps,
                          "L1 F = rho_2 (Jacobi, exact), L2 F = rho_1 (Jacobi), L3 F = p (AMG V-cycle), "
                          "coarse = wells (direct)", 10)
    # ---- secondary: the two reductions of the hybrid system (Sec. 3.1) on its TPFA
    # variant, where both eliminate a diagonal block: MGR_P (F = cells, faces to
    # AMG) against MGR_Pi (F = faces, the 7-point cell Schur complement to AMG)
    tpfa = None
    if args.tpfa_steps > 0:
        tpfa = {"workload": f"hybrid_mimetic_tpfa_{g}x{g}x{g}", "apply": "fp64"}
        for red, key in (("p", "mgr_p"), ("pi", "mgr_pi")):
            log(f"generating hybrid mimetic TPFA {g}^3, reduction {key} ...")
            st = W.hybrid_mimetic(g, g, g, seed=1, consistent=False, reduction=red)
            vt = torch.tensor(st["vals"], device="cuda")
            bt = torch.tensor(st["rhs"], device="cuda")
            sv, rt, _, _, _ = run_steps(P, st, vt, bt, 64, args.tpfa_steps, 1)
            hi = sv.info()
            tpfa[key] = {"time_to_tol_s": round(statistics.mean(a + b for a, b, _, _ in rt), 6),
                         "setup_s": round(statistics.mean(a for a, _, _, _ in rt), 6),
                         "solve_s": round(statistics.mean(b for _, b, _, _ in rt), 6),
                         "iterations": rt[-1][2], "rel_res_true": rt[-1][3],
                         "coarse_n": hi["amg_levels"][0][0], "coarse_nnz": hi["amg_levels"][0][1],
                         "amg_levels": len(hi["amg_levels"])}
            sv.close()
        tpfa["speedup_pi_over_p"] = round(tpfa["mgr_p"]["time_to_tol_s"] / tpfa["mgr_pi"]["time_to_tol_s"], 4)

    # ---- secondary: the same mimetic workload with extended+i (distance-two) AMG
    # interpolation instead of direct interpolation
    ext = None
    if args.interp_steps > 0:
        log(f"mimetic {g}^3 with extended+i interpolation ...")
        se, re_, _, _, _ = run_steps(P, s, vals, rhs, 64, args.interp_steps, 1, interp="ext+i")
        hi, hd = se.info(), solver.info()
        ext = {"workload": f"hybrid_mimetic_consistent_{g}x{g}x{g}", "apply": "fp64",
               "direct": {"time_to_tol_s": round(value, 6), "iterations": rec64[-1][2],
                          "amg_nnz": int(sum(a[1] for a in hd["amg_levels"]))},
               "ext+i": {"time_to_tol_s": round(statistics.mean(a + b for a, b, _, _ in re_), 6),
                         "setup_s": round(statistics.mean(a for a, _, _, _ in re_), 6),
                         "solve_s": round(statistics.mean(b for _, b, _, _ in re_), 6),
                         "iterations": re_[-1][2], "rel_res_true": re_[-1][3],
                         "amg_nnz": int(sum(a[1] for a in hi["amg_levels"]))}}
        se.close()

    # ---- secondary: the fracturing system (Q1 elasticity on 96^3 nodes + a 96 x 96
    # planar fracture; MGR_U with an unknown-based AMG V-cycle as F-relaxation)
    if args.frac_steps > 0:
        log("generating fracturing 96^3 ...")
        frac = secondary(W.fracturing(96, seed=3), args.frac_steps,
                         "F = displacements (unknown-based AMG V(2,2) F-relaxation), C = fracture pressures -> AMG",
                         5, reuse=(3, True))

    # ---- FP64 oracle on the machine's host cores (bounded sample: one full setup + solve of this workload)
    cpu = None
    x_err64 = x_err32 = None
    if not args.no_cpu_baseline:
        import oracle as O
        log("oracle (CPU, single thread): one setup + solve of the same workload ...")
        t0 = time.perf_counter()
        om = O.MGR(s["b"], s["rp"], s["ci"], s["vals"], s["field"], [O.LevelOpts(**l) for l in s["levels"]])
        t1 = time.perf_counter()
        xo, io = om.solve(s["rhs"])
        t2 = time.perf_counter()
        log(f"  oracle setup {t1 - t0:.2f} s, solve {t2 - t1:.2f} s, iters {io.iterations}")
        cpu = {"value": round(t2 - t0, 4), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"one full setup + FGMRES solve to 1e-8 of the {g}^3 mimetic system "
                         f"(setup {t1 - t0:.2f} s, solve {t2 - t1:.2f} s, {io.iterations} iterations)"}
        nx = np.linalg.norm(xo)
        x_err64 = float(np.linalg.norm(X64.cpu().numpy() - xo) / nx)
        x_err32 = float(np.linalg.norm(X32.cpu().numpy() - xo) / nx)

    out = {
        "metric": "FGMRES+MGR time-to-1e-8 (s), HBM GB/s; FP32-vs-FP64 apply speedup",
        "value": round(value, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * value, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hybrid_mimetic_consistent_{g}x{g}x{g}", "n": n, "nnz": nnz, "nnz_operator": nnz_op,
                   "mgr": "1 level, F = cells (Jacobi), C = faces -> AMG V(1,1)", "rtol": 1e-8,
                   "restart": 50},
        "setup_s": round(statistics.mean(a for a, _, _, _ in rec64), 6),
        "solve_s": round(statistics.mean(b for _, b, _, _ in rec64), 6),
        "iterations": rec64[-1][2],
        "rel_res_true": rec64[-1][3],
        "x_rel_err_vs_oracle": x_err64,
        "setup_reuse": reuse64,
        "fp32_apply": {
            "time_to_tol_s": round(statistics.mean(tot32), 6),
            "setup_s": round(statistics.mean(a for a, _, _, _ in rec32), 6),
            "solve_s": round(statistics.mean(b for _, b, _, _ in rec32), 6),
            "iterations": rec32[-1][2],
            "rel_res_true": rec32[-1][3],
            "x_rel_err_vs_oracle": x_err32,
            "speedup_time_to_tol": round(value / statistics.mean(tot32), 4),
            "apply_ms_fp64": round(1e3 * t_ap64, 4),
            "apply_ms_fp32": round(1e3 * t_ap32, 4),
            "speedup_per_apply": round(t_ap64 / t_ap32, 4),
        },
        "roofline": {"kernel": "k_spmv_ell<double, 1, SpmvOp> (FGMRES matvec y = A x, sliced ELL copy of the CSR, FP64, "
                               f"{nnz_op} entries)",
                     "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": kernel_traffic("k_spmv_fgmres_mimetic64.md"),
                     "bytes_per_launch": nbytes, "avg_launch_us": round(1e6 * t_spmv, 2)},
        "secondary_compositional": comp,
        "secondary_compositional_4level": comp4,
        "secondary_fracturing": frac,
        "secondary_mimetic_tpfa_reductions": tpfa,
        "secondary_mimetic_ext_interp": ext,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    solver.close()
    solver32.close()


if __name__ == "__main__":
    main()
