"""Benchmark: FGMRES + MGR time-to-1e-8 on one MI355X.

Workload (headline): the compositional-style system with wells on a
128 x 128 x 64 grid, 4 unknowns per cell (pressure + 3 component densities) in
4 x 4 blocks plus 16 wells (4,194,368 unknowns, 116,391,936 stored block
values), lognormal permeability; MGR in two levels (components by
block-Jacobi, then wells by Jacobi), AMG V-cycle on the pressure system,
FGMRES(50) to a relative residual of 1e-8.  One step = MGR/AMG setup + solve,
with the matrix already resident in HBM.  The FP64 apply is the headline; the
same steps with the FP32 MGR apply are reported beside it (FP32-vs-FP64
speedup).  The other workloads (hybrid mimetic 64^3, the paper's four-level
compositional order, fracturing with MGR_U and MGR_P, MGR_P vs MGR_Pi on the
TPFA mimetic system) are reported as secondaries.

Prints one JSON line (stdout).  Progress goes to stderr.
"""
import argparse
import json
import os
import statistics
import subprocess
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


def kernel_source_sha256(kernel):
    """sha256 of the text of one kernel in k_apply.hip: from the line that
    declares `__global__ ... kernel(` to the first closing brace in column 0."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2101_11649_amd", "csrc", "k_apply.hip")).read().splitlines(keepends=True)
    for i, line in enumerate(src):
        if "__global__" in line and f" {kernel}(" in line:
            j = i
            while src[j].rstrip("\n") != "}":
                j += 1
            return hashlib.sha256("".join(src[i:j + 1]).encode()).hexdigest()
    return None


def kernel_traffic(name):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None if
    the summary is missing or the kernel's source text changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    kern = fields.get("kernel")
    if not kern or "traffic bytes per launch" not in fields:
        return None
    if fields.get("kernel source sha256") != kernel_source_sha256(kern):
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


def apply_launches(solver, precision, nu_pre=1, nu_post=1, levels=None, smoother="l1-jacobi"):
    """The launches of one forward MGR apply (Algorithm 1, then the AMG V-cycle
    on the coarse system), in order, each with its algorithmic bytes: operator
    values + column indices + row pointers once, every vector it reads or
    writes once.  s = bytes of a value in the apply precision; the apply's
    input and output stay FP64.  One-sweep levels with injection are the fused
    pair R_J / P_J; other levels (one sweep, injection) gather, relax (M, or
    the F-relaxation AMG's V-cycle), restrict with A_CF, interpolate with P_F
    and scatter.  With the hybrid Gauss-Seidel smoother the per-chunk pass
    counts its slot table as stored (padding included), the diagonal in the
    table's layout and its vectors.  None for level options this
    model does not list (several sweeps, Jacobi restriction, ILU(0))."""
    s = 4 if precision == 32 else 8
    info = solver.info()
    mgr, amg = info["mgr_levels"], info["amg_levels"]
    levels = levels or [{}] * len(mgr)
    gs = smoother == "hybrid-gs"
    out = []

    def sp(nr, nnz):
        return nnz * (s + 4) + 4 * (nr + 1)

    def amg_sizes(kind, sub):
        if kind == 1:
            return amg
        sz, k = [], 0
        while True:
            a = solver.export_sizes(2, k, 1, sub)
            if a is None:
                return sz
            sz.append((a[0], a[2]))
            k += 1

    def amg_cycle(kind, sub, lv, k, tag):
        n = lv[k][0]
        last = len(lv) - 1
        if k == last:
            out.append((f"{tag}{k} coarsest GEMV", n * n * s + 2 * n * s))
            return
        if solver.export_sizes(kind, k, 6, sub) is not None:
            out.append((f"{tag}{k} dense cycle GEMV", n * n * s + 2 * n * s))
            return
        nc = lv[k + 1][0]
        g = solver.export_sizes(kind, k, 4, sub)
        if g is not None:
            wq = solver.export_sizes(kind, k, 5, sub)
            out.append((f"{tag}{k} G (composed restriction)", sp(nc, g[2]) + n * s + nc * s))
            amg_cycle(kind, sub, lv, k + 1, tag)
            out.append((f"{tag}{k} [W|Q] (composed smoothing + prolongation)", sp(n, wq[2]) + 2 * n * s + nc * s))
            return
        a = sp(n, lv[k][1])
        p = solver.export_sizes(kind, k, 2, sub)[2]
        if gs:
            def chunk(what, from_zero):
                # slot table (local column byte + value per slot), d in the
                # table layout, r read, x read (not from zero) and written
                per, _, slots = solver.export_sizes(kind, k, what, sub)
                return slots * (1 + s) + per * s + (2 if from_zero else 3) * n * s
            if nu_pre >= 1:
                out.append((f"{tag}{k} Gauss-Seidel chunks (from zero)", chunk(7, True)))
                for _ in range(1, nu_pre):
                    out.append((f"{tag}{k} residual", a + 3 * n * s))
                    out.append((f"{tag}{k} Gauss-Seidel chunks", chunk(7, False)))
                out.append((f"{tag}{k} residual", a + 3 * n * s))
            else:
                out.append((f"{tag}{k} set", n * s))
                out.append((f"{tag}{k} copy", 2 * n * s))
            out.append((f"{tag}{k} restriction", sp(nc, p) + n * s + nc * s))
            amg_cycle(kind, sub, lv, k + 1, tag)
            out.append((f"{tag}{k} prolongation", sp(n, p) + nc * s + 2 * n * s))
            for _ in range(nu_post):
                out.append((f"{tag}{k} residual", a + 3 * n * s))
                out.append((f"{tag}{k} Gauss-Seidel chunks", chunk(8, False)))
            return
        if nu_pre >= 1:
            out.append((f"{tag}{k} pre-smoothing + residual", a + 4 * n * s))
            for _ in range(1, nu_pre):
                out.append((f"{tag}{k} Jacobi sweep", a + 4 * n * s))
                out.append((f"{tag}{k} copy", 2 * n * s))
            if nu_pre > 1:
                out.append((f"{tag}{k} residual", a + 3 * n * s))
        else:
            out.append((f"{tag}{k} set", n * s))
            out.append((f"{tag}{k} copy", 2 * n * s))
        nxt_plain = (k + 2 <= last) and solver.export_sizes(kind, k + 1, 4, sub) is None \
            and solver.export_sizes(kind, k + 1, 6, sub) is None
        if nu_pre >= 1 and nxt_plain:
            out.append((f"{tag}{k} restriction (+ D^-1 b_c)", sp(nc, p) + n * s + 3 * nc * s))
        else:
            out.append((f"{tag}{k} restriction", sp(nc, p) + n * s + nc * s))
        amg_cycle(kind, sub, lv, k + 1, tag)
        out.append((f"{tag}{k} prolongation", sp(n, p) + nc * s + 2 * n * s))
        for _ in range(nu_post):
            out.append((f"{tag}{k} post-smoothing", a + 4 * n * s))

    def mgr_level(l):
        n, nF, nC, _ = mgr[l]
        vs = 8 if l == 0 else s                 # level-0 vectors are the caller's FP64 ones
        lo = levels[l] if l < len(levels) else {}
        if lo.get("sweeps", 1) != 1 or lo.get("restrict", "injection") != "injection":
            return False
        rj = solver.export_sizes(0, l, 6)
        if rj is not None:
            first_plain = len(amg) >= 2 and solver.export_sizes(1, 0, 4) is None \
                and solver.export_sizes(1, 0, 6) is None and nu_pre >= 1 and not gs
            scaled = (l + 1 == len(mgr)) and first_plain
            # the FP32 apply converts the FP64 input once; both transfers then read it in FP32
            conv = l == 0 and s == 4
            xs = s if conv else vs
            if conv:
                out.append((f"MGR{l} input to FP32", n * 8 + n * 4))
            out.append((f"MGR{l} restriction R_J", sp(nC, rj[2]) + n * xs + (3 if scaled else 1) * nC * s))
            if l + 1 < len(mgr):
                if not mgr_level(l + 1):
                    return False
            else:
                amg_cycle(1, -1, amg, 0, "AMG")
            pj = solver.export_sizes(0, l, 7)[2]
            out.append((f"MGR{l} interpolation P_J", sp(n, pj) + nC * s + n * xs + n * vs))
            return True
        fr = lo.get("frelax", "jacobi")
        if fr == "ilu0":
            return False
        out.append((f"MGR{l} gather v_F", 4 * nF + nF * vs + nF * s))
        out.append((f"MGR{l} gather v_C", 4 * nC + nC * vs + nC * s))
        if fr == "amg":
            famg = amg_sizes(2, l)
            amg_cycle(2, l, famg, 0, f"MGR{l}.FAMG")
        else:
            m = solver.export_sizes(0, l, 5)
            out.append((f"MGR{l} F-relaxation M", sp(nF, m[2]) + 2 * nF * s))
        out.append((f"MGR{l} scale z_F = omega t_F", 2 * nF * s))
        acf = solver.export_sizes(0, l, 9)
        out.append((f"MGR{l} restriction A_CF", sp(nC, acf[2]) + nF * s + 2 * nC * s))
        if l + 1 < len(mgr):
            if not mgr_level(l + 1):
                return False
        else:
            amg_cycle(1, -1, amg, 0, "AMG")
        pf = solver.export_sizes(0, l, 2)
        out.append((f"MGR{l} interpolation P_F", sp(nF, pf[2]) + nC * s + 2 * nF * s))
        out.append((f"MGR{l} scatter z_F", 4 * nF + nF * s + nF * vs))
        out.append((f"MGR{l} scatter z_C", 4 * nC + nC * s + nC * vs))
        return True

    if not mgr:
        return None
    if not mgr_level(0):
        return None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mimetic-steps", type=int, default=2,
                    help="timed steps of the hybrid mimetic 64^3 secondary (0 = skip)")
    ap.add_argument("--comp4-steps", type=int, default=2,
                    help="timed steps of the paper's four-level compositional order (0 = skip)")
    ap.add_argument("--tpfa-steps", type=int, default=2,
                    help="timed steps of the MGR_P vs MGR_Pi comparison on the TPFA mimetic system (0 = skip)")
    ap.add_argument("--interp-steps", type=int, default=1,
                    help="timed steps of the mimetic system with extended+i AMG interpolation (0 = skip)")
    ap.add_argument("--frac-steps", type=int, default=1,
                    help="timed steps of the fracturing workload, MGR_U and MGR_P (0 = skip)")
    ap.add_argument("--ilu-steps", type=int, default=1,
                    help="timed steps of the headline system with ILU(0) F-relaxation of the components (0 = skip)")
    ap.add_argument("--frac-variant", default="all", choices=["all", "u", "u_paper_v11", "u_paper_v22", "u_paper_sdc_v11", "u_paper_sdc_v22", "p"],
                    help="run one fracturing variant only (profiling runs); 'all' adds the grid sweep")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the headline workload (profiling runs of the secondaries alone)")
    ap.add_argument("--launch-table", action="store_true",
                    help="add each workload's list of apply launches with their algorithmic bytes (to pair "
                         "with a kernel trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the solver runs on a single device and "
              f"has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import ctypes

    import numpy as np
    import torch

    import paper_2101_11649_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    lib = P.lib()
    stream = torch.cuda.current_stream()
    flush = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    # calibration launch for the byte counters: a plain 512 MB device copy
    calib = torch.empty_like(flush)
    calib.copy_(flush)
    del calib

    def stats(rec):
        return {"time_to_tol_s": round(statistics.mean(a + b for a, b, _, _ in rec), 6),
                "setup_s": round(statistics.mean(a for a, _, _, _ in rec), 6),
                "solve_s": round(statistics.mean(b for _, b, _, _ in rec), 6),
                "iterations": rec[-1][2], "rel_res_true": rec[-1][3]}

    def apply_timing(s64, s32, n, reps):
        """Per-apply FP64 and FP32 time (Infinity Cache flushed between applies) and
        the apply chain's algorithmic bytes and GB/s."""
        vin = torch.randn(n, dtype=torch.float64, device="cuda")
        zout = torch.empty_like(vin)
        a64 = lambda: lib.mgr_apply(s64._h, ctypes.c_void_p(vin.data_ptr()), ctypes.c_void_p(zout.data_ptr()))
        a32 = lambda: lib.mgr_apply(s32._h, ctypes.c_void_p(vin.data_ptr()), ctypes.c_void_p(zout.data_ptr()))
        a64(); a32()
        t64, _ = time_kernel(a64, stream, reps, flush)
        t32, _ = time_kernel(a32, stream, reps, flush)
        o = s64.opts.amg
        res = {"apply_ms_fp64": round(1e3 * t64, 4), "apply_ms_fp32": round(1e3 * t32, 4),
               "speedup_per_apply": round(t64 / t32, 4)}
        sm = "hybrid-gs" if o.smoother == 1 else "l1-jacobi"
        for key, sv, t, prec in (("fp64", s64, t64, 64), ("fp32", s32, t32, 32)):
            la = apply_launches(sv, prec, o.nu_pre, o.nu_post, levels=sv.levels, smoother=sm)
            if la is None:
                continue
            b = sum(x for _, x in la)
            res[f"apply_roofline_{key}"] = {"bound": "hbm", "bytes_per_apply": int(b), "launches": len(la),
                                            "achieved": round(b / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
            if args.launch_table:
                res[f"apply_launches_{key}"] = [[lbl, int(x)] for lbl, x in la]
        return res

    # ---- headline: compositional 128x128x64 + 16 wells, FP64 apply (and FP32 beside it)
    s = solver = solver32 = X64 = X32 = None
    value = value32 = t_mv = mv_bytes = None
    rec64 = rec32 = reuse64 = app = None
    n = nnzb = b = 0
    if not args.no_headline:
        log("generating compositional 128x128x64 + 16 wells ...")
        s = W.compositional_wells(seed=2)
        n, nnzb, b = s["n"], len(s["ci"]), s["b"]
        log(f"n = {n}, block nnz = {nnzb}")
        vals = torch.tensor(s["vals"], device="cuda")
        rhs = torch.tensor(s["rhs"], device="cuda")
        torch.cuda.synchronize()
        solver, rec64, X64, info64, _ = run_steps(P, s, vals, rhs, 64, args.steps, args.warmup)
        solver32, rec32, X32, info32, _ = run_steps(P, s, vals, rhs, 32, args.steps, args.warmup)
        value = statistics.mean(a + b_ for a, b_, _, _ in rec64)
        value32 = statistics.mean(a + b_ for a, b_, _, _ in rec32)
        reuse64 = time_reuse(solver, s, row_scaled(s, seed=11), False)

        # roofline of the dominant kernel: the FGMRES block SpMV on A (FP64)
        xv = torch.randn(n, dtype=torch.float64, device="cuda")
        yv = torch.empty_like(xv)
        mv = lambda: lib.mgr_matvec(solver._h, 0, ctypes.c_void_p(xv.data_ptr()), ctypes.c_void_p(yv.data_ptr()))
        mv()
        t_mv, _ = time_kernel(mv, stream, 20, flush)
        mv_bytes = bsr_spmv_bytes(b, len(s["rp"]) - 1, nnzb)
        app = apply_timing(solver, solver32, n, 10)

    def secondary(sysd, steps, mgr_desc, apply_reps, reuse=None, matvec_roof=None):
        """FP64 and FP32 apply on one more workload: time to 1e-8, per-apply time
        (cache flushed) and the apply chain's GB/s."""
        vv_ = torch.tensor(sysd["vals"], device="cuda")
        bb_ = torch.tensor(sysd["rhs"], device="cuda")
        o = sysd.get("solver_opts", {})
        s64, r64, _, _, _ = run_steps(P, sysd, vv_, bb_, 64, steps, 1, **o)
        s32, r32, _, _, _ = run_steps(P, sysd, vv_, bb_, 32, steps, 1, **o)
        out_ = {"workload": sysd["name"], "n": sysd["n"], "nnz": int(len(sysd["ci"]) * sysd["b"] ** 2),
                "mgr": mgr_desc, "fp64": stats(r64), "fp32": stats(r32)}
        out_["speedup_time_to_tol"] = round(out_["fp64"]["time_to_tol_s"] / out_["fp32"]["time_to_tol_s"], 4)
        out_.update(apply_timing(s64, s32, sysd["n"], apply_reps))
        if matvec_roof:
            xs = torch.randn(sysd["n"], dtype=torch.float64, device="cuda")
            ys = torch.empty_like(xs)
            f = lambda: lib.mgr_matvec(s64._h, 0, ctypes.c_void_p(xs.data_ptr()), ctypes.c_void_p(ys.data_ptr()))
            f()
            t, _ = time_kernel(f, stream, 50, flush)
            nb = matvec_roof[0](sysd)
            out_["matvec_roofline"] = {"kernel": matvec_roof[1], "bound": "hbm", "achieved": round(nb / t / 1e9, 1),
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(nb / t / 1e9 / HBM_PEAK_GBS, 4),
                                       "traffic": kernel_traffic(matvec_roof[2]),
                                       "bytes_per_launch": nb, "avg_launch_us": round(1e6 * t, 2)}
        if reuse is not None:
            out_["setup_reuse"] = time_reuse(s64, sysd, row_scaled(sysd, seed=11, rows_field=reuse[0]), reuse[1])
        s64.close()
        s32.close()
        return out_

    def mimetic_matvec_bytes(sysd):
        # the library's scalar operator leaves out the exact zeros of the input (diagonal kept)
        rows = np.repeat(np.arange(sysd["n"]), np.diff(sysd["rp"]))
        return spmv_bytes(sysd["n"], int(np.count_nonzero((sysd["vals"] != 0.0) | (sysd["ci"] == rows))))

    mim = comp4 = tpfa = ext = frac = fracp = frac_paper = frac_grid = ilu = None
    if args.ilu_steps > 0 and s is not None:
        # ILU(0) as F-relaxation of the three component densities (Sec. 3.2), level-scheduled
        log("compositional 128x128x64 with ILU(0) on the components ...")
        si = dict(s, name=s["name"] + "_ilu0", levels=[dict(s["levels"][0], frelax="ilu0"), s["levels"][1]])
        ilu = secondary(si, args.ilu_steps, "L1 F = components (ILU(0)), L2 F = wells (Jacobi), coarse pressure AMG", 5)
        del si
    if args.mimetic_steps > 0:
        log("generating hybrid mimetic 64^3 ...")
        sm = W.hybrid_mimetic(64, 64, 64, seed=1)
        mim = secondary(sm, args.mimetic_steps, "1 level, F = cells (Jacobi), C = faces -> AMG V(1,1)", 20,
                        reuse=(None, False),
                        matvec_roof=(mimetic_matvec_bytes,
                                     "k_spmv_ell<double, 1, SpmvOp> (FGMRES matvec, sliced ELL copy of the CSR, FP64)",
                                     "k_spmv_fgmres_mimetic64.md"))
        if args.interp_steps > 0:
            # the same system with extended+i (distance-two) AMG interpolation
            log("mimetic 64^3 with extended+i interpolation ...")
            vm = torch.tensor(sm["vals"], device="cuda")
            bm = torch.tensor(sm["rhs"], device="cuda")
            se, re_, _, _, _ = run_steps(P, sm, vm, bm, 64, args.interp_steps, 1, interp="ext+i")
            hi = se.info()
            ext = {"workload": sm["name"], "apply": "fp64", "direct": {k: mim["fp64"][k] for k in
                                                                      ("time_to_tol_s", "iterations")},
                   "ext+i": stats(re_), "ext+i_amg_nnz": int(sum(a[1] for a in hi["amg_levels"]))}
            se.close()
        del sm
    if args.comp4_steps > 0:
        # the paper's own four-level order: rho_2, rho_1, p (AMG F-relaxation), then
        # the well system (zero diagonals) as the coarse grid
        log("generating compositional 4-level 128x128x64 + 16 wells ...")
        comp4 = secondary(W.compositional_4level(seed=4), args.comp4_steps,
                          "L1 F = rho_2 (Jacobi, exact), L2 F = rho_1 (Jacobi), L3 F = p (AMG V-cycle), "
                          "coarse = wells (direct)", 10)
    if args.tpfa_steps > 0:
        # the two reductions of the hybrid system (Sec. 3.1) on its TPFA variant, where
        # both eliminate a diagonal block: MGR_P (F = cells, faces to AMG) against
        # MGR_Pi (F = faces, the 7-point cell Schur complement to AMG)
        tpfa = {"workload": "hybrid_mimetic_tpfa_64x64x64", "apply": "fp64"}
        for red, key in (("p", "mgr_p"), ("pi", "mgr_pi")):
            log(f"generating hybrid mimetic TPFA 64^3, reduction {key} ...")
            st = W.hybrid_mimetic(64, 64, 64, seed=1, consistent=False, reduction=red)
            vt = torch.tensor(st["vals"], device="cuda")
            bt = torch.tensor(st["rhs"], device="cuda")
            sv, rt, _, _, _ = run_steps(P, st, vt, bt, 64, args.tpfa_steps, 1)
            hi = sv.info()
            tpfa[key] = dict(stats(rt), coarse_n=hi["amg_levels"][0][0], coarse_nnz=hi["amg_levels"][0][1],
                             amg_levels=len(hi["amg_levels"]))
            sv.close()
        tpfa["speedup_pi_over_p"] = round(tpfa["mgr_p"]["time_to_tol_s"] / tpfa["mgr_pi"]["time_to_tol_s"], 4)
    if args.frac_steps > 0:
        # the fracturing system (Q1 elasticity on 96^3 nodes + a 96 x 96 planar
        # fracture) with both reductions of Sec. 3.3
        log("generating fracturing 96^3 ...")
        sf = W.fracturing(96, seed=3)
        fv = args.frac_variant
        if fv in ("all", "u"):
            frac = secondary(sf, args.frac_steps,
                             "MGR_U: F = displacements (unknown-based AMG V(2,2) F-relaxation), C = fracture "
                             "pressures -> AMG", 5, reuse=(3, True))
        # the AMG settings of Sec. 4.1 for the mechanics block: one level of aggressive
        # coarsening (multi-pass interpolation) and hybrid L1 Gauss-Seidel, V(1,1)
        # and V(2,2) (chunks of 32 rows); sdc: built on the separate displacement
        # component approximation of A_uu (Sec. 4.4)
        frac_paper = {}
        for sdc in (False, True):
            for nu in (1, 2):
                key = ("sdc_" if sdc else "") + f"v{nu}{nu}"
                if fv not in ("all", "u_paper_" + key):
                    continue
                sfa = dict(sf, levels=[W.level(7, "amg", amg_unknown_based=2 if sdc else 1, amg_agg_levels=1)],
                           solver_opts=dict(nu_pre=nu, nu_post=nu, smoother="hybrid-gs", chunk=32))
                frac_paper[key] = secondary(
                    dict(sfa, name=sf["name"] + ("_sdc" if sdc else "") + f"_agg1_hgs_v{nu}{nu}"), args.frac_steps,
                    "MGR_U, F-relaxation AMG" + (" on the separate-component approximation of A_uu" if sdc else "")
                    + f" with one aggressive level and hybrid L1 Gauss-Seidel V({nu},{nu})", 5, reuse=(3, True))
        if fv in ("all", "p"):
            sp_ = dict(sf, name=sf["name"] + "_mgr_p", levels=[W.level(1 << 3, "amg")],
                       solver_opts=dict(nu_pre=2, nu_post=2, unknown_based=True))
            fracp = secondary(sp_, args.frac_steps,
                              "MGR_P: F = fracture pressures (AMG V(2,2) F-relaxation), C = displacements -> "
                              "unknown-based AMG", 5)
            del sp_
        del sf
        # iteration counts to 1e-8 against the grid, for each setting
        frac_grid = {} if fv == "all" else None
        for nn, sd in ((12, 5), (18, 6), (30, 7), (48, 8)) if fv == "all" else ():
            sg = W.fracturing(nn, seed=sd)
            row = {}
            for key, lv, o in (
                    ("mgr_u_l1jacobi_v22", sg["levels"], dict(nu_pre=2, nu_post=2)),
                    ("mgr_u_agg1_hgs_v11", [W.level(7, "amg", amg_unknown_based=True, amg_agg_levels=1)],
                     dict(nu_pre=1, nu_post=1, smoother="hybrid-gs", chunk=32)),
                    ("mgr_u_agg1_hgs_v22", [W.level(7, "amg", amg_unknown_based=True, amg_agg_levels=1)],
                     dict(nu_pre=2, nu_post=2, smoother="hybrid-gs", chunk=32)),
                    ("mgr_u_sdc_agg1_hgs_v11", [W.level(7, "amg", amg_unknown_based=2, amg_agg_levels=1)],
                     dict(nu_pre=1, nu_post=1, smoother="hybrid-gs", chunk=32))):
                g_ = P.Solver(sg["b"], sg["rp"], sg["ci"], sg["vals"], sg["field"], lv, **o)
                _, [ig] = g_.solve(torch.tensor(sg["rhs"], device="cuda"))
                row[key] = ig.iterations
                g_.close()
            frac_grid[f"{nn}^3"] = row
            log(f"  fracturing {nn}^3 iterations: {row}")
        if frac_grid is not None:
            frac_grid["96^3"] = {"mgr_u_l1jacobi_v22": frac["fp64"]["iterations"],
                                 "mgr_u_agg1_hgs_v11": frac_paper["v11"]["fp64"]["iterations"],
                                 "mgr_u_agg1_hgs_v22": frac_paper["v22"]["fp64"]["iterations"],
                                 "mgr_u_sdc_agg1_hgs_v11": frac_paper["sdc_v11"]["fp64"]["iterations"]}

    # ---- FP64 oracle on the machine's host cores, on the headline workload
    cpu = None
    x_err64 = x_err32 = None
    host = {"nproc": len(os.sched_getaffinity(0)), "cpu_model": None}
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                host["cpu_model"] = line.split(":", 1)[1].strip()
    except OSError:
        pass
    if not args.no_cpu_baseline and s is not None:
        import oracle as O
        ncores = host["nproc"]
        O.set_threads(1)
        log("oracle (CPU): setup (serial), solve on 1 thread, solve on all host cores ...")
        t0 = time.perf_counter()
        om = O.MGR(s["b"], s["rp"], s["ci"], s["vals"], s["field"], [O.LevelOpts(**l) for l in s["levels"]])
        t1 = time.perf_counter()
        xo, io = om.solve(s["rhs"])
        t2 = time.perf_counter()
        used = O.set_threads(ncores)
        t3 = time.perf_counter()
        xo2, io2 = om.solve(s["rhs"])
        t4 = time.perf_counter()
        O.set_threads(1)
        assert np.array_equal(xo, xo2), "oracle result depends on the thread count"
        log(f"  oracle setup {t1 - t0:.2f} s, solve {t2 - t1:.2f} s (1 thread), {t4 - t3:.2f} s ({used} threads), "
            f"iters {io.iterations}")
        cpu = {"value": round((t1 - t0) + (t4 - t3), 4), "unit": "s", "cores": used, "kind": "oracle",
               "sample": f"one full setup (serial code) + FGMRES solve to 1e-8 of the headline compositional "
                         f"system: setup {t1 - t0:.2f} s, solve {t4 - t3:.2f} s on {used} threads, "
                         f"{io.iterations} iterations",
               "single_thread": {"value": round(t2 - t0, 4), "setup_s": round(t1 - t0, 4),
                                 "solve_s": round(t2 - t1, 4)},
               "host": host}
        nx = np.linalg.norm(xo)
        x_err64 = float(np.linalg.norm(X64.cpu().numpy() - xo) / nx)
        x_err32 = float(np.linalg.norm(X32.cpu().numpy() - xo) / nx)

    head = {}
    if s is not None:
        head = {
            "value": round(value, 6),
            "ms_per_step": round(1e3 * value, 3),
            "config": {"workload": s["name"], "n": n, "nnz": int(nnzb * b * b), "block_size": b,
                       "mgr": "L1 F = components (block-Jacobi), L2 F = wells (Jacobi), coarse pressure AMG V(1,1)",
                       "rtol": 1e-8, "restart": 50},
            "setup_s": round(statistics.mean(a for a, _, _, _ in rec64), 6),
            "solve_s": round(statistics.mean(b_ for _, b_, _, _ in rec64), 6),
            "iterations": rec64[-1][2],
            "rel_res_true": rec64[-1][3],
            "x_rel_err_vs_oracle": x_err64,
            "setup_reuse": reuse64,
            "fp32_apply": dict(stats(rec32), x_rel_err_vs_oracle=x_err32,
                               speedup_time_to_tol=round(value / value32, 4)),
            "apply": app,
            "roofline": {"kernel": f"k_bsr_spmv<{b}, 8> (FGMRES matvec y = A x, {b} x {b} block CSR, FP64)",
                         "bound": "hbm", "achieved": round(mv_bytes / t_mv / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(mv_bytes / t_mv / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": kernel_traffic("k_bsr_spmv_compositional.md"),
                         "bytes_per_launch": mv_bytes, "avg_launch_us": round(1e6 * t_mv, 2)},
        }
    out = {
        "metric": "FGMRES+MGR time-to-1e-8 (s), HBM GB/s; FP32-vs-FP64 apply speedup",
        "value": head.pop("value", None),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step", None),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head.pop("config", None),
    }
    out.update(head)
    out.update({
        "secondary_mimetic": mim,
        "secondary_mimetic_ext_interp": ext,
        "secondary_compositional_4level": comp4,
        "secondary_compositional_ilu0": ilu,
        "secondary_mimetic_tpfa_reductions": tpfa,
        "secondary_fracturing_mgr_u": frac,
        "secondary_fracturing_mgr_p": fracp,
        "secondary_fracturing_mgr_u_paper_amg": frac_paper,
        "fracturing_iterations_by_grid": frac_grid,
        "cpu_baseline": cpu,
    })
    print(json.dumps(out), flush=True)
    if solver is not None:
        solver.close()
        solver32.close()


if __name__ == "__main__":
    main()
