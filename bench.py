#!/usr/bin/env python3
"""Benchmark of the condensed-Helmholtz BT solve on one MI355X.

Workload (default line): 24^3 uniform elements on the unit cube, GLL degree
p = 12, lambda = 1, homogeneous Dirichlet, 16 N(0,1) nodal right-hand sides
from the seeded generator (N = 289^3 = 24,137,569 nodes per RHS, N_s =
5,737,825 skeleton nodes).

One step = one batched solve of the 16 right-hand sides to ||r~|| <= 1e-10
||F^~|| each, in mixed precision: FP32 operator and inner BT conjugate
gradients (FP64 dot products), FP64 iterative refinement (residual with the
FP64 operator), then back-transform and interior recovery in FP64 (all on the
GPU; inputs resident in HBM).  The same batch solved in plain FP64 is timed
beside it over the same number of steps (mixed vs FP64 time to 1e-10).

value = N * sum_r (operator applications of RHS r) / step time [GDOF/s]:
the condensed-operator DOF applications per second sustained inside the
solve, the reciprocal of the PCG time per DOF and iteration.  The roofline is
that of the dominant kernel of the timed steps (the FP32 CG apply), from its
algorithmic bytes and its kernel time from HIP events the library records on
the launch stream during the timed steps.  The line also reports the FP64
solve's CG apply roofline, the standalone applies, the one-launch-per-solve
(persistent) CG, the 16^3, p = 8 single-RHS FP64 solve (extra keys), and the
FP64 CPU oracle's condensed apply on the same mesh on all host cores and on
one core.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GDOF/s condensed Helmholtz apply; PCG time/DOF/iter, mixed vs FP64 @1e-10"
HBM_PEAK_GBS = 8000.0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _apply_rate(ctx, semcond, torch, k=1, reps=20):
    """Kernel time (HIP events) of the transformed-basis apply on k random RHS."""
    xs = torch.randn((ctx.N_s, k) if k > 1 else (ctx.N_s,), dtype=torch.float64, device="cuda")
    ys = torch.empty_like(xs)
    for _ in range(3):
        ctx.apply(xs, out=ys)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.apply(xs, out=ys)
    ms, n, _ = ctx.profile_read(semcond.KERNEL_APPLY)
    ctx.profile_enable(False)
    return ms / 1e3 / max(n, 1)


def suite(args):
    """Measurements beyond the default line, one JSON line per case:
    p/aspect-ratio sweep at N = 257^3 (FP64 solve to 1e-10 and apply rate),
    16 right-hand sides at 24^3 elements, p = 12 (FP64 batched vs mixed
    precision, each CG launch kind), the differentiable solve's forward and
    backward on 8^3 elements, p = 8, k = 8, and the paper's solver experiment
    (manufactured solution with inhomogeneous Dirichlet values, lambda = 0,
    8^3 elements, expansion factors 1, 1.5, 2, p = 8..32)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1601_08179_amd import autograd as AG
    from paper_1601_08179_amd import semcond

    def emit(d):
        print(json.dumps(d), flush=True)

    if "2" in args.suite:
        # the 16^3, p = 8 single-RHS FP64 line alone (its kernel trace)
        d = config2_line(args, semcond, torch)
        d["case"] = "config2: 16^3 elements, p=8, one RHS, FP64"
        emit(d)
    if "3" in args.suite:
        for p in (2, 4, 8, 16, 32):
            for ar in (1, 8, 32, 128):
                wmesh, f = W.config3(p, ar)
                ctx = semcond.Context(wmesh)
                ft = torch.tensor(f, device="cuda")
                u = torch.zeros_like(ft)
                ctx.solve(ft, out=u, tol=1e-10)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = ctx.solve(ft, out=u, tol=1e-10)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ks = _apply_rate(ctx, semcond, torch)
                bw = 2 * 8 * ctx.N_s / ks / 1e9
                emit({"case": "p/AR sweep, N=257^3", "p": p, "aspect": ar, "n_e": ctx.n_e, "N": ctx.N,
                      "N_s": ctx.N_s, "iters": info[0]["iters"], "rel_res": info[0]["rel_res"],
                      "solve_ms": dt * 1e3, "ns_per_dof_iter": dt / (ctx.N * info[0]["iters"]) * 1e9,
                      "apply_us": ks * 1e6, "apply_gdof_s": ctx.N / ks / 1e9, "apply_gbs": bw,
                      "apply_hbm_frac": bw / HBM_PEAK_GBS})
                del ft, u
                ctx.close()
                torch.cuda.empty_cache()
    if "4" in args.suite:
        wmesh, f = W.config4()
        k = f.shape[0]
        ctx = semcond.Context(wmesh)
        ft = torch.tensor(f, device="cuda")
        del f
        u = torch.zeros_like(ft)
        res = {"case": "k=16 RHS, 24^3 elements, p=12", "n_e": ctx.n_e, "N": ctx.N, "N_s": ctx.N_s, "k": k}
        for name, kw in [("f64_stepwise", dict(persistent=False)), ("f64_persistent", dict(persistent=True)),
                         ("mixed_stepwise", dict(precision=semcond.PREC_MIXED_IR, persistent=False)),
                         ("mixed_persistent", dict(precision=semcond.PREC_MIXED_IR, persistent=True)),
                         ("mixed_restart_stepwise", dict(precision=semcond.PREC_MIXED_IR, inner_tol=1e-4,
                                                         ir_restart=True, persistent=False))]:
            ctx.solve(ft, out=u, tol=1e-10, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = ctx.solve(ft, out=u, tol=1e-10, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[name] = {"ms_per_rhs": dt * 1e3 / k, "iters_max": max(i["iters"] for i in info),
                         "outer_max": max(i["outer"] for i in info),
                         "rel_res_max": max(i["rel_res"] for i in info)}
        res["mixed_speedup_vs_f64"] = res["f64_stepwise"]["ms_per_rhs"] / res["mixed_stepwise"]["ms_per_rhs"]
        for dt_name, dt_t in (("f64", torch.float64), ("f32", torch.float32)):
            S, G = ctx.autotune(k=k, dtype=dt_t)
            res["tuned_" + dt_name] = "stepwise" if S == 0 else "persistent S=%d G=%d" % (S, G)
        ks = _apply_rate(ctx, semcond, torch, k=k, reps=10)
        bw = 2 * 8 * ctx.N_s * k / ks / 1e9
        res["apply_k16"] = {"us": ks * 1e6, "gdof_s": ctx.N * k / ks / 1e9, "gbs": bw, "hbm_frac": bw / HBM_PEAK_GBS}
        emit(res)
        del ft, u
        ctx.close()
        torch.cuda.empty_cache()
    if "D" in args.suite:
        # Solver experiment of Sec. 8: manufactured u (stiffness 5) on (0, 2 pi)^3,
        # lambda = 0, 8^3 elements with expansion factor alpha, inhomogeneous
        # Dirichlet values u_ex, stop at a 1e-12 residual reduction.  For alpha = 2
        # the paper's BT iteration counts follow from its iteration-times table (Sec. 8) as solution time per
        # DOF / iteration time per DOF (upper bounds: the solution time includes
        # the precomputation).
        table3 = {8: (4.25, 25.6), 12: (3.73, 20.3), 16: (3.47, 17.7), 20: (3.31, 16.1), 24: (3.09, 14.4),
                  28: (2.88, 13.1), 32: (2.81, 12.4)}
        # one context first, so that the first case's set-up time does not
        # include loading the library's kernels
        semcond.Context(W.solver_experiment_mesh(8, 1.0)).close()
        for alpha in (1.0, 1.5, 2.0):
            for p in (8, 12, 16, 20, 24, 28, 32):
                wm = W.solver_experiment_mesh(p, alpha)
                X = W.nodal_coordinates(p, wm["n"], wm["widths"], semcond.host_tables(p)["x"])
                uex = W.manufactured_u(X, 5.0)
                f = -W.manufactured_laplacian(X, 5.0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx = semcond.Context(wm)
                torch.cuda.synchronize()
                setup_s = time.perf_counter() - t0
                ft = torch.as_tensor(f, device="cuda")
                gt = torch.as_tensor(uex, device="cuda")
                u = torch.zeros_like(ft)
                ctx.solve(ft, out=u, tol=1e-12, g=gt)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = ctx.solve(ft, out=u, tol=1e-12, g=gt)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                err = float(np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max())
                rec = {"case": "solver experiment (Sec. 8): 8^3 elements, lambda=0, inhomogeneous Dirichlet",
                       "alpha": alpha, "p": p, "N": ctx.N, "iters": info[0]["iters"],
                       "rel_res": info[0]["rel_res"], "solve_ms": dt * 1e3, "setup_ms": setup_s * 1e3,
                       "ns_per_dof_iter": dt / (ctx.N * info[0]["iters"]) * 1e9,
                       "us_per_dof_solve_incl_setup": (dt + setup_s) / ctx.N * 1e6,
                       "max_rel_error_vs_exact": err}
                if alpha == 2.0:
                    sol_us, it_ns = table3[p]
                    rec["paper_bt_iters_from_table3"] = round(sol_us * 1e3 / it_ns)
                    rec["paper_bt_ns_per_dof_iter"] = it_ns
                emit(rec)
                del ft, gt, u
                ctx.close()
                torch.cuda.empty_cache()
    if "S" in args.suite:
        # Element-count scaling of the solver experiment (Sec. 8): expansion factor
        # 1, p = 16, n^3 elements for n = 2..16.
        for n in (2, 4, 6, 8, 10, 12, 14, 16):
            wm = W.solver_experiment_mesh(16, 1.0, n=n)
            X = W.nodal_coordinates(16, wm["n"], wm["widths"], semcond.host_tables(16)["x"])
            uex = W.manufactured_u(X, 5.0)
            ctx = semcond.Context(wm)
            ft = torch.as_tensor(-W.manufactured_laplacian(X, 5.0), device="cuda")
            gt = torch.as_tensor(uex, device="cuda")
            u = torch.zeros_like(ft)
            ctx.solve(ft, out=u, tol=1e-12, g=gt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = ctx.solve(ft, out=u, tol=1e-12, g=gt)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec = {"case": "element-count scaling (Sec. 8): expansion factor 1, p=16, lambda=0", "n_e": n ** 3,
                   "N": ctx.N, "iters": info[0]["iters"], "solve_ms": dt * 1e3,
                   "ns_per_dof_iter": dt / (ctx.N * info[0]["iters"]) * 1e9,
                   "max_rel_error_vs_exact": float(np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max())}
            # the same solve with the two-level preconditioner (first call builds the coarse matrix)
            ctx.solve(ft, out=u, tol=1e-12, g=gt, coarse=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info2 = ctx.solve(ft, out=u, tol=1e-12, g=gt, coarse=True)
            torch.cuda.synchronize()
            rec["two_level_iters"] = info2[0]["iters"]
            rec["two_level_solve_ms"] = (time.perf_counter() - t0) * 1e3
            rec["two_level_max_rel_error_vs_exact"] = float(np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max())
            emit(rec)
            del ft, gt, u
            ctx.close()
            torch.cuda.empty_cache()
    if "E" in args.suite:
        # Operator experiment of Sec. 7: 8^3 uniform elements (n_e = 512), lambda =
        # pi, p = 2..32, one RHS: TPT (transformed basis), TPC and MMC (physical
        # basis) apply times from HIP events over repeated launches, and their
        # precomputation times (context creation for TPT and TPC, plus the class
        # matrices for MMC).
        import math

        def ev_time(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps / 1e3

        for p in range(2, 33):
            wm = W.mesh(p, (8, 8, 8), lam=math.pi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx = semcond.Context(wm)
            torch.cuda.synchronize()
            setup_tpt = time.perf_counter() - t0
            x = torch.randn(ctx.N_s, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            t_tpt = ev_time(lambda: ctx.apply(x, out=y), 50)
            t_tpc = ev_time(lambda: ctx.apply_variant(x, semcond.VARIANT_TPC, out=y), 20)
            rec = {"case": "operator experiment (Sec. 7): 8^3 elements, lambda=pi", "p": p, "n_e": 512,
                   "N": ctx.N, "N_s": ctx.N_s, "tpt_us": t_tpt * 1e6, "tpc_us": t_tpc * 1e6,
                   "tpc_over_tpt": t_tpc / t_tpt, "setup_tpt_ms": setup_tpt * 1e3}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.variant_setup(semcond.VARIANT_MMC)
            torch.cuda.synchronize()
            rec["setup_mmc_ms"] = (time.perf_counter() - t0) * 1e3
            t_mmc = ev_time(lambda: ctx.apply_variant(x, semcond.VARIANT_MMC, out=y), 20)
            rec["mmc_us"] = t_mmc * 1e6
            rec["mmc_over_tpt"] = t_mmc / t_tpt
            rec["mmc_over_tpc"] = t_mmc / t_tpc
            emit(rec)
            del x, y
            ctx.close()
            torch.cuda.empty_cache()
    if "5" in args.suite:
        wmesh, f, t = W.config5()
        ctx = semcond.Context(wmesh)
        ft = torch.tensor(f, device="cuda")
        tt = torch.tensor(t, device="cuda")
        lam_e = torch.tensor(wmesh["lam_e"], dtype=torch.float64, requires_grad=True)
        h = [np.asarray(w) for w in wmesh["widths"]]
        e1, e2, e3 = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
        J = (h[0][e1] * h[1][e2] * h[2][e3] / 8.0).transpose(2, 1, 0).reshape(-1)
        dm = np.stack([J * 4 / h[0][e1].transpose(2, 1, 0).reshape(-1) ** 2,
                       J * 4 / h[1][e2].transpose(2, 1, 0).reshape(-1) ** 2,
                       J * 4 / h[2][e3].transpose(2, 1, 0).reshape(-1) ** 2], axis=1)
        dmetric = torch.tensor(dm, dtype=torch.float64, requires_grad=True)
        fv = ft.clone().requires_grad_(True)
        times = []
        for rep in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uu = AG.solve(ctx, fv, lam_e, dmetric, tol=1e-12)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss = 0.5 * ((uu - tt) ** 2).sum()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append((t1 - t0, t2 - t1))
            fv.grad = None
            lam_e.grad = None
            dmetric.grad = None
        fw = min(x[0] for x in times)
        bw_ = min(x[1] for x in times)
        emit({"case": "differentiable solve, 8^3 elements, p=8, k=8", "N": ctx.N, "forward_ms": fw * 1e3,
              "backward_ms": bw_ * 1e3})
        ctx.close()


# ---------------------------------------------------------------------------
# HBM traffic of the dominant kernel from rocprofv3 counters
# ---------------------------------------------------------------------------
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cg_apply_f32_config4_p12_k16.md")
NI4 = 11  # interior nodes per direction at p = 12
DOMINANT = "k_apply_tpt<float, %d, true, false>" % NI4
KERNEL_SOURCES = ["apply.hip", "apply_element.h", "cg_device.h", "device_common.h", "kernels.h", "layout.h"]
COPY_BYTES = 256 << 20


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1601_08179_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_workload():
    """Dispatches the counter runs read: a plain device copy of COPY_BYTES
    (calibration) and one mixed-precision solve of the default workload (its
    FP32 CG applies are the dominant kernel)."""
    import torch

    import workloads as W
    from paper_1601_08179_amd import semcond

    x = torch.randn(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)  # a plain streaming kernel: reads and writes COPY_BYTES
    torch.cuda.synchronize()
    del x, y
    wmesh, f = W.config4()
    ctx = semcond.Context(wmesh)
    ft = torch.tensor(f, device="cuda")
    del f
    u = torch.zeros_like(ft)
    _, info = ctx.solve(ft, out=u, tol=1e-10, precision=semcond.PREC_MIXED_IR, persistent=False)
    torch.cuda.synchronize()
    print("pmc workload: inner iterations per RHS", [i["iters"] for i in info], flush=True)
    ctx.close()


def pmc_summary(fetch_csv, write_csv, commands):
    """Per-launch HBM bytes of the dominant kernel from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled by what the counter reads for the
    calibration copy; written to TRAFFIC_FILE."""
    import csv

    def read(path, counter):
        rows = {}
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                rows.setdefault(row["Kernel_Name"], []).append((int(row["Grid_Size"]), float(row["Counter_Value"])))
        return rows

    fe, wr = read(fetch_csv, "FETCH_SIZE"), read(write_csv, "WRITE_SIZE")

    def copy_value(rows):
        # the calibration kernel: torch's elementwise multiply by a scalar (largest grid)
        cand = [(g, v) for name, lst in rows.items()
                if "elementwise" in name and ("Mul" in name or "UnaryFunctor" in name) for g, v in lst]
        gmax = max(g for g, _ in cand)
        big = [v for g, v in cand if g == gmax]
        return sum(big) / len(big)

    def dominant(rows):
        # full applies only: launches in which every RHS has stopped exit at once
        # and read a few KiB (below a tenth of the median)
        for name, lst in rows.items():
            if name.startswith("void semcond::" + DOMINANT):
                vals = sorted(v for _, v in lst)
                full = [v for v in vals if v >= 0.1 * vals[len(vals) // 2]]
                return sum(full) / len(full), len(full), len(vals)
        raise KeyError(DOMINANT)

    ff = COPY_BYTES / (copy_value(fe) * 1024.0)
    fw = COPY_BYTES / (copy_value(wr) * 1024.0)
    (fk, nf, naf), (wk, nw, naw) = dominant(fe), dominant(wr)
    fetch_b, write_b = fk * 1024.0 * ff, wk * 1024.0 * fw
    lines = [
        "# HBM traffic of %s (FP32 CG apply of the mixed-precision solve: 24^3 elements, p = 12, "
        "k = 16 RHS; MI355X)" % DOMINANT,
        "",
        "Commands (from the repository root, on one MI355X):",
        "",
        "```",
    ] + commands + [
        "```",
        "",
        "| quantity | value |",
        "|---|---|",
        "| calibration: FETCH_SIZE of a streaming kernel reading and writing %d MiB | %.0f KiB (factor %.4f) |" % (
            COPY_BYTES >> 20, copy_value(fe), ff),
        "| calibration: WRITE_SIZE of the same kernel | %.0f KiB (factor %.4f) |" % (copy_value(wr), fw),
        "| dominant kernel FETCH_SIZE per full dispatch (%d of %d dispatches) | %.1f KiB |" % (nf, naf, fk),
        "| dominant kernel WRITE_SIZE per full dispatch (%d of %d dispatches) | %.1f KiB |" % (nw, naw, wk),
        "| scaled HBM read bytes per full launch | %.0f |" % fetch_b,
        "| scaled HBM write bytes per full launch | %.0f |" % write_b,
        "",
        "traffic_bytes_per_launch: %.0f" % (fetch_b + write_b),
        "kernel_sources_sha256: %s" % kernel_sources_hash(),
        "",
    ]
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def stored_traffic():
    """Per-launch HBM bytes of the dominant kernel from TRAFFIC_FILE, or None when
    absent or taken from kernel sources other than the current ones."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes", "kernel_sources")))
    if vals.get("kernel_sources_sha256", "").strip() != kernel_sources_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_cg_apply_f32_config4_p12_k16.md")


def stored_valu_busy():
    """Fraction of SIMD cycles issuing VALU instructions in the dominant kernel,
    from the SQ counter summary, or None when absent or taken from other kernel
    sources."""
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("valu_busy", "kernel_sources")))
    if vals.get("kernel_sources_sha256", "").strip() != kernel_sources_hash():
        return None
    return float(vals["valu_busy"])


def copy_bandwidth(torch):
    """STREAM-style copy on this GPU (1 GiB read + 1 GiB written), GB/s."""
    ca = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    cb = torch.empty_like(ca)
    for _ in range(3):
        cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * ca.numel() * 8 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del ca, cb
    return gbs


def cpu_baseline_config4(wmesh, seconds):
    """The FP64 CPU oracle's condensed apply (explicit Schur complement of the
    single element class, one DGEMM, index gather and scatter-add) of one RHS on
    the default mesh: on all host cores, and on one core (BLAS limited to one
    thread), each for about `seconds` (at least one apply)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import workloads as W
    from oracle import mesh as M
    from oracle.operators import CondensedOperator

    t0 = time.perf_counter()
    op = CondensedOperator(M.make_mesh(**wmesh))
    setup = time.perf_counter() - t0
    u = W.random_skeleton_input(op.sizes["N"], k=1, seed=0)[0]
    N = op.sizes["N"]

    def run(limit):
        reps, t0 = 0, time.perf_counter()
        while True:
            op.apply(u)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= seconds or reps >= 200:
                return reps, dt

    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    op.apply(u)
    reps, dt = run(None)
    with threadpool_limits(limits=1, user_api="blas"):
        reps1, dt1 = run(1)
    model = cpu_model()
    full = {"value": N * reps / dt / 1e9, "unit": "GDOF/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d oracle condensed applies of one RHS (explicit Schur complement of the one element "
                      "class, one DGEMM per apply, index gather and scatter-add; no CG vector work) on the "
                      "24^3, p = 12 mesh, %.1f s on %d BLAS threads, %s; oracle set-up %.1f s not timed" % (
                          reps, dt, threads, model, setup)}
    one = {"value": N * reps1 / dt1 / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
           "sample": "%d oracle condensed applies of one RHS, same mesh, %.1f s with BLAS limited to one "
                     "thread, %s" % (reps1, dt1, model)}
    return full, one


def config2_line(args, semcond, torch):
    """The 16^3, p = 8, lambda = 1e-3 single-RHS FP64 solve (the earlier default
    line), its standalone apply and the CG apply roofline, as extra keys."""
    import workloads as W

    wmesh, f = W.config2(k=1)
    ctx = semcond.Context(wmesh)
    ft = torch.tensor(f, device="cuda")
    u = torch.zeros_like(ft)
    N, Ns = ctx.N, ctx.N_s
    for _ in range(2):
        ctx.solve(ft, out=u, tol=args.tol, persistent=False)
    reps = 10
    torch.cuda.synchronize()
    # solve time without the tracing events (two event records around each
    # 20 us apply launch would add to it), then the apply times with them
    t0 = time.perf_counter()
    iters = 0
    for _ in range(reps):
        _, info = ctx.solve(ft, out=u, tol=args.tol, persistent=False)
        iters += info[0]["iters"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    it = iters / reps
    preps, piters = 3, 0
    ctx.profile_enable(True)
    for _ in range(preps):
        _, info = ctx.solve(ft, out=u, tol=args.tol, persistent=False)
        piters += info[0]["iters"]
    torch.cuda.synchronize()
    ap_ms, ap_launches, _ = ctx.profile_read(semcond.KERNEL_APPLY)
    ctx.profile_enable(False)
    # CG apply: gathers p, r and P^-1 and writes q (4 N_s FP64) per full launch
    full = int(piters)
    cg_gbs = 4 * 8 * Ns * full / (ap_ms / 1e3) / 1e9
    ks = _apply_rate(ctx, semcond, torch, k=1, reps=100)
    out = {"workload": "BT solve to 1e-10, FP64: 16^3 uniform elements, p=8, lambda=1e-3, one N(0,1) RHS",
           "N": N, "N_s": Ns, "iterations": it, "ms_per_solve": dt * 1e3,
           "gdof_s": N * it / dt / 1e9, "ns_per_dof_iter": dt / (N * it) * 1e9,
           "cg_apply": {"kernel": "k_apply_tpt<double,7,true,true>", "us_per_launch": ap_ms * 1e3 / ap_launches,
                        "launches": ap_launches, "full_launches": full, "gbs": cg_gbs,
                        "hbm_frac": cg_gbs / HBM_PEAK_GBS},
           "apply": {"kernel": "k_apply_tpt<double,7,false,false>", "us": ks * 1e6, "gdof_s": N / ks / 1e9,
                     "gbs": 2 * 8 * Ns / ks / 1e9, "hbm_frac": 2 * 8 * Ns / ks / 1e9 / HBM_PEAK_GBS}}
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config2", action="store_true")
    ap.add_argument("--no-persistent", action="store_true", help="skip the one-launch-per-solve CG runs")
    ap.add_argument("--no-two-level", action="store_true", help="skip the two-level preconditioner runs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--suite", default="", help="extra measurements instead of the default line: "
                    "any of 2 (the 16^3, p = 8 single-RHS FP64 solve alone), 3 (p/AR sweep), 4 (16 RHS, "
                    "every launch kind), 5 (differentiable solve), "
                    "D (the paper's solver experiment with inhomogeneous Dirichlet values), S (its "
                    "element-count scaling), E (the operator experiment: TPT, TPC, MMC at p = 2..32), "
                    "e.g. --suite 345DSE")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="run only the dispatches the rocprofv3 counter runs read")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from the two counter runs' CSV files")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="command line recorded in the traffic summary (repeatable)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single GPU and has no "
              "multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.suite:
        suite(args)
        return
    if args.pmc_workload:
        pmc_workload()
        return

    import torch

    import workloads as W
    from paper_1601_08179_amd import semcond

    wmesh, f = W.config4()
    k = f.shape[0]
    ctx = semcond.Context(wmesh)
    ft = torch.tensor(f, device="cuda")
    del f
    u = torch.zeros_like(ft)
    N, Ns = ctx.N, ctx.N_s
    mixed = dict(precision=semcond.PREC_MIXED_IR, persistent=False)
    fp64 = dict(precision=semcond.PREC_F64, persistent=False)
    for _ in range(args.warmup):
        ctx.solve(ft, out=u, tol=args.tol, **mixed)
        ctx.solve(ft, out=u, tol=args.tol, **fp64)
    torch.cuda.synchronize()

    def timed(kw, kind):
        """K solves; the apply launches of `kind` are bracketed by HIP events on
        the launch stream during the timed solves."""
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        applies = 0
        iters = []
        for _ in range(args.steps):
            _, info = ctx.solve(ft, out=u, tol=args.tol, **kw)
            iters.append([i["iters"] for i in info])
            applies += sum(i["iters"] + i["outer"] for i in info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, launches, _ = ctx.profile_read(kind)
        ctx.profile_enable(False)
        return dt, applies, iters, info, ms, launches

    # ---- timed region: K mixed-precision batched solves ---------------------------
    m_dt, m_applies, m_iters, m_info, m_ms, m_launches = timed(mixed, semcond.KERNEL_APPLY_F32)
    # ---- the same K solves in plain FP64 -------------------------------------------
    d_dt, d_applies, d_iters, d_info, d_ms, d_launches = timed(fp64, semcond.KERNEL_APPLY)
    step_s = m_dt / args.steps
    f64_s = d_dt / args.steps
    value = N * m_applies / m_dt / 1e9

    # Roofline of the dominant kernel (the CG apply): algorithmic bytes per RHS
    # and application are 3 s N_s (gather of the direction's p and r, store of
    # q; P^-1 is shared by the RHS and left out); the applications are the RHS'
    # CG iterations (an RHS that has stopped is skipped in the launch).
    rhs_its_m = sum(sum(x) for x in m_iters)
    rhs_its_d = sum(sum(x) for x in d_iters)
    bytes_m = 3 * 4 * Ns * rhs_its_m
    bytes_d = 3 * 8 * Ns * rhs_its_d
    ach_m = bytes_m / (m_ms / 1e3) / 1e9
    ach_d = bytes_d / (d_ms / 1e3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    traffic = stored_traffic()
    # launches count every dispatch, also those in which some RHS have stopped (the
    # time per launch is an average over them); the counter traffic is per full
    # launch (all 16 RHS active), next to algorithmic_bytes_per_full_launch
    roof = {"bound": "hbm", "achieved": ach_m, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach_m / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per full launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            # what the counters show limits it: the SIMDs' VALU issue (fraction of cycles)
            "valu_busy": stored_valu_busy(),
            "kernel": DOMINANT.replace(" ", ""), "launches": m_launches,
            "kernel_us_per_launch": m_ms * 1e3 / max(m_launches, 1),
            "algorithmic_bytes_per_launch": bytes_m / max(m_launches, 1),
            "rhs_applications": rhs_its_m, "bytes_per_rhs_application": 3 * 4 * Ns,
            "algorithmic_bytes_per_full_launch": 3 * 4 * Ns * k,
            "copy_gbs_measured": copy_gbs, "frac_of_measured_copy": ach_m / copy_gbs}
    roof64 = {"bound": "hbm", "achieved": ach_d, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach_d / HBM_PEAK_GBS,
              "kernel": "k_apply_tpt<double,%d,true,false>" % NI4, "launches": d_launches,
              "kernel_us_per_launch": d_ms * 1e3 / max(d_launches, 1),
              "algorithmic_bytes_per_launch": bytes_d / max(d_launches, 1),
              "rhs_applications": rhs_its_d, "bytes_per_rhs_application": 3 * 8 * Ns}

    # ---- standalone applies of all 16 RHS (transformed basis), HIP-event kernel time
    ks64 = _apply_rate(ctx, semcond, torch, k=k, reps=10)
    xs = torch.randn((Ns, k), dtype=torch.float32, device="cuda")
    ys = torch.empty_like(xs)
    for _ in range(3):
        ctx.apply(xs, out=ys)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    for _ in range(10):
        ctx.apply(xs, out=ys)
    ms32, n32, _ = ctx.profile_read(semcond.KERNEL_APPLY_F32)
    ctx.profile_enable(False)
    ks32 = ms32 / 1e3 / max(n32, 1)
    del xs, ys
    # ---- one persistent (cooperative, one launch per solve) CG run of each precision
    pers = {}
    for name, kw in () if args.no_persistent else (("f64", dict(precision=semcond.PREC_F64)),
                                                   ("mixed", dict(precision=semcond.PREC_MIXED_IR))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, pinfo = ctx.solve(ft, out=u, tol=args.tol, persistent=True, **kw)
        torch.cuda.synchronize()
        pers[name + "_ms_per_rhs"] = (time.perf_counter() - t0) * 1e3 / k
    # ---- the two-level preconditioner (BT diagonal + trilinear coarse correction)
    two = {}
    if not args.no_two_level:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(ft, out=u, tol=args.tol, precision=semcond.PREC_F64, persistent=False, coarse=True)
        torch.cuda.synchronize()
        two["first_solve_ms_incl_setup"] = (time.perf_counter() - t0) * 1e3
        for name, prec in (("f64", semcond.PREC_F64), ("mixed", semcond.PREC_MIXED_IR)):
            ctx.solve(ft, out=u, tol=args.tol, precision=prec, persistent=False, coarse=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                _, tinfo = ctx.solve(ft, out=u, tol=args.tol, precision=prec, persistent=False, coarse=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            two[name] = {"ms_per_step": dt * 1e3, "ms_per_rhs": dt * 1e3 / k,
                         "iterations_per_rhs": [i["iters"] for i in tinfo],
                         "outer_steps_per_rhs": [i["outer"] for i in tinfo],
                         "rel_res_max": max(i["rel_res"] for i in tinfo)}
        two["f64_speedup_vs_bt_f64"] = f64_s * 1e3 / two["f64"]["ms_per_step"]
        two["mixed_speedup_vs_bt_f64"] = f64_s * 1e3 / two["mixed"]["ms_per_step"]
        two["mixed_speedup_vs_bt_mixed"] = step_s * 1e3 / two["mixed"]["ms_per_step"]
    ctx.close()
    del ft, u
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operator and inner CG, f64 refinement",
        "data": "synthetic",
        "config": {"workload": "mixed-precision batched BT solve to 1e-10: 24^3 uniform elements, p=12, "
                               "lambda=1, unit cube, Dirichlet, k=16 N(0,1) nodal RHS (seeded)",
                   "p": 12, "n_e": 13824, "N": N, "N_s": Ns, "k": k, "tol": args.tol,
                   "parallelism": "single GPU"},
        "ms_per_rhs": step_s * 1e3 / k,
        "ns_per_dof_iter": m_dt / (N * m_applies) * 1e9,
        "mixed": {"inner_iterations_per_rhs": [i["iters"] for i in m_info],
                  "outer_steps_per_rhs": [i["outer"] for i in m_info],
                  "rel_res_max": max(i["rel_res"] for i in m_info)},
        "f64": {"ms_per_step": f64_s * 1e3, "ms_per_rhs": f64_s * 1e3 / k,
                "gdof_s": N * d_applies / d_dt / 1e9, "ns_per_dof_iter": d_dt / (N * d_applies) * 1e9,
                "iterations_per_rhs": [i["iters"] for i in d_info],
                "rel_res_max": max(i["rel_res"] for i in d_info)},
        "mixed_speedup_vs_f64": f64_s / step_s,
        "roofline": roof,
        "roofline_f64_cg_apply": roof64,
        "apply_k16": {"f64": {"kernel": "k_apply_tpt<double,%d,false,false>" % NI4, "us": ks64 * 1e6,
                              "gdof_s": N * k / ks64 / 1e9, "gbs": 2 * 8 * Ns * k / ks64 / 1e9,
                              "hbm_frac": 2 * 8 * Ns * k / ks64 / 1e9 / HBM_PEAK_GBS},
                      "f32": {"kernel": "k_apply_tpt<float,%d,false,false>" % NI4, "us": ks32 * 1e6,
                              "gdof_s": N * k / ks32 / 1e9, "gbs": 2 * 4 * Ns * k / ks32 / 1e9,
                              "hbm_frac": 2 * 4 * Ns * k / ks32 / 1e9 / HBM_PEAK_GBS}},
        "persistent_cg": pers,
        "two_level": two,
    }
    if not args.no_config2:
        out["config2"] = config2_line(args, semcond, torch)
    if not args.no_cpu_baseline:
        full, one = cpu_baseline_config4(wmesh, args.cpu_seconds)
        out["cpu_baseline"] = full
        out["cpu_baseline_1core"] = one
    print(json.dumps(out))


if __name__ == "__main__":
    main()
