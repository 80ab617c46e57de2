#!/usr/bin/env python3
"""Benchmark of the condensed-Helmholtz BT solve on one MI355X.

Workload (default): 16^3 uniform elements on the unit cube, GLL degree p = 8,
lambda = 1e-3, homogeneous Dirichlet, one N(0,1) nodal right-hand side drawn
from the seeded generator; FP64 throughout.  N = 129^3 = 2,146,689 nodes.

One step = one full solve: condensed transformed right-hand side, BT conjugate
gradients to ||r~|| <= 1e-10 ||F^~||, back-transform of the skeleton and
recovery of the interior (all on the GPU; inputs resident in HBM).

value = N * iterations / solve time  [GDOF/s]: total unknowns times CG
iterations per second, i.e. the reciprocal of the time per DOF and iteration.
The CG launch (one launch per step, or one persistent cooperative launch) is
the one the library's autotuner picks for this problem.  The roofline is that
of the dominant kernel of the timed solves, from its algorithmic bytes and the
kernel time from HIP events the library records on the launch stream.  The
line also reports the solve with each launch kind forced, the mixed-precision
solve, the standalone apply kernel's rate and roofline, and the FP64 CPU
oracle's apply rate on this workload.

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


def cpu_baseline(wmesh, seconds=12.0):
    """Time the FP64 CPU oracle's condensed apply (explicit Schur complements,
    one GEMM per element class) on the same mesh, for about `seconds`."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle import mesh as M
    from oracle.operators import CondensedOperator

    op = CondensedOperator(M.make_mesh(**wmesh))
    u = W.random_skeleton_input(op.sizes["N"], k=1, seed=0)[0]
    op.apply(u)
    reps, t0 = 0, time.perf_counter()
    while True:
        op.apply(u)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or reps >= 2000:
            break
    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    return {"value": op.sizes["N"] * reps / dt / 1e9, "unit": "GDOF/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d oracle condensed applies (explicit Schur complement, one DGEMM per element "
                      "class; no CG vector work) on the same mesh, %.1f s, %s" % (reps, dt, cpu_model())}


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
        # the paper's BT iteration counts follow from Table 3 as solution time per
        # DOF / iteration time per DOF (upper bounds: the solution time includes
        # the precomputation).
        table3 = {8: (4.25, 25.6), 12: (3.73, 20.3), 16: (3.47, 17.7), 20: (3.31, 16.1), 24: (3.09, 14.4),
                  28: (2.88, 13.1), 32: (2.81, 12.4)}
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
            emit({"case": "element-count scaling (Sec. 8): expansion factor 1, p=16, lambda=0", "n_e": n ** 3,
                  "N": ctx.N, "iters": info[0]["iters"], "solve_ms": dt * 1e3,
                  "ns_per_dof_iter": dt / (ctx.N * info[0]["iters"]) * 1e9,
                  "max_rel_error_vs_exact": float(np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max())})
            del ft, gt, u
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_apply_config2_p8.md")
DOMINANT = "k_apply_tpt<double, 7, true, true>"
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
    (calibration), one timed-workload FP64 solve (its CG applies are the
    dominant kernel) and standalone applies."""
    import torch

    import workloads as W
    from paper_1601_08179_amd import semcond

    x = torch.randn(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)  # a plain streaming kernel: reads and writes COPY_BYTES
    torch.cuda.synchronize()
    wmesh, f = W.config2(k=1)
    ctx = semcond.Context(wmesh)
    ft = torch.tensor(f, device="cuda")
    u = torch.zeros_like(ft)
    ctx.solve(ft, out=u, tol=1e-10, persistent=False)
    torch.cuda.synchronize()
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
        # full applies only: launches queued after convergence exit at once and
        # read a few KiB (below a tenth of the median)
        for name, lst in rows.items():
            if name.startswith("void semcond::" + DOMINANT):
                vals = sorted(v for _, v in lst)
                full = [v for v in vals if v >= 0.1 * vals[len(vals) // 2]]
                return sum(full) / len(full), len(full)
        raise KeyError(DOMINANT)

    ff = COPY_BYTES / (copy_value(fe) * 1024.0)
    fw = COPY_BYTES / (copy_value(wr) * 1024.0)
    (fk, nf), (wk, nw) = dominant(fe), dominant(wr)
    fetch_b, write_b = fk * 1024.0 * ff, wk * 1024.0 * fw
    lines = [
        "# HBM traffic of %s (bench.py workload, FP64 CG apply, MI355X)" % DOMINANT,
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
        "| dominant kernel FETCH_SIZE per full dispatch (%d dispatches) | %.1f KiB |" % (nf, fk),
        "| dominant kernel WRITE_SIZE per full dispatch (%d dispatches) | %.1f KiB |" % (nw, wk),
        "| scaled HBM read bytes per launch | %.0f |" % fetch_b,
        "| scaled HBM write bytes per launch | %.0f |" % write_b,
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--apply-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--suite", default="", help="extra measurements instead of the default line: "
                    "any of 3 (p/AR sweep), 4 (16 RHS), 5 (differentiable solve), D (the paper's "
                    "solver experiment with inhomogeneous Dirichlet values), S (its element-count "
                    "scaling), e.g. --suite 345DS")
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
        print("bench.py measures one GPU only; multi-GPU runs are not part of this build "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
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

    wmesh, f = W.config2(k=1)
    ctx = semcond.Context(wmesh)
    ft = torch.tensor(f, device="cuda")
    u = torch.zeros_like(ft)
    N, Ns = ctx.N, ctx.N_s

    # CG launch choice for (k = 1, FP64): one launch per step or a persistent grid
    tS, tG = ctx.autotune(k=1, dtype=torch.float64)
    for _ in range(args.warmup):
        ctx.solve(ft, out=u, tol=args.tol)
    torch.cuda.synchronize()

    # ---- timed region: K full solves with the tuned CG launch ------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(args.steps):
        _, info = ctx.solve(ft, out=u, tol=args.tol)
        iters += info[0]["iters"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    solve_s = (t1 - t0) / args.steps
    it_per_solve = iters / args.steps
    value = N * iters / (t1 - t0) / 1e9

    # ---- kernel times of the same solves: HIP events around every apply / persistent
    # CG launch on the launch stream (a separate pass: the events cost a few us each)
    side_steps = max(3, args.steps // 4)
    ctx.profile_enable(True)
    for _ in range(side_steps):
        ctx.solve(ft, out=u, tol=args.tol)
    ap_ms, ap_launches, _ = ctx.profile_read(semcond.KERNEL_APPLY)
    cg_ms, cg_launches, cg_iters = ctx.profile_read(semcond.KERNEL_PCG)
    ctx.profile_enable(False)

    # ---- the same solves with each launch kind forced --------------------------------

    def timed(**kw):
        ctx.solve(ft, out=u, tol=args.tol, **kw)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(side_steps):
            _, inf = ctx.solve(ft, out=u, tol=args.tol, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - ta) / side_steps, inf

    step_s, _ = timed(persistent=False)
    pers_s, _ = timed(persistent=True)
    # FP32 inner CG + FP64 iterative refinement
    mixed_s, minfo = timed(precision=semcond.PREC_MIXED_IR)

    # ---- apply alone (transformed basis, back-to-back), kernel time from events ------
    xs = torch.randn(Ns, dtype=torch.float64, device="cuda")
    ys = torch.empty_like(xs)
    for _ in range(10):
        ctx.apply(xs, out=ys)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    for _ in range(args.apply_reps):
        ctx.apply(xs, out=ys)
    pa_ms, pa_launches, _ = ctx.profile_read(semcond.KERNEL_APPLY)
    ctx.profile_enable(False)
    kern_s = pa_ms / 1e3 / max(pa_launches, 1)
    # the same apply with a cold last-level cache: 512 MiB written between launches
    flush = torch.empty((512 << 20) // 8, dtype=torch.float64, device="cuda")
    ctx.profile_enable(True)
    for rep in range(20):
        flush.fill_(float(rep))
        ctx.apply(xs, out=ys)
    pc_ms, pc_launches, _ = ctx.profile_read(semcond.KERNEL_APPLY)
    ctx.profile_enable(False)
    cold_s = pc_ms / 1e3 / max(pc_launches, 1)
    # STREAM-style copy on this GPU (1 GiB read + 1 GiB written), next to the nominal peak
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
    copy_gbs = 2 * ca.numel() * 8 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del flush, ca, cb

    # Roofline of the dominant kernel of the timed solves.  Algorithmic FP64 bytes
    # (k = 1): the CG apply gathers p, r and P^-1 (it forms the direction) and
    # produces q: 4 N_s (its per-side slot stores are an implementation choice and
    # show in the counter traffic, not here); the persistent CG per iteration
    # moves 13 N_s (apply 4; step: reads r, q, P^-1, p, x and writes q, p, x, r).
    if cg_ms >= ap_ms:
        dom = {"kernel": "k_pcg_persistent<double,7,%d>" % tS, "ms": cg_ms, "launches": cg_launches,
               "bytes": 13 * 8 * Ns * cg_iters, "traffic": None}
    else:
        # one full apply per CG iteration; the launches queued after convergence
        # leave at once, their (small) time stays in the total
        full = int(round(it_per_solve * side_steps))
        dom = {"kernel": "k_apply_tpt<double,7,true,true>", "ms": ap_ms, "launches": full,
               "bytes": 4 * 8 * Ns * full, "traffic": stored_traffic(), "early_exit_launches": ap_launches - full}
    dom_achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
    apply_bytes = 2 * 8 * Ns
    apply_achieved = apply_bytes / kern_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": solve_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "BT solve to 1e-10: 16^3 uniform elements, p=8, lambda=1e-3, unit cube, "
                               "Dirichlet, one N(0,1) nodal RHS (seeded)",
                   "p": 8, "n_e": ctx.n_e, "N": N, "N_s": Ns, "k": 1, "tol": args.tol,
                   "parallelism": "single GPU"},
        "iterations": it_per_solve,
        "ns_per_dof_iter": solve_s / (N * it_per_solve) * 1e9,
        "cg_launch": {"tuned": "stepwise" if tS == 0 else "persistent S=%d G=%d" % (tS, tG),
                      "stepwise_ms_per_solve": step_s * 1e3, "persistent_ms_per_solve": pers_s * 1e3},
        "mixed_ir": {"ms_per_solve": mixed_s * 1e3, "speedup_vs_fp64": solve_s / mixed_s,
                     "inner_iterations": minfo[0]["iters"], "outer_steps": minfo[0]["outer"],
                     "rel_res": minfo[0]["rel_res"]},
        "roofline": {"bound": "hbm", "achieved": dom_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom_achieved / HBM_PEAK_GBS, "traffic": dom["traffic"],
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": dom["kernel"], "launches": dom["launches"],
                     "bytes_per_launch": dom["bytes"] / max(dom["launches"], 1),
                     "kernel_us_per_launch": dom["ms"] * 1e3 / max(dom["launches"], 1),
                     "early_exit_launches": dom.get("early_exit_launches", 0),
                     "copy_gbs_measured": copy_gbs, "frac_of_measured_copy": dom_achieved / copy_gbs},
        "apply_roofline": {"bound": "hbm", "achieved": apply_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": apply_achieved / HBM_PEAK_GBS, "kernel": "k_apply_tpt<double,7,false,false>",
                           "kernel_us": kern_s * 1e6, "gdof_s": N / kern_s / 1e9,
                           "bytes_per_launch": apply_bytes, "cold_cache_kernel_us": cold_s * 1e6,
                           "cold_cache_frac": apply_bytes / cold_s / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wmesh, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
