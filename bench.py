#!/usr/bin/env python3
"""Benchmark: solve to 1e-8 true relative residual, FP64 vs mixed precision,
on the 4,194,304-DOF layered-battery system (128x128x64 cells, 4 fields).

One step = the whole hot path on one synthetic system already resident in
HBM: device setup of the preconditioner from the CSR values (block split,
strength, MIS-2 aggregation, prolongator smoothing, Galerkin products,
coarsest factor), the mixed-precision forward solve, the FP64 forward solve,
the mixed-precision adjoint solve and the value gradient.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve s to 1e-8 rel resid (fp64 vs mixed), V-cycle HBM GB/s, at 4.2M DOF"
HBM_PEAK_GBS = 8000.0
VCYCLE_KINDS = ("cheb_pre", "cheb_post_a", "cheb_post_b", "cheb_other", "resid", "restrict", "prolong", "coarse",
                "couple", "cheb_pre_c", "cheb_post_a_c", "cheb_post_b_c", "cheb_other_c", "resid_c", "restrict_c",
                "prolong_c")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="layered-battery configuration (default: 4.2M DOF)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the preconditioner variants and sweeps")
    ap.add_argument("--protocol-reps", type=int, default=None,
                    help="repetitions of each solve in the timing protocol after the timed steps (the first is "
                         "discarded; default 100, 5 on the 50.3M-DOF system)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the solver is single-device and has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_13079_amd as H
    import synth

    dev = torch.device("cuda:0")
    t = time.time()
    s = synth.make_system(cfg=args.config)
    log(f"system: n={s.n} nnz={s.nnz} fields={s.nf} ({time.time() - t:.1f}s to generate)")
    rp, ci, val, fl = (torch.from_numpy(a).to(dev) for a in (s.rowptr, s.col, s.val, s.field_of_row))
    b = torch.from_numpy(s.b).to(dev)
    xt = torch.from_numpy(s.x_t).to(dev)
    solver = H.Solver(rp, ci, val, fl, s.nf, s.tree, precision=1)
    st0 = solver.stats()
    log("levels", st0["levels"], "rows", st0["rows"])

    def step(prof_kinds=None):
        """One pass of the hot path.  prof_kinds: kernel classes to time with
        events during the mixed forward solve only (None: no timing)."""
        r = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.set_values(val)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        solver.set_precision(1)
        if prof_kinds is not None:
            solver.profile(True, kinds=prof_kinds)
        x, stm, itm, hm = solver.solve(b)
        if prof_kinds is not None:
            r["kernel_times"] = solver.kernel_times()
            solver.profile(False)
        t2 = time.perf_counter()
        solver.set_precision(0)
        x64, st64, it64, h64 = solver.solve(b)
        t3 = time.perf_counter()
        solver.set_precision(1)
        lam, sta, ita, _ = solver.solve(x - xt, transpose=True)
        t4 = time.perf_counter()
        solver.set_precision(0)
        lam64, sta64, ita64, _ = solver.solve(x64 - xt, transpose=True)
        t5 = time.perf_counter()
        g = solver.grad_values(lam, x)
        torch.cuda.synchronize()
        t6 = time.perf_counter()
        assert stm == 0 and st64 == 0 and sta == 0 and sta64 == 0, (stm, st64, sta, sta64)
        r.update(setup_s=t1 - t0, mixed_s=t2 - t1, fp64_s=t3 - t2, adjoint_s=t4 - t3, adjoint64_s=t5 - t4,
                 grad_s=t6 - t5, it_mixed=itm, it_fp64=it64, it_adjoint=ita, it_adjoint64=ita64,
                 res_mixed=hm[-1], res_fp64=h64[-1],
                 err_mixed_vs_fp64=float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64)),
                 err_adjoint_mixed_vs_fp64=float(torch.linalg.norm(lam - lam64) / torch.linalg.norm(lam64)),
                 grad_finite=bool(torch.isfinite(g).all()))
        return r

    # plain device copy of a known size: the practical HBM ceiling, and the
    # reference kernel that scales the PMC byte counters
    copy_gbs = copy_probe(torch, dev)
    log(f"copy probe: {copy_gbs:.1f} GB/s")

    # warmup; the first warmup step times every kernel class of the mixed solve
    prof_steps = []
    for w in range(max(1, args.warmup)):
        r = step(prof_kinds=list(solver.kernel_times()) if w == 0 else None)
        if w == 0:
            kt = r.pop("kernel_times")
        log(f"warmup {w}: " + ", ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}" for k, v in r.items()))
        prof_steps.append(r)
    # the dominant kernel class ("sweep" times a whole preconditioner
    # application, many kernels, and is not a candidate)
    tot_ms = {k: v["ms"] for k, v in kt.items() if k != "sweep"}
    dominant = max(tot_ms, key=tot_ms.get)
    vc_ms = sum(kt[k]["ms"] for k in VCYCLE_KINDS)
    vc_bytes = sum(kt[k]["bytes"] for k in VCYCLE_KINDS)
    log("kernel classes (mixed solve of the first warmup step, launches timed one by one):")
    for k, v in sorted(kt.items(), key=lambda kv: -kv[1]["ms"]):
        if v["launches"]:
            log(f"  {k:14s} {v['ms']:9.3f} ms {v['launches']:7d} launches "
                f"{v['bytes'] / max(v['ms'], 1e-9) / 1e6:8.1f} GB/s")

    # timed region.  Every launch of the dominant class and of the outer SpMV
    # in the mixed solves is timed with HIP events on the stream it runs on
    # (stamped by the dispatch for the outer SpMV, event records around it
    # otherwise); the other classes are not timed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed_kinds = list(dict.fromkeys([dominant, "spmv_outer"]))
    rs = [step(prof_kinds=timed_kinds) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dk = dict(ms=0.0, launches=0, bytes=0.0)
    so = dict(ms=0.0, launches=0, bytes=0.0)
    for r in rs:
        kts = r.pop("kernel_times")
        for key in dk:
            dk[key] += kts[dominant][key]
            so[key] += kts["spmv_outer"][key]
    # whole preconditioner applications, event-timed (before the sweep's fork
    # and after its join) in mixed solves after the timed region, so that
    # their events do not weigh on the timed solves
    solver.set_precision(1)
    solver.profile(True, kinds=["sweep"])
    for _ in range(max(3, args.steps)):
        solver.solve(b)
    sw = solver.kernel_times()["sweep"]
    solver.profile(False)
    for i, r in enumerate(rs):
        log(f"step {i}: " + ", ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}" for k, v in r.items()))
    log(f"timed steps: {dominant}: {dk['launches']} launches, {dk['ms']:.3f} ms")

    def mean(k):
        return float(np.mean([r[k] for r in rs]))

    def std(k):
        return float(np.std([r[k] for r in rs], ddof=1)) if len(rs) > 1 else 0.0

    # V-cycle bandwidth: preconditioner applies in mixed precision
    solver.set_precision(1)
    v0 = torch.randn(s.n, dtype=torch.float64, device=dev)
    for _ in range(3):
        solver.apply(v0)
    torch.cuda.synchronize()
    napply = 20
    ta = time.perf_counter()
    for _ in range(napply):
        solver.apply(v0)
    torch.cuda.synchronize()
    apply_s = (time.perf_counter() - ta) / napply
    st = solver.stats()
    vbytes = st["vcycle_bytes"][1]

    achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9 if dk["ms"] > 0 else 0.0
    traffic, traffic_src = measured_traffic(dominant, round(dk["bytes"] / max(dk["launches"], 1)))
    out = {
        "metric": METRIC,
        "value": round(mean("mixed_s"), 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 GMRES + f32 V-cycle (mixed); f64 reference solve",
        "data": "synthetic",
        "config": {
            "workload": f"layered-battery FV system {'x'.join(str(d) for d in s.dims if d)} cells, {s.nf} fields, "
                        f"{s.n} DOF, {s.nnz} nnz; GMRES({solver.opts.restart}) to 1e-8 true relative residual, "
                        f"block lower Gauss-Seidel with one SA-AMG V-cycle per field",
            "n_dof": s.n, "nnz": s.nnz, "fields": s.nf, "seed": s.seed,
        },
        "mixed_solve_s": round(mean("mixed_s"), 6),
        "mixed_solve_s_std": round(std("mixed_s"), 6),
        "fp64_solve_s": round(mean("fp64_s"), 6),
        "fp64_solve_s_std": round(std("fp64_s"), 6),
        "mixed_speedup_vs_fp64": round(mean("fp64_s") / mean("mixed_s"), 3),
        "iters_mixed": int(rs[-1]["it_mixed"]),
        "iters_fp64": int(rs[-1]["it_fp64"]),
        "ms_per_iter_mixed": round(mean("mixed_s") / rs[-1]["it_mixed"] * 1e3, 4),
        "ms_per_iter_fp64": round(mean("fp64_s") / rs[-1]["it_fp64"] * 1e3, 4),
        "true_res_mixed": float(rs[-1]["res_mixed"]),
        "true_res_fp64": float(rs[-1]["res_fp64"]),
        "err_mixed_vs_fp64": float(rs[-1]["err_mixed_vs_fp64"]),
        "setup_s": round(mean("setup_s"), 4),
        "setup_s_std": round(std("setup_s"), 4),
        "setup_stage_s": dict(zip(("extract", "aggregation", "prolongator", "transpose_P", "galerkin", "coarse_lu",
                                   "smoother_data", "solve_data"), (round(x, 4) for x in st["setup_stage_seconds"]))),
        "setup_field_s": [round(x, 4) for x in st["setup_field_seconds"]],
        "adjoint_mixed_s": round(mean("adjoint_s"), 6),
        "adjoint_mixed_s_std": round(std("adjoint_s"), 6),
        "adjoint_fp64_s": round(mean("adjoint64_s"), 6),
        "adjoint_fp64_s_std": round(std("adjoint64_s"), 6),
        "iters_adjoint": int(rs[-1]["it_adjoint"]),
        "iters_adjoint_fp64": int(rs[-1]["it_adjoint64"]),
        "err_adjoint_mixed_vs_fp64": float(rs[-1]["err_adjoint_mixed_vs_fp64"]),
        "copy_gbs": round(copy_gbs, 1),
        "grad_s": round(mean("grad_s"), 6),
        "vcycle_gbs_kernels": round(vc_bytes / (vc_ms * 1e-3) / 1e9, 1) if vc_ms > 0 else None,
        "vcycle_gbs_sweep": round(sw["bytes"] / (sw["ms"] * 1e-3) / 1e9, 1) if sw["ms"] > 0 else None,
        "vcycle_frac_sweep": round(sw["bytes"] / (sw["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if sw["ms"] > 0 else None,
        "vcycle_us_sweep": round(sw["ms"] / max(sw["launches"], 1) * 1e3, 2),
        "spmv_outer_gbs": round(so["bytes"] / (so["ms"] * 1e-3) / 1e9, 1) if so["ms"] > 0 else None,
        "spmv_outer_frac": round(so["bytes"] / (so["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if so["ms"] > 0 else None,
        "spmv_outer_us": round(so["ms"] / max(so["launches"], 1) * 1e3, 2),
        "vcycle_gbs_apply": round(vbytes / apply_s / 1e9, 1),
        "vcycle_frac_apply": round(vbytes / apply_s / 1e9 / HBM_PEAK_GBS, 4),
        "apply_ms_mixed": round(apply_s * 1e3, 4),
        "levels": st["levels"],
        "roofline": {
            "kernel": dominant,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "launches": dk["launches"],
            "avg_launch_us": round(dk["ms"] / max(dk["launches"], 1) * 1e3, 3),
            "bytes_per_launch": round(dk["bytes"] / max(dk["launches"], 1)),
            "traffic_source": traffic_src,
        },
    }
    reps = args.protocol_reps if args.protocol_reps is not None else (5 if s.n > 10_000_000 else 100)
    if reps > 1:
        out["protocol"] = protocol(solver, b, xt, reps)
    if not args.no_variants:
        out["variants"] = variants(H, torch, s, rp, ci, val, fl, b)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


def protocol(solver, b, xt, reps):
    """The paper's timing protocol (Sec. 4: repeated runs, the first
    discarded, mean and standard deviation) on each solve of the step, with
    the preconditioner kept: `reps` solves each, the first dropped."""
    import numpy as np
    import torch
    out = {"repetitions": reps, "discarded": 1}
    for name, prec, tr in (("mixed", 1, False), ("fp64", 0, False), ("adjoint_mixed", 1, True),
                           ("adjoint_fp64", 0, True)):
        solver.set_precision(prec)
        rhs = xt if tr else b
        ts, its = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, it, _ = solver.solve(rhs, transpose=tr)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            its.append(it)
        ts = np.array(ts[1:])
        out[name] = {"mean_s": round(float(ts.mean()), 6),
                     "std_s": round(float(ts.std(ddof=1)) if len(ts) > 1 else 0.0, 6),
                     "min_s": round(float(ts.min()), 6), "iters": its[-1],
                     "ms_per_iter": round(float(ts.mean()) / its[-1] * 1e3, 4)}
        log(f"protocol {name}: {out[name]}")
    solver.set_precision(1)
    return out


def variants(H, torch, s, rp, ci, val, fl, b, reps=3):
    """Other configurations of the method on the same system (each a fresh
    setup, then the mean of `reps` mixed-precision solves to 1e-8):
      * nested: the paper's nested form -- outer flexible GMRES(5); the
        voltage block (phi_s, phi_e) and the non-voltage block (p, c...) each
        solved by an inner GMRES(30) to 1e-6 preconditioned by its own sweep,
        degree-4 Chebyshev on the voltage leaves;
      * block_jacobi: couplings dropped, all field V-cycles concurrent;
      * theta_phi_s: strength threshold of the phi_s hierarchy;
      * cheb_degree_4: degree-4 Chebyshev on every level of every field;
      * species_ilu0 / species_jacobi: the species leaves solved by DD(0)-ILU(0)
        (4096-row subdomains) or one Jacobi sweep instead of SA-AMG."""
    nsp = s.nf - 3
    tree2 = [-1, -1, 0, 1, -2, -1] + list(range(2, 3 + nsp)) + [-2, -2]
    cases = {
        "nested": dict(tree=tree2, nested=1, restart=5, field_cheb_degree=[4, 4]),
        "block_jacobi": dict(block_jacobi=1),
        "cheb_degree_4": dict(cheb_degree=4),
        "species_ilu0": dict(field_leaf=[0, 0, 0] + [2] * nsp, ilu_block=4096),
        "species_jacobi": dict(field_leaf=[0, 0, 0] + [1] * nsp),
    }
    for th in (0.0, 0.01, 0.04, 0.16, 0.64):
        cases[f"theta_phi_s={th}"] = dict(theta=[th])
    out = {}
    for name, opt in cases.items():
        opt = dict(opt)
        tree = opt.pop("tree", s.tree)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            g = H.Solver(rp, ci, val, fl, s.nf, tree, precision=1, **opt)
        except H.HBGSError as e:  # e.g. coarsening stalls above the dense coarse-solve limit
            out[name] = dict(error=str(e))
            log(f"variant {name}: {e}")
            continue
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        times, its = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            x, st, it, hist = g.solve(b)
            times.append(time.perf_counter() - t0)
            its.append(it)
        xa, sta, ita, _ = g.solve(b, transpose=True)
        out[name] = dict(setup_s=round(setup_s, 4), solve_s=round(min(times), 6), iters=its[-1], status=st,
                         true_res=float(hist[-1]), levels=g.stats()["levels"], adjoint_iters=ita,
                         adjoint_status=sta)
        log(f"variant {name}: setup {setup_s:.3f}s, solve {min(times) * 1e3:.2f} ms, {its[-1]} iterations, "
            f"levels {out[name]['levels']}, adjoint {ita} iterations")
        del g
    return out


def copy_probe(torch, dev, mib=512, reps=5):
    """y = -x over `mib` MiB of float32 (read once, written once); returns GB/s
    of the best of `reps` launches."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.neg(x, out=y)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del x, y
    return 2 * n * 4 / best / 1e9


def measured_traffic(kind, alg_bytes):
    """HBM bytes per launch of the `kind` kernel from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading for
    the copy probe of known size), or None when no summary covers this kind
    on this workload (its algorithmic bytes per launch, `alg_bytes`, differ)
    or the solve kernels have changed since it was taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2602_13079_amd", "csrc", "solve_kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "pmc_*.md"))):
        text = open(path).read()
        if "```json" not in text:
            continue
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if rec.get("kind") != kind or rec.get("algorithmic_bytes_per_launch") != alg_bytes:
            continue
        if rec.get("solve_kernels_sha256") != digest:
            return None, f"{os.path.relpath(path, ROOT)} is stale (solve kernels changed since)"
        return round(rec["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, "no PMC summary for this kernel class on this workload"


def cpu_baseline(s, reps=3):
    """The CPU oracle (plain loops; OpenMP over rows and element-wise work
    with sequential reductions, so every thread count gives the same bits)
    on the same system: `reps` mixed-precision solves to 1e-8 with every
    thread of the process's CPU share (OMP_NUM_THREADS, else os.cpu_count()),
    then `reps` with one thread; the setup (all threads) is timed apart."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    oracle.set_threads(threads)
    t = time.perf_counter()
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, precision=1)
    setup_s = time.perf_counter() - t
    runs = {}
    for nth in (threads, 1):
        oracle.set_threads(nth)
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            r = o.solve(s.b)
            ts.append(time.perf_counter() - t)
        runs[nth] = (np.array(ts), r["iters"])
        log(f"cpu oracle, {nth} thread(s): mixed solve {np.mean(ts):.2f} +- {np.std(ts):.2f} s, {r['iters']} iterations")
    oracle.set_threads(threads)
    ts, iters = runs[threads]
    ts1, _ = runs[1]
    return {"value": round(float(ts.mean()), 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"the full {s.n}-DOF system: mixed-precision solves to 1e-8 ({iters} iterations), "
                      f"{reps} with {threads} threads and {reps} with one; the oracle setup "
                      f"({setup_s:.2f} s with {threads} threads) not included",
            "std": round(float(ts.std(ddof=1)), 3) if reps > 1 else 0.0,
            "single_thread_s": round(float(ts1.mean()), 3),
            "single_thread_std": round(float(ts1.std(ddof=1)), 3) if reps > 1 else 0.0,
            "repetitions": reps, "setup_s": round(setup_s, 3), "iters": iters,
            "os_cpu_count": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


if __name__ == "__main__":
    main()
