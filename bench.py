"""Benchmark of the HSS-ULV factorization + solve on one MI355X.

Workload (default): N = 262144 points uniform in the unit cube, Matern nu=3/2
kernel with length 0.2 plus 1e-6 on the diagonal, leaf 256 (10 levels), rank
96, one N(0,1) right-hand side; the HSS matrix is built on the GPU (scaled
randomized compression, untimed). A step is one factorization + one solve
(plus the refinement corrections and their FP64 matvecs for the mixed form).

Prints ONE JSON line. `value` is seconds per factor+solve (lower is better).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0




def step_flops(step, n, r):
    """Algorithmic flops of one node for one profiled kernel launch class."""
    m = n - r
    table = {
        "gemm_W=MY": 2.0 * n * n * r,
        "gemm_F_update": 2.0 * n * (n + 1) * r,  # lower triangle of M - Z V^T - V Z^T
        "gemm_Y=VT": 2.0 * n * r * r,
        "gemm_C=YtW": 2.0 * n * r * r,
        "gemm_Z": 2.0 * n * r * r,
        "gemm_V2": 2.0 * m * r * r,
        "basis_top": 5.0 / 3.0 * r ** 3,  # LU of the top block, two triangular inverses, T
        "pchol_RR": m ** 3 / 3.0,
        "sr_schur": r * m * m + r * r * m,
        "pchol": m ** 3 / 3.0 + r * m * m + r * r * m,
        "chol_lds": 2.0 * m ** 3 / 3.0,  # Cholesky and explicit inverse
        "gemm_LSR": 2.0 * r * m * m,
        "gemm_Sigma": 2.0 * r * r * m,
        "root": n ** 3 / 3.0,
    }
    return table.get(step, 0.0)


def step_bytes(step, n, r):
    """Algorithmic HBM bytes of one node (each operand read once, result written once)."""
    m = n - r
    if step == "merge":
        return 8.0 * 2 * n * n
    if step in ("solve_forward", "solve_backward"):
        return 8.0 * (2 * n * r + m * (m + 1) / 2 + r * m + 2 * n)
    if step == "copy_lsr":
        return 8.0 * 2 * r * m
    return 0.0


# position of each GEMM label in a stage's list of GEMM batches (the library's plan order)
GEMM_STEP_INDEX = {"gemm_V2": 0, "gemm_Y=VT": 2, "gemm_W=MY": 3, "gemm_C=YtW": 4, "gemm_Z": 5, "gemm_F_update": 6,
                   "gemm_LSR": 7, "gemm_Sigma": 8}

FACTOR_STEPS = ("gemm_W=MY", "gemm_F_update", "gemm_Y=VT", "gemm_C=YtW", "gemm_Z", "gemm_V2", "basis_top",
                "pchol_RR", "sr_schur", "pchol", "chol_lds", "gemm_LSR", "gemm_Sigma", "root")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="matern32_n262144")
    ap.add_argument("--rank", type=int, default=0, help="override the workload's fixed rank (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-system batched leg")
    ap.add_argument("--no-tune", action="store_true", help="skip autotuning and graph replay")
    ap.add_argument("--save-tiles", default="", help="write the tuned GEMM tile choice to this JSON file")
    ap.add_argument("--load-tiles", default="", help="use the GEMM tile choice saved in this JSON file")
    ap.add_argument("--no-graph", action="store_true", help="time the tuned configuration with eager launches")
    ap.add_argument("--no-fused", action="store_true", help="skip the one-call factor + solve")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision legs (FP32 and BF16 forms + refinement)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-rank ablation leg")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the 16-right-hand-side leg (HSS-ULV and BLR^2-ULV at N = 65536)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling hardware byte counters) and exit")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the one-GPU scaling sweeps (N and leaf size) and print them as one JSON line")
    ap.add_argument("--table2", action="store_true",
                    help="only run the Table 2 accuracy leg (Eq. 18-19 on the 256 x 256 grid) and print it")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the oracle's factor + solve on the whole exported HSS matrix of the workload "
                         "(all host threads, then one thread) and print it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2311_00921_amd import hss

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        nel = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nel * 8, "copy_bytes_written": nel * 8}))
        return
    if args.sweep:
        ctx = hss.hss_ctx_create(0)
        print(json.dumps({"sweep": sweep_leg(hss, torch, np, ctx, args.steps, args.warmup)}))
        hss.hss_ctx_destroy(ctx)
        return
    if args.table2:
        ctx = hss.hss_ctx_create(0)
        print(json.dumps({"table2": table2_leg(hss, torch, np, ctx)}))
        hss.hss_ctx_destroy(ctx)
        return
    w = synth.WORKLOADS[args.workload]
    if args.rank:
        import dataclasses

        w = dataclasses.replace(w, name=f"{w.name}_r{args.rank}", rank=args.rank)
    s = (w.rank if w.rank > 0 else 128) + w.oversample
    X = torch.from_numpy(w.points()).cuda()
    Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
    b = torch.from_numpy(np.ascontiguousarray(w.rhs()[:, 0])).cuda()
    ctx = hss.hss_ctx_create(0)
    print(f"# building HSS: N={w.n} leaf={w.leaf} rank={w.rank} s={s}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = hss.hss_construct(ctx, X, w.kernel, w.leaf, rank=w.rank, tol=w.tol, omega=Om, length=w.length,
                          nugget=w.nugget)
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    del Om
    print(f"# construct {construct_s:.2f} s", file=sys.stderr, flush=True)

    exp = hss.hss_export(ctx, m)
    if args.cpu_full:
        hss.hss_ulv_factor(ctx, m)
        x_gpu = hss.hss_ulv_solve(ctx, m, b).cpu().numpy()
        ld_gpu = hss.hss_logdet(ctx, m)
        hss.hss_matrix_destroy(m)
        hss.hss_ctx_destroy(ctx)
        print(json.dumps({"cpu_full": cpu_full(exp, w, b.cpu().numpy(), x_gpu, ld_gpu)}))
        return
    L = exp["levels"]
    leaf_lo = exp["leaf_lo"]
    rank = exp["rank"]
    nodes = []  # (heap index, level, n, r)
    for k in range(2 ** (L + 1) - 1):
        l = int(math.floor(math.log2(k + 1)))
        if l == L:
            i = k - (2 ** L - 1)
            n = int(leaf_lo[i + 1] - leaf_lo[i])
        else:
            n = int(rank[2 * k + 1] + rank[2 * k + 2])
        nodes.append((k, l, n, int(rank[k]) if k > 0 else 0))

    def run_fp64(steps, profile=False):
        if profile:
            hss.hss_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x = None
        for _ in range(steps):
            hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP64)
            x = hss.hss_ulv_solve(ctx, m, b)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        prof = hss.hss_profile_read(ctx) if profile else None
        if profile:
            hss.hss_profile_enable(ctx, False)
        return dt, x, prof

    for _ in range(args.warmup):
        run_fp64(1)
    print("# timing FP64 factor+solve", file=sys.stderr, flush=True)
    t_fp64, x, _ = run_fp64(args.steps)
    # relative residual with the FP64 HSS matvec
    r = b - hss.hss_matvec(ctx, m, x)
    relres = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    logdet = hss.hss_logdet(ctx, m)
    info = hss.hss_get_info(m)
    # library's tuned mode: autotuned GEMM tiles (or a saved choice), factor and solve replayed from HIP graphs
    tuned = None
    t_best = t_fp64
    tile_choice = None
    if args.load_tiles:
        with open(args.load_tiles) as f:
            hss.hss_set_gemm_variants(ctx, m, json.load(f)["tile_choice"], hss.HSS_P_FP64)
        rep = None
    elif not args.no_tune:
        print("# autotuning GEMM tiles (FP64)", file=sys.stderr, flush=True)
        rep = hss.hss_autotune(ctx, m, hss.HSS_P_FP64, 4)
    if args.load_tiles or not args.no_tune:
        tile_choice = hss.hss_gemm_variants(m, hss.HSS_P_FP64)
        if args.save_tiles:
            with open(args.save_tiles, "w") as f:
                json.dump({"workload": w.name, "tile_choice": tile_choice}, f)
        for _ in range(args.warmup):
            run_fp64(1)
        print("# timing FP64 factor+solve (tuned, eager launches)", file=sys.stderr, flush=True)
        t_tuned, xg, _ = run_fp64(args.steps)
        t_eager = t_tuned
        t_graph = None
        if not args.no_graph:
            hss.hss_use_graphs(ctx, m, True)
            for _ in range(args.warmup):
                run_fp64(1)
            print("# timing FP64 factor+solve (tuned, graph replay)", file=sys.stderr, flush=True)
            t_graph, xgg, _ = run_fp64(args.steps)
            if t_graph < t_tuned:
                t_tuned, xg = t_graph, xgg
            hss.hss_use_graphs(ctx, m, False)
        # one call for both: each stage's forward sweep overlaps the factorization of the stages above
        t_fused = None
        if not args.no_fused:
            def run_fused(steps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                xx = None
                for _ in range(steps):
                    xx = hss.hss_ulv_factor_solve(ctx, m, b)
                torch.cuda.synchronize()
                return (time.perf_counter() - t) / steps, xx

            for _ in range(args.warmup):
                run_fused(1)
            print("# timing FP64 fused factor+solve (tuned)", file=sys.stderr, flush=True)
            t_fused, xf = run_fused(args.steps)
            rf = b - hss.hss_matvec(ctx, m, xf)
            if float(torch.linalg.norm(rf) / torch.linalg.norm(b)) <= 1e-8 and t_fused < t_tuned:
                t_tuned, xg = t_fused, xf
        rg = b - hss.hss_matvec(ctx, m, xg)
        relres_g = float(torch.linalg.norm(rg) / torch.linalg.norm(b))
        tuned = {"factor_plus_solve_s": round(t_tuned, 6), "eager_launches_s": round(t_eager, 6),
                 "graph_replay_s": round(t_graph, 6) if t_graph else None,
                 "fused_factor_solve_s": round(t_fused, 6) if t_fused else None,
                 "relres": relres_g,
                 "rel_diff_x_vs_eager": float(torch.linalg.norm(xg - x) / torch.linalg.norm(x)),
                 "gemm_ms_per_factor_by_tile": dict(zip(list(hss.GEMM_TILES) + ["tuned"], rep)) if rep else None,
                 "tile_choice": tile_choice}
        if relres_g <= 1e-8:
            t_best = min(t_best, t_tuned)
    # per-launch events over a further timed region of the same configuration (graphs are bypassed while
    # profiling): the dominant kernel's average launch duration
    t_prof, _, prof = run_fp64(args.steps, profile=True)
    by_step = {}
    for (step, lvl), (cnt, ms) in prof.items():
        by_step.setdefault(step, 0.0)
        by_step[step] += ms
    # the dominant kernel: the (kernel, level) with the largest summed event time; one launch per (kernel, level)
    cands = {k: v for k, v in prof.items() if k[1] >= 0 and (k[0] in FACTOR_STEPS or step_bytes(k[0], 2, 1) > 0)}
    dom_key = max(cands.items(), key=lambda kv: kv[1][1])[0]
    dom_step, dom_level = dom_key
    cnt, ms_total = prof[dom_key]
    avg_ms = ms_total / cnt
    lvl_nodes = [nd for nd in nodes if nd[1] == dom_level and (nd[3] > 0 or dom_step == "root")]
    flops = sum(step_flops(dom_step, n, rr) for _, _, n, rr in lvl_nodes)
    byts = sum(step_bytes(dom_step, n, rr) for _, _, n, rr in lvl_nodes)
    if dom_step in FACTOR_STEPS:
        ach = flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": MFMA_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / MFMA_FP64_PEAK_TFLOPS, 4), "traffic": None}
    else:
        ach = byts / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    tile = None
    if dom_step in GEMM_STEP_INDEX and tile_choice is not None:
        tile = hss.GEMM_TILES[tile_choice[(L - dom_level) * 9 + GEMM_STEP_INDEX[dom_step]]]
    elif dom_step in GEMM_STEP_INDEX:
        tile = hss.GEMM_TILES[0]
    roof.update({"kernel": f"{dom_step}@level{dom_level}", "tile": tile, "avg_launch_ms": round(avg_ms, 4),
                 "algorithmic_per_launch": flops if roof["unit"] == "TFLOP/s" else byts})
    roof["traffic"] = measured_traffic(f"{dom_step}@level{dom_level}", w.name, tile)
    # mixed form: FP32 factorization + refinement with the FP64 HSS matvec to rel. residual 1e-8
    mixed = None
    try:
        if args.no_mixed:
            raise RuntimeError("skipped (--no-mixed)")
        def run_mixed(steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = None
            for _ in range(steps):
                hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP32)
                out = hss.hss_ulv_solve_refined(ctx, m, b, 1e-8, 50)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / steps, out

        # the first mixed factorization of the matrix decides which leaves the FP32
        # products are accurate enough for (the rest are redone in FP64)
        hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP32)
        first = hss.hss_get_info(m)
        first_promoted, first_ms = int(first.promoted_nodes), round(first.factor_ms, 3)
        if not args.no_tune:
            hss.hss_autotune(ctx, m, hss.HSS_P_FP32, 2)
        for _ in range(args.warmup):
            run_mixed(1)
        print("# timing mixed factor+refined solve", file=sys.stderr, flush=True)
        t_mixed, (xm, iters, rr_m, ok_m) = run_mixed(args.steps)
        minfo = hss.hss_get_info(m)
        rr_check = float(torch.linalg.norm(b - hss.hss_matvec(ctx, m, xm)) / torch.linalg.norm(b))
        err_vs_fp64 = float(torch.linalg.norm(xm - x) / torch.linalg.norm(x))
        logdet32 = hss.hss_logdet(ctx, m)
        leaves = 2 ** L
        mixed = {"factor_plus_refined_solve_s": round(t_mixed, 6), "converged": bool(ok_m) and rr_check <= 1e-8,
                 "corrections": iters, "relres": rr_m, "relres_recomputed": rr_check,
                 "rel_diff_x_vs_fp64": err_vs_fp64, "logdet": logdet32,
                 "rel_diff_logdet_vs_fp64": abs(logdet32 - logdet) / abs(logdet),
                 "leaves": leaves, "first_factor_promoted_leaves": first_promoted,
                 "first_factor_ms": first_ms, "promoted_leaves": int(minfo.promoted_nodes),
                 "fp32_products_used": int(minfo.promoted_nodes) < leaves,
                 "reading": ("the leaf products in FP32 perturb each leaf block by about u32 |D|, above the "
                             "smallest pivots of these leaves: the accuracy guard factors them in FP64")}
        # the BF16 forms' guards (2^-10 and 2^-2 |D|_inf) on the same leaves: one factorization each
        for name, prec in (("bf16x3", hss.HSS_P_BF16X3), ("bf16", hss.HSS_P_BF16)):
            hss.hss_ulv_factor(ctx, m, prec)
            mixed[f"first_factor_promoted_leaves_{name}"] = int(hss.hss_get_info(m).promoted_nodes)
    except Exception as e:  # report, keep the FP64 result
        mixed = {"error": str(e)}
    # leave the matrix factored in FP64 for anything after
    hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP64)
    total_factor_flops = sum(step_flops(sname, n, rr) for _, l, n, rr in nodes if l > 0
                             for sname in ("gemm_W=MY", "gemm_F_update", "gemm_Y=VT", "gemm_C=YtW", "gemm_Z",
                                           "gemm_V2", "basis_top", "pchol"))
    total_factor_flops += sum(step_flops("root", n, 0) for _, l, n, rr in nodes if l == 0)

    use_mixed = bool(mixed and mixed.get("converged")) and mixed["factor_plus_refined_solve_s"] < t_best
    value = mixed["factor_plus_refined_solve_s"] if use_mixed else t_best
    fp64_variant = ("default tiles, eager" if t_best == t_fp64 else
                    "fused" if tuned and round(t_best, 6) == tuned.get("fused_factor_solve_s") else
                    "graph" if tuned and round(t_best, 6) == tuned.get("graph_replay_s") else "tuned, eager")
    result = {
        "metric": "HSS-ULV factor+solve s at N=262144; mixed+IR vs FP64 at rel. residual 1e-8",
        "value": round(value, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(value * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if use_mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.n, "dim": w.dim, "kernel": w.kernel, "length": w.length,
                   "nugget": w.nugget, "leaf": w.leaf, "levels": L, "rank": w.rank, "nrhs": 1,
                   "compression": "scaled randomized", "samples": s,
                   "precision": "mixed fp32/fp64 + refinement" if use_mixed else "fp64"},
        "roofline": roof,
        "fp64": {"factor_plus_solve_s": round(t_fp64, 6), "relres": relres, "logdet": logdet,
                 "tuned_graph": tuned,
                 "factor_ms_events": round(info.factor_ms, 3), "algorithmic_factor_gflop": round(total_factor_flops / 1e9, 2),
                 "factor_gflops_per_s": round(total_factor_flops / 1e9 / (info.factor_ms * 1e-3), 1),
                 "profiled_step_s": round(t_prof, 6),
                 "ms_by_step": {k: round(v / args.steps, 3) for k, v in sorted(by_step.items(), key=lambda kv: -kv[1])},
                 "ms_by_step_level": {f"{k[0]}@{k[1]}": round(v[1] / args.steps, 4) for k, v in sorted(prof.items())}},
        "mixed": mixed,
        "speedup_mixed_vs_fp64": (round(t_best / mixed["factor_plus_refined_solve_s"], 3)
                                  if mixed and mixed.get("converged") else None),
        "speedup_reference": f"fastest FP64 variant ({fp64_variant}, {round(t_best * 1e3, 3)} ms)",
        "construct_s": round(construct_s, 3),
    }
    hss.hss_matrix_destroy(m)
    m = None
    if not args.no_batched:
        result["batched"] = batched_leg(hss, torch, np, ctx, args.steps, args.warmup)
    if not args.no_mixed:
        result["mixed_exp3d"] = mixed_exp_leg(hss, torch, np, ctx, args.steps, args.warmup, args.no_tune)
    if not args.no_learned:
        result["learned_rank"] = learned_leg(hss, torch, np, ctx)
    if not args.no_config2:
        result["config2"] = config2_leg(hss, torch, np, ctx, args.steps, args.warmup, args.no_tune)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(exp, w, b.cpu().numpy(), x.cpu().numpy())
    hss.hss_ctx_destroy(ctx)
    print(json.dumps(result))


def config2_leg(hss, torch, np, ctx, steps, warmup, no_tune):
    """The 16-right-hand-side workload (Matern-3/2, N = 65536, leaf 256, rank
    64): the autotuned FP64 one-call factor + solve of all 16 columns, and the
    BLR^2-ULV (Alg. 1) of the same matrix beside it: its leaf stage is the
    same, its skeleton matrix (256 leaves x rank 64 = 16384 rows) is factored
    densely, which is what the nested basis of the HSS-ULV avoids."""
    import synth

    w = synth.WORKLOADS["matern32_n65536"]
    print(f"# config2 leg on {w.name}", file=sys.stderr, flush=True)
    s = w.rank + w.oversample
    X = torch.from_numpy(w.points()).cuda()
    Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
    B = torch.from_numpy(np.ascontiguousarray(w.rhs().T)).cuda().t()
    t0 = time.perf_counter()
    m = hss.hss_construct(ctx, X, w.kernel, w.leaf, rank=w.rank, omega=Om, length=w.length, nugget=w.nugget)
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    del X, Om
    try:
        if not no_tune:
            hss.hss_autotune(ctx, m, hss.HSS_P_FP64, 2)

        def timed(fn, n):
            ts = []
            out = None
            for _ in range(n):
                torch.cuda.synchronize()
                t = time.perf_counter()
                out = fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            return float(np.median(ts)), out

        for _ in range(warmup):
            hss.hss_ulv_factor_solve(ctx, m, B)
        t_hss, x_h = timed(lambda: hss.hss_ulv_factor_solve(ctx, m, B), steps)
        ld_h = hss.hss_logdet(ctx, m)
        rr = torch.linalg.norm(B - hss.hss_matvec(ctx, m, x_h), dim=0) / torch.linalg.norm(B, dim=0)
        K, _ = hss.hss_blr2_stats(m)

        def blr2_step():
            hss.hss_blr2_factor(ctx, m)
            return hss.hss_blr2_solve(ctx, m, B)

        blr2_step()
        t_blr2, x_b = timed(blr2_step, max(1, min(steps, 3)))
        f_ms = hss.hss_blr2_stats(m)[1]
        torch.cuda.synchronize()
        t = time.perf_counter()
        hss.hss_blr2_solve(ctx, m, B)
        torch.cuda.synchronize()
        t_bsolve = time.perf_counter() - t
        ld_b = hss.hss_blr2_logdet(ctx, m)
        rr_b = torch.linalg.norm(B - hss.hss_matvec(ctx, m, x_b), dim=0) / torch.linalg.norm(B, dim=0)
        chol_gflop = K ** 3 / 3 / 1e9
        return {"workload": w.name, "N": w.n, "leaf": w.leaf, "rank": w.rank, "nrhs": 16,
                "construct_s": round(construct_s, 3),
                "hss_factor_plus_solve_s": round(t_hss, 6), "hss_relres_max": float(rr.max()),
                "blr2": {"skeleton_rows": K, "factor_plus_solve_s": round(t_blr2, 6),
                         "factor_ms_events": round(f_ms, 3), "solve_s": round(t_bsolve, 6),
                         "skeleton_cholesky_gflop": round(chol_gflop, 1),
                         "cholesky_gflop_over_factor_ms": round(chol_gflop / f_ms, 2) if f_ms > 0 else None,
                         "relres_max": float(rr_b.max()),
                         "rel_diff_x_vs_hss": float(torch.linalg.norm(x_b - x_h) / torch.linalg.norm(x_h)),
                         "logdet_abs_diff_vs_hss": abs(ld_b - ld_h)},
                "hss_speedup_vs_blr2": round(t_blr2 / t_hss, 1)}
    finally:
        hss.hss_matrix_destroy(m)


def mixed_exp_leg(hss, torch, np, ctx, steps, warmup, no_tune):
    """The precision form where the FP32 products pass the accuracy guard: the
    exponential kernel exp(-r/0.1) (the kernel of the N = 2^20 workload, no
    nugget) on N = 262144 uniform points in the unit cube, leaf 256, rank 96,
    scaled construction. The fastest FP64 variant (autotuned one-call factor +
    solve) beside the mixed factorization + refined solve to 1e-8."""
    import dataclasses

    import synth

    w = dataclasses.replace(synth.WORKLOADS["matern32_n262144"], name="exp3d_n262144", kernel="exponential",
                            length=0.1, nugget=0.0)
    print(f"# mixed leg on {w.name}", file=sys.stderr, flush=True)
    s = w.rank + w.oversample
    X = torch.from_numpy(w.points()).cuda()
    Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
    b = torch.from_numpy(np.ascontiguousarray(w.rhs()[:, 0])).cuda()
    m = hss.hss_construct(ctx, X, w.kernel, w.leaf, rank=w.rank, omega=Om, length=w.length, nugget=w.nugget)
    del X, Om
    try:
        hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP32)
        promoted = int(hss.hss_get_info(m).promoted_nodes)
        if not no_tune:
            hss.hss_autotune(ctx, m, hss.HSS_P_FP64, 2)
            hss.hss_autotune(ctx, m, hss.HSS_P_FP32, 2)

        def timed(fn, n):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = None
            for _ in range(n):
                out = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / n, out

        def mixed_step():
            hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP32)
            return hss.hss_ulv_solve_refined(ctx, m, b, 1e-8, 50)

        def fac(prec):
            hss.hss_ulv_factor(ctx, m, prec)
            return hss.hss_get_info(m).factor_ms

        for _ in range(warmup):
            hss.hss_ulv_factor_solve(ctx, m, b)
            mixed_step()
        t64, x64 = timed(lambda: hss.hss_ulv_factor_solve(ctx, m, b), steps)
        tmx, (xm, iters, rr, ok) = timed(mixed_step, steps)
        rr_check = float(torch.linalg.norm(b - hss.hss_matvec(ctx, m, xm)) / torch.linalg.norm(b))
        f64 = float(np.median([fac(hss.HSS_P_FP64) for _ in range(steps)]))
        f32 = float(np.median([fac(hss.HSS_P_FP32) for _ in range(steps)]))
        # the BF16 forms (sharing the FP32 form's tile choices): the split products
        # and plain BF16, each with its own accuracy guard
        low = {}
        for name, prec in (("bf16x3", hss.HSS_P_BF16X3), ("bf16", hss.HSS_P_BF16)):
            hss.hss_ulv_factor(ctx, m, prec)
            first = int(hss.hss_get_info(m).promoted_nodes)

            def low_step(p=prec):
                hss.hss_ulv_factor(ctx, m, p)
                return hss.hss_ulv_solve_refined(ctx, m, b, 1e-8, 50)

            low_step()
            tq, (xq, itq, rq, okq) = timed(low_step, steps)
            rq_check = float(torch.linalg.norm(b - hss.hss_matvec(ctx, m, xq)) / torch.linalg.norm(b))
            low[name] = {"first_factor_promoted_leaves": first,
                         "promoted_leaves": int(hss.hss_get_info(m).promoted_nodes),
                         "factor_plus_refined_solve_s": round(tq, 6), "converged": bool(okq) and rq_check <= 1e-8,
                         "corrections": itq, "relres_recomputed": rq_check,
                         "factor_ms_events": round(float(np.median([fac(prec) for _ in range(steps)])), 3)}
        return {"workload": w.name, "kernel": "exponential", "length": w.length, "nugget": w.nugget,
                "fp64_fused_factor_solve_s": round(t64, 6), "mixed_factor_plus_refined_solve_s": round(tmx, 6),
                "speedup_mixed_vs_fp64": round(t64 / tmx, 3), "converged": bool(ok) and rr_check <= 1e-8,
                "corrections": iters, "relres_recomputed": rr_check, "promoted_leaves": promoted,
                "factor_ms_fp64_events": round(f64, 3), "factor_ms_mixed_events": round(f32, 3), **low}
    finally:
        hss.hss_matrix_destroy(m)


def sweep_leg(hss, torch, np, ctx, steps, warmup):
    """One-GPU scaling sweeps for the paper's linear-complexity and leaf-size
    claims (Sec. 5.4-5.5): the FP64 one-call factor + solve (autotuned tiles)
    of the Matern-3/2 workload (3-D uniform points, length 0.2, nugget 1e-6,
    scaled construction, rank 100) for N = 4096 .. 262144 at leaf 256, and for
    leaf 128, 512 and 1024 at N = 262144."""
    import dataclasses

    import synth

    base = dataclasses.replace(synth.WORKLOADS["matern32_n262144"], rank=100)
    configs = [dataclasses.replace(base, name=f"matern32_n{n}_r100", n=n) for n in
               (4096, 8192, 16384, 32768, 65536, 131072, 262144)]
    configs += [dataclasses.replace(base, name=f"matern32_n262144_r100_leaf{lf}", leaf=lf) for lf in (128, 512, 1024)]
    out = []
    for w in configs:
        print(f"# sweep: {w.name} N={w.n} leaf={w.leaf}", file=sys.stderr, flush=True)
        s = w.rank + w.oversample
        X = torch.from_numpy(w.points()).cuda()
        Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
        b = torch.from_numpy(np.ascontiguousarray(w.rhs()[:, 0])).cuda()
        m = hss.hss_construct(ctx, X, w.kernel, w.leaf, rank=w.rank, omega=Om, length=w.length, nugget=w.nugget)
        del X, Om
        try:
            hss.hss_autotune(ctx, m, hss.HSS_P_FP64, 3)
            for _ in range(warmup):
                hss.hss_ulv_factor_solve(ctx, m, b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x = None
            for _ in range(steps):
                x = hss.hss_ulv_factor_solve(ctx, m, b)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / steps
            rr = float(torch.linalg.norm(b - hss.hss_matvec(ctx, m, x)) / torch.linalg.norm(b))
            info = hss.hss_get_info(m)
            out.append({"workload": w.name, "N": w.n, "leaf": w.leaf, "levels": int(info.levels), "rank": w.rank,
                        "factor_plus_solve_ms": round(dt * 1e3, 4), "ns_per_unknown": round(dt / w.n * 1e9, 3),
                        "relres": rr})
        finally:
            hss.hss_matrix_destroy(m)
    return out


def table2_leg(hss, torch, np, ctx):
    """Accuracy on the paper's Table 2 setting (Sec. 5.1): N = 65536 points on
    the uniform 256 x 256 grid, the three kernels of Table 3 (Laplace-2D,
    Yukawa, and Matern with rho = 1/2, i.e. exp(-d / 0.03)), and the table's
    (max rank, leaf) rows, with the paper's construction (PLAIN: pivoted QR of
    the off-diagonal row blocks, here seen through rank + 16 random samples).
    Eq. 18 (construction error) on 256 sampled rows of A b with the exact rows
    by direct kernel evaluation; Eq. 19 (solve error) in full. The (400, 512)
    row has blocks of 800 rows above the leaves."""
    import dataclasses
    import csv

    import synth

    with open(os.path.join(ROOT, "tests", "golden", "table2_hatrix.csv")) as f:
        rows = [r for r in csv.reader(line for line in f if not line.startswith("#"))]
    printed = {(int(r[0]), int(r[1])): [float(v) for v in r[2:]] for r in rows}
    base = synth.Workload("table2_grid_n65536", 65536, 2, "exponential", 0.03, 0.0, 256, 100, geometry="grid2d",
                          seed_k=5)
    kernels = (("laplace2d", dict(kernel="laplace2d", extra={"eps": 1e-9, "alpha": 1.0}), 0),
               ("yukawa", dict(kernel="yukawa", extra={"eps": 1e-9, "alpha": 1.0}), 2),
               ("matern_rho_half_mu_0.03", dict(kernel="exponential"), 4))
    out = []
    for (rank, leaf) in sorted(printed):
        for name, kw, col in kernels:
            rec = {"kernel": name, "N": base.n, "max_rank": rank, "leaf": leaf, "construction": "plain",
                   "paper_construct_error": printed[(rank, leaf)][col],
                   "paper_solve_error": printed[(rank, leaf)][col + 1]}
            w = dataclasses.replace(base, name=f"table2_{name}_r{rank}_l{leaf}", rank=rank, leaf=leaf, **kw)
            print(f"# table2 leg: {name} rank {rank} leaf {leaf}", file=sys.stderr, flush=True)
            s = rank + 16
            X = torch.from_numpy(w.points()).cuda()
            Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
            b = torch.from_numpy(np.ascontiguousarray(w.rhs()[:, 0])).cuda()
            extra = w.extra or {}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m = hss.hss_construct(ctx, X, w.kernel, w.leaf, rank=w.rank, omega=Om, length=w.length,
                                  nugget=w.nugget, alpha=extra.get("alpha", 1.0), eps=extra.get("eps", 1e-9),
                                  mode="plain")
            torch.cuda.synchronize()
            rec["construct_s"] = round(time.perf_counter() - t0, 3)
            try:
                sel = torch.from_numpy(np.random.default_rng(78).choice(w.n, 256, replace=False)).cuda()
                ab = hss.hss_matvec(ctx, m, b)
                y_exact = exact_rows(torch, X, b, sel, w)
                rec["construct_error_eq18_rows"] = float(torch.linalg.norm(ab[sel] - y_exact) /
                                                         torch.linalg.norm(y_exact))
                hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP64)
                rec["factor_ms"] = round(hss.hss_get_info(m).factor_ms, 3)
                x = hss.hss_ulv_solve(ctx, m, ab)
                rec["solve_error_eq19"] = float(torch.linalg.norm(b - x) / torch.linalg.norm(b))
            except hss.HSSError as e:
                rec["error"] = str(e)
            finally:
                hss.hss_matrix_destroy(m)
            out.append(rec)
    return out


def measured_traffic(label, workload, tile):
    """HBM bytes per launch of the profiled kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters), or
    None if there is none or the kernel's source changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    ent = tab.get(f"{label}:{workload}")
    if not ent:
        return None
    src = os.path.join(ROOT, ent["source"])
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if sha != ent["source_sha256"] or ent.get("tile") != tile:
        return None
    return ent["hbm_bytes_per_launch"]


def gpu_rank_labels(hss, torch, np, ctx, problems, cap=128, samples=136):
    """(features, ranks) of every non-root node of the plain adaptive
    construction (Eq. 2 with |R_jj| > tol |R_00|, capped) of each problem: the
    labels the rank model learns, produced by the library's own construction
    (its ranks are pinned to the oracle's pivoted QR in the construction tests)."""
    import synth

    feats, ranks = [], []
    cache = {}
    for (n, geo, seed, leaf, tol) in problems:
        key = (n, geo, seed)
        if key not in cache:
            cache.clear()
            X = synth.points_grid2d(n) if geo == "grid2d" else synth.points_uniform(n, 2, 1200 + seed)
            Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
            Om = torch.from_numpy(np.ascontiguousarray(synth.test_matrix(n, samples, 3200 + seed).T)).cuda().t()
            cache[key] = (Xd, Om)
        Xd, Om = cache[key]
        m = hss.hss_construct(ctx, Xd, "laplace2d", leaf, tol=tol, max_rank=cap, omega=Om, length=1.0, eps=1e-9,
                              mode="plain")
        try:
            rk = hss.hss_get_ranks(m)[1:]
        finally:
            hss.hss_matrix_destroy(m)
        f = hss.hss_rank_features(ctx, Xd, leaf, 1.0, tol).reshape(-1, 7)
        assert f.shape[0] == rk.shape[0]
        feats.append(f)
        ranks.append(rk)
    return np.concatenate(feats), np.concatenate(ranks)


def learned_leg(hss, torch, np, ctx):
    """Learned rank model (form 4): trained on the GPU on about 1e5 labelled
    nodes of Laplace-2D constructions whose ranks vary below the cap (plain
    construction, tolerances 3e-2 .. 1e-8), then three ways of sizing the
    random samples of a held-out construction -- the 256 x 256 grid of Table 2,
    leaf 256, cap 128, at two tolerances -- compared: model-presized, fixed
    conservative (cap + 8 samples) and adaptive doubling from 16, all with the
    8-column probe judge."""
    import synth

    t0 = time.perf_counter()
    feats, ranks = gpu_rank_labels(hss, torch, np, ctx, synth.rank_label_problems())
    label_s = time.perf_counter() - t0
    F = torch.from_numpy(feats).cuda()
    T = torch.from_numpy(np.log2(1.0 + ranks).astype(np.float32)).cuda()
    mlp = hss.hss_rankmlp_create(ctx)
    init = synth.mlp_init((7, 128, 128, 128, 1), seed=5000)
    hss.hss_rankmlp_set_weights(ctx, mlp, init)
    epochs = 8
    order = torch.from_numpy(synth.minibatch_order(len(ranks), epochs, seed=5100)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hss.hss_rankmlp_train(ctx, mlp, F, T, order, 256, lr=1e-3, tau=0.9, record_losses=False)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    pred = hss.hss_rankmlp_predict(ctx, mlp, F, 128).cpu().numpy()
    out = {"labels": {"kernel": "laplace2d", "construction": "plain", "problems": len(synth.rank_label_problems()),
                      "nodes": int(len(ranks)), "generate_s": round(label_s, 2),
                      "rank_quartiles": [int(v) for v in np.percentile(ranks, [25, 50, 75])],
                      "at_cap": float(np.mean(ranks >= 128))},
           "train": {"epochs": epochs, "batch": 256, "steps": int((len(order) + 255) // 256),
                     "train_s": round(train_s, 3), "coverage_pred_ge_label": float(np.mean(pred >= ranks)),
                     "mean_abs_rank_error": float(np.mean(np.abs(pred - ranks)))}}
    cap = 128
    s = cap + 8 + 8
    n = 65536
    w = synth.Workload("laplace2d_grid_n65536", n, 2, "laplace2d", 1.0, 0.0, 256, 0, geometry="grid2d",
                       extra={"eps": 1e-9, "alpha": 1.0}, seed_k=7)
    X = torch.from_numpy(w.points()).cuda()
    Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
    b = torch.from_numpy(np.ascontiguousarray(w.rhs()[:, 0])).cuda()
    rows = torch.from_numpy(np.random.default_rng(77).choice(n, 256, replace=False)).cuda()
    y_exact = exact_rows(torch, X, b, rows, w)
    out["heldout"] = {"name": w.name, "N": n, "leaf": w.leaf, "cap": cap, "s_available": s}
    for tol in (1e-2, 1e-3):
        res = {}
        for name, kw in (("model", dict(rank_model=mlp)), ("fixed", dict(sample_start=cap + 8)),
                         ("doubling_from_16", dict(sample_start=16))):
            print(f"# learned-rank leg: tol {tol:g} {name}", file=sys.stderr, flush=True)
            ts = []
            m = None
            for rep in range(3):
                if m is not None:
                    hss.hss_matrix_destroy(m)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                m = hss.hss_construct(ctx, X, w.kernel, w.leaf, tol=tol, max_rank=cap, omega=Om, length=1.0,
                                      eps=1e-9, mode="plain", **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            st = hss.hss_get_construct_stats(m)
            rec = {"construct_s": round(float(np.median(ts)), 4), "attempts": st.attempts, "samples": st.samples,
                   "probes": st.probes, "judge_failures": st.judge_failures, "predicted_max": st.predicted_max,
                   "max_rank": st.max_rank, "sample_buffer_bytes": int(st.sample_bytes)}
            try:
                y = hss.hss_matvec(ctx, m, b)[rows]
                rec["construction_error_rows"] = float(torch.linalg.norm(y - y_exact) / torch.linalg.norm(y_exact))
                x = hss.hss_ulv_factor_solve(ctx, m, b)
                rec["relres"] = float(torch.linalg.norm(b - hss.hss_matvec(ctx, m, x)) / torch.linalg.norm(b))
            except hss.HSSError as e:
                rec["error"] = str(e)
            hss.hss_matrix_destroy(m)
            res[name] = rec
            print(f"# {name}: {rec}", file=sys.stderr, flush=True)
        res["model_vs_fixed"] = {
            "construct_time_ratio": round(res["model"]["construct_s"] / res["fixed"]["construct_s"], 3),
            "sample_bytes_ratio": round(res["model"]["sample_buffer_bytes"] / res["fixed"]["sample_buffer_bytes"], 3)}
        out[f"tol_{tol:g}"] = res
    hss.hss_rankmlp_destroy(mlp)
    return out


def exact_rows(torch, X, v, rows, w):
    """(A v)[rows] by direct evaluation of the kernel (plain torch, FP64)."""
    out = torch.zeros(rows.shape[0], dtype=torch.float64, device=X.device)
    Xr = X[rows]
    step = 1 << 14
    for c0 in range(0, X.shape[0], step):
        Xc = X[c0:c0 + step]
        dist = torch.sqrt(((Xr[:, None, :] - Xc[None, :, :]) ** 2).sum(-1))
        if w.kernel == "exponential":
            K = torch.exp(-dist / w.length)
        elif w.kernel == "laplace2d":
            K = -torch.log(w.extra["eps"] + dist)
        elif w.kernel == "yukawa":
            K = torch.exp(-w.extra["alpha"] * (w.extra["eps"] + dist)) / (w.extra["eps"] + dist)
        elif w.kernel == "matern32":
            a = (3.0 ** 0.5) * dist / w.length
            K = (1.0 + a) * torch.exp(-a)
        else:
            K = torch.exp(-(dist / w.length) ** 2)
        out += K @ v[c0:c0 + step]
    return out + w.nugget * v[rows]


def batched_leg(hss, torch, np, ctx, steps, warmup):
    """64 independent Gaussian-kernel systems of uneven N factored and solved as
    one batch (stages by height, autotuned tiles, graph replay), against a loop
    over the same systems one at a time (eager launches, default tiles)."""
    import synth

    ws = synth.batch_gaussian()
    print(f"# batched leg: {len(ws)} systems, N_total={sum(w.n for w in ws)}", file=sys.stderr, flush=True)
    singles = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w in ws:
        s = w.extra["max_rank"] + w.oversample
        X = torch.from_numpy(w.points()).cuda()
        Om = torch.from_numpy(np.ascontiguousarray(w.omega(s).T)).cuda().t()
        singles.append(hss.hss_construct(ctx, X, w.kernel, w.leaf, tol=w.tol, max_rank=w.extra["max_rank"],
                                         omega=Om, length=w.length, nugget=w.nugget))
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    batch = hss.hss_batch_create(ctx, singles)
    cnt = len(ws)
    off, _, _ = hss.hss_batch_query(ctx, batch, cnt, factored=False)
    b = torch.from_numpy(np.concatenate([w.rhs()[:, 0] for w in ws])).cuda()
    x = torch.empty_like(b)
    parts = [(b[off[k]:off[k + 1]], x[off[k]:off[k + 1]]) for k in range(cnt)]
    ranks = [hss.hss_get_info(sm).max_rank for sm in singles]
    out = {"workload": f"gaussian_batch{cnt}", "systems": cnt, "N_total": int(off[-1]),
           "N_min": int(min(w.n for w in ws)), "N_max": int(max(w.n for w in ws)),
           "heights": int(hss.hss_get_info(batch).levels) + 1, "max_rank_range": [min(ranks), max(ranks)],
           "construct_s": round(construct_s, 3)}

    def per_system_relres(xv):
        r = b - hss.hss_matvec(ctx, batch, xv)
        return max(float(torch.linalg.norm(r[off[k]:off[k + 1]]) / torch.linalg.norm(b[off[k]:off[k + 1]]))
                   for k in range(cnt))

    for prec, name in ((hss.HSS_P_FP32, "fp32"), (hss.HSS_P_FP64, "fp64")):
        leg = {}
        try:
            hss.hss_use_graphs(ctx, batch, False)
            rep = hss.hss_autotune(ctx, batch, prec, 2)
            hss.hss_use_graphs(ctx, batch, True)

            def run_batch(n):
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(n):
                    hss.hss_ulv_factor(ctx, batch, prec)
                    hss.hss_ulv_solve(ctx, batch, b, x)
                torch.cuda.synchronize()
                return (time.perf_counter() - t) / n

            def run_loop(n):
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(n):
                    for sm, (bk, xk) in zip(singles, parts):
                        hss.hss_ulv_factor(ctx, sm, prec)
                        hss.hss_ulv_solve(ctx, sm, bk, xk)
                torch.cuda.synchronize()
                return (time.perf_counter() - t) / n

            for _ in range(warmup):
                run_batch(1)
            leg["batch_factor_plus_solve_s"] = round(run_batch(steps), 6)
            leg["relres_max_over_systems"] = per_system_relres(x)
            leg["gemm_ms_per_factor_uniform_64x64"] = rep[0]
            leg["gemm_ms_per_factor_tuned"] = rep[-1]
            for _ in range(warmup):
                run_loop(1)
            leg["loop_factor_plus_solve_s"] = round(run_loop(steps), 6)
            leg["speedup_batch_vs_loop"] = round(leg["loop_factor_plus_solve_s"] / leg["batch_factor_plus_solve_s"], 2)
            if prec == hss.HSS_P_FP32:
                hss.hss_ulv_factor(ctx, batch, prec)
                torch.cuda.synchronize()
                t = time.perf_counter()
                xr, iters, rr, ok = hss.hss_ulv_solve_refined(ctx, batch, b, 1e-8, 50)
                torch.cuda.synchronize()
                leg["refined_solve_to_1e-8_s"] = round(time.perf_counter() - t, 6)
                leg["refined_corrections"] = iters
                leg["refined_converged"] = bool(ok)
        except hss.HSSError as e:
            leg["error"] = str(e)
            try:
                _, failed, _ = hss.hss_batch_query(ctx, batch, cnt)
                leg["failed_systems"] = [int(i) for i in np.nonzero(failed)[0]]
            except hss.HSSError:
                pass
        out[name] = leg
        print(f"# batched {name}: {leg}", file=sys.stderr, flush=True)
    hss.hss_matrix_destroy(batch)
    for sm in singles:
        hss.hss_matrix_destroy(sm)
    return out


def cpu_baseline(exp, w, b, x_gpu):
    """The oracle's factor + solve of the whole exported HSS matrix of the
    workload with one BLAS thread (its operations are on blocks of a few hundred
    rows, where a threaded BLAS spends more on synchronization than it saves:
    76.8 s with 16 threads against 3.2 s with one on the benchmark's box; see
    --cpu-full). Nothing is extrapolated."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import hss_oracle as O
    from paper_2311_00921_amd import hss

    full = hss.unpack_desc(exp)
    h = O.HSS(full["n"], full["levels"], full["ranges"], full["rank"], full["D"], full["U"], full["E"], full["S"])
    perm = exp["perm"]
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        F = O.ulv_factor(h)
        xt = O.ulv_solve(h, F, b[perm])
        dt = time.perf_counter() - t
    x = np.empty_like(xt)
    x[perm] = xt
    diff = float(np.linalg.norm(x - x_gpu) / np.linalg.norm(x))
    return {"value": round(dt, 3), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"the whole matrix: oracle ULV factor + solve of the exported HSS matrix (N={w.n}, "
                      f"{2 ** full['levels']} leaves), one BLAS thread; solution vs the GPU's: {diff:.1e} relative"}


def cpu_full(exp, w, b, x_gpu, ld_gpu):
    """The oracle's factor + solve on the whole exported HSS matrix of the
    workload (tree order in, the caller's order out), timed with all host threads
    and with one thread (BLAS thread pools limited), beside the GPU's solution
    and log-determinant of the same matrix."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import hss_oracle as O
    from paper_2311_00921_amd import hss

    full = hss.unpack_desc(exp)
    h = O.HSS(full["n"], full["levels"], full["ranges"], full["rank"], full["D"], full["U"], full["E"], full["S"])
    perm = exp["perm"]
    bt = b[perm]
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    out = {"workload": w.name, "N": w.n, "cpu_model": model, "nproc": os.cpu_count(), "blas_threads": threads}
    for label, limit in (("all_threads", None), ("one_thread", 1)):
        print(f"# oracle factor + solve on the full matrix ({label})", file=sys.stderr, flush=True)
        if limit:
            with threadpool_limits(limits=limit):
                t = time.perf_counter()
                F = O.ulv_factor(h)
                xt = O.ulv_solve(h, F, bt)
                dt = time.perf_counter() - t
        else:
            t = time.perf_counter()
            F = O.ulv_factor(h)
            xt = O.ulv_solve(h, F, bt)
            dt = time.perf_counter() - t
        x = np.empty_like(xt)
        x[perm] = xt
        out[label] = {"factor_plus_solve_s": round(dt, 3),
                      "rel_diff_x_vs_gpu": float(np.linalg.norm(x - x_gpu) / np.linalg.norm(x)),
                      "logdet_abs_diff_vs_gpu": abs(F.logdet - ld_gpu), "logdet": F.logdet}
    return out


if __name__ == "__main__":
    main()
