"""Benchmark: repeated refactorisation + solve of a circuit-like matrix on one MI355X.

Workload (the repeated-solve scenario of the paper, Sec. 3.2): a circuit-like
nonsymmetric matrix with n = 200000, mean 5 stored entries per row and a
power-law column degree (exponent 2.1, max 2000), diagonally dominant with
N(0,1) off-diagonals.  It is analysed once; every step redraws all values on
the same pattern (seed 1100+r), refactorises on the GPU and solves one
right-hand side (b = A x_true, x_true ~ U[-1,1], seed 2100+r).  All value sets
and right-hand sides are resident in HBM before timing starts.

Prints one JSON line.  `value` is milliseconds per refactor+solve step
(lower is better); factor GFLOP/s = F / refactor time, with F the flop count
of the exact symbolic structure.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=200000)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--amd-dense", type=float, default=0.0)
    ap.add_argument("--dense-tail", type=float, default=0.15)
    ap.add_argument("--pipeline-rows", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 + refinement leg of the headline")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the other workloads (27-point grid, batch, adjoint) appended to the headline line")
    ap.add_argument("--value-sets", type=int, default=100,
                    help="value sets of the circuit workload (the workload refactorises each once)")
    ap.add_argument("--cpu-sample-refactors", type=int, default=3)
    ap.add_argument("--workload", default="circuit", choices=["circuit", "batch", "grid27", "adjoint", "copy"],
                    help="circuit (default): the headline line; the others print their own line")
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--sn-tile", type=int, default=0)
    ap.add_argument("--sn-dense", type=int, default=64)
    ap.add_argument("--sn-inverse", type=int, default=1)
    ap.add_argument("--tail-sparse", type=int, default=1)
    ap.add_argument("--side-rows", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick per-level launch shapes with hylu_autotune before timing (untimed setup)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload != "circuit":
        {"batch": bench_batch, "grid27": bench_grid27, "adjoint": bench_adjoint,
         "copy": bench_copy}[args.workload](args)
        return

    import torch
    from paper_2509_07690_amd import synth, hylu

    dev = torch.device("cuda:0")
    t0 = time.time()
    base = synth.circuit_powerlaw(args.n)  # refactor 0 values define the analysis
    A0 = base.A
    log(f"pattern n={A0.n} nnz={A0.nnz} ({time.time() - t0:.1f}s)")
    opts = dict(amd_dense=args.amd_dense, dense_tail=args.dense_tail, pipeline_rows=args.pipeline_rows,
                sn_dense=args.sn_dense, sn_inverse=args.sn_inverse, tail_sparse=args.tail_sparse,
                side_rows=args.side_rows)
    t0 = time.time()
    h = hylu.Handle(A0.row_ptr, A0.col, A0.val, precision=args.precision, **opts)
    t_analyze = time.time() - t0
    info = h.info()
    log(f"analyze {t_analyze:.1f}s: F={info['flops']:.3e} nnz(L+U)={info['nnz_l'] + info['nnz_u']:.3e} "
        f"supernodes={info['n_supernodes']} levels={info['n_levels']} tail={info['tail_rows']}")
    # the workload's value sets (one per refactorisation), resident in HBM
    nsets = max(args.value_sets, args.warmup + args.steps)
    t0 = time.time()
    vals, bs, xts = [], [], []
    for r in range(nsets):
        w = base.revalue(r + 1)
        vals.append(torch.from_numpy(w.A.val).to(dev))
        bs.append(torch.from_numpy(np.ascontiguousarray(w.b[:, 0])).to(dev))
        xts.append(w.x_true[:, 0])
    xs = [torch.empty_like(b) for b in bs]
    log(f"{nsets} value sets ({time.time() - t0:.1f}s)")
    v0 = torch.from_numpy(A0.val).to(dev)
    h.factorize(v0)
    torch.cuda.synchronize()
    tune = None
    if args.autotune:
        t0 = time.time()
        t_def, t_tuned = h.autotune(v0, reps=2)
        tune = {"builtin": round(t_def, 3), "tuned": round(t_tuned, 3), "s": round(time.time() - t0, 2)}
        log(f"autotune: level launches {t_def:.2f} ms with built-in shapes, {t_tuned:.2f} ms tuned")

    def run(hd, steps, warmup, first=0):
        """warmup + timed refactor+solve steps over consecutive value sets;
        returns (ms per step by the host clock, median refactor ms, median
        solve ms, the value-set indices timed)"""
        idx = [(first + r) % nsets for r in range(warmup + steps)]
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in idx]
        for r in idx[:warmup]:
            hd.refactor(vals[r])
            hd.solve(bs[r], out=xs[r])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for q, r in enumerate(idx[warmup:]):
            e0, e1, e2 = ev[q]
            e0.record()
            hd.refactor(vals[r])
            e1.record()
            hd.solve(bs[r], out=xs[r])
            e2.record()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / steps
        tr = float(np.median([ev[q][0].elapsed_time(ev[q][1]) for q in range(steps)]))
        tsv = float(np.median([ev[q][1].elapsed_time(ev[q][2]) for q in range(steps)]))
        return ms, tr, tsv, idx[warmup:]

    ms_step, t_ref, t_sol, timed = run(h, args.steps, args.warmup)
    errs = [float(np.abs(xs[r].cpu().numpy() - xts[r]).max()) for r in timed]
    eta, res1 = h.residual(bs[timed[-1]], xs[timed[-1]])
    # the workload as specified: every value set refactorised and solved once, back to back
    ms_seq, _, _, _ = run(h, nsets, 0)
    x64 = xs[timed[-1]].clone()

    # per-kernel-class device time from HIP events around every launch of one
    # eager refactor+solve (same stream), with the algorithmic bytes / flops
    xprof = torch.empty_like(bs[0])
    prof = h.profile(vals[timed[-1]], bs[timed[-1]], xprof)
    torch.cuda.synchronize()
    fp_peak = FP64_PEAK_TFLOPS if args.precision == "fp64" else FP32_PEAK_TFLOPS
    kernels = {}
    for k in prof:
        e = {"launches": k["launches"], "ms": round(k["ms"], 4),
             "avg_launch_us": round(k["ms"] * 1e3 / max(k["launches"], 1), 3),
             "GBps": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 2),
             "TFLOPs": round(k["flops"] / max(k["ms"], 1e-9) / 1e9, 4)}
        if k["name"] in ALGORITHMIC_CLASSES:
            e["hbm_frac"] = round(e["GBps"] / HBM_PEAK_GBS, 5)
        kernels[k["name"]] = e
    dom = max(prof, key=lambda k: k["ms"])
    if dom["name"] == "tail_gemm":
        ach = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
        roof = {"kernel": dom["name"], "bound": "mfma", "achieved": round(ach, 3), "peak": fp_peak,
                "unit": "TFLOP/s", "frac": round(ach / fp_peak, 5), "traffic": None}
    else:
        ach = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
        roof = {"kernel": dom["name"], "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None}
    roof["algorithmic_bytes_per_launch"] = round(dom["bytes"] / max(dom["launches"], 1))
    tr = _traffic(dom["name"]) if args.precision == "fp64" else None
    if tr is not None:
        # measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)
        roof["traffic"] = round(tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"])
        roof["traffic_over_algorithmic"] = round(roof["traffic"] / max(roof["algorithmic_bytes_per_launch"], 1), 2)
    roof["launches"] = dom["launches"]
    roof["avg_launch_us"] = round(dom["ms"] * 1e3 / max(dom["launches"], 1), 3)
    roof["bytes_basis"] = ("exact symbolic structure, unit costs per (target, source) update and per factor "
                           "entry of a solve; no padded or dense widths")

    fp32 = None
    if args.precision == "fp64" and not args.no_fp32:
        fp32 = fp32_ir_leg(args, A0, opts, vals, bs, xs, xts, v0, run, x64, timed)

    symb = None
    if not args.headline_only:
        symb = symbolic_compare(info, lambda: hylu.Handle(A0.row_ptr, A0.col, A0.val, precision=args.precision,
                                                          gpu_symbolic=1, **opts))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A0, base, h, args.cpu_sample_refactors, args.warmup)
    others = None
    if not args.headline_only and args.precision == "fp64":
        h.close()
        del vals, bs, xs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        others = other_configs(args)
    out = {
        "metric": "refactor+solve ms (circuit n=200000, repeated solve)",
        "value": round(ms_step, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64ir",
        "data": "synthetic",
        "config": {"workload": f"circuit_powerlaw n={A0.n} nnz={A0.nnz} refactor+solve, 1 rhs",
                   "n": A0.n, "nnz": A0.nnz, "precision": args.precision, "value_sets": nsets},
        "refactor_ms_median": round(t_ref, 4),
        "solve_ms_median": round(t_sol, 4),
        "ms_per_step_all_value_sets": round(ms_seq, 4),
        "factor_gflops": round(info["flops"] / (t_ref * 1e-3) / 1e9, 3),
        "flops": info["flops"],
        "flops_issued": info["flops_issued"],
        "backward_error": eta,
        "resid_1": res1,
        "max_abs_err_vs_x_true": max(errs),
        "analyze_s": round(t_analyze, 2),
        "autotune_level_ms": tune,
        "tail_rows": info["tail_rows"],
        "roofline": roof,
        "kernels": kernels,
        "fp32_ir": fp32,
        "symbolic": symb,
        "cpu_baseline": cpu,
        "other_configs": others,
    }
    print(json.dumps(out))


# kernel classes whose byte figures follow the per-update and per-entry unit
# costs on the exact structure (the others count the blocks they issue)
ALGORITHMIC_CLASSES = ("rows", "lsolve", "usolve", "tail_solve", "snlu", "sn_inverse", "scatter")


def symbolic_compare(info_host, make_gpu_handle):
    """The same analysis with the symbolic factorisation, supernodes and
    level sets computed on the GPU (untimed in the step): its time against the
    host's, and whether the result is the same (structure and level hash)."""
    hg = make_gpu_handle()
    ig = hg.info()
    hg.close()
    return {"host_ms": round(info_host["sym_ms"], 2), "gpu_ms": round(ig["sym_ms"], 2),
            "gpu_kernel_ms": round(ig["sym_kernel_ms"], 2), "identical": ig["sym_hash"] == info_host["sym_hash"]}


def fp32_ir_leg(args, A0, opts, vals, bs, xs, xts, v0, run, x64, timed):
    """The same workload with FP32 factors and FP64 refinement, to a backward
    error of 1e-10 and of 1e-12: ms per step, backward error, refinement
    steps and the difference from the FP64 solution."""
    import torch
    from paper_2509_07690_amd import hylu
    out = {}
    for tol in (1e-10, 1e-12):
        hf = hylu.Handle(A0.row_ptr, A0.col, A0.val, precision="fp32", ir_tol=tol, **opts)
        hf.factorize(v0)
        if args.autotune:
            hf.autotune(v0, reps=2)
        ms, tr, tsv, idx = run(hf, args.steps, args.warmup)
        r = idx[-1]
        eta, res1 = hf.residual(bs[r], xs[r])
        inf = hf.info()
        d = float((xs[r] - x64).abs().max() / x64.abs().max()) if r == timed[-1] else None
        out[f"{tol:.0e}"] = {"ms_per_step": round(ms, 4), "refactor_ms_median": round(tr, 4),
                             "solve_ms_median": round(tsv, 4), "backward_error": eta, "resid_1": res1,
                             "ir_iters": inf["ir_iters"], "n_perturbed": inf["n_perturbed"],
                             "rel_diff_vs_fp64": d,
                             "max_abs_err_vs_x_true": float(np.abs(xs[r].cpu().numpy() - xts[r]).max())}
        hf.close()
        torch.cuda.synchronize()
    return out


def bench_copy(args):
    """A plain device copy of 1 GiB (3 times): the reference that scales the
    HBM counters (FETCH_SIZE, WRITE_SIZE) to bytes."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copies": 3}))


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "circuit_n200000_hbm_traffic.md")
# kernel class -> (kernel family, first and last marker of its source in kernels.hip)
TRAFFIC_SOURCES = {
    "rows": ("k_factor_rows", "__device__ void apply_source_direct(", "// pipeline mode (Sec. 2.2.1): the narrow levels"),
    "tail_gemm": ("k_tail_gemm", "template <typename T> struct Mfma;", "// ---- row tiles of supernode targets"),
}


def _kernel_source_hash(cls):
    """Hash of a kernel class's source text: counter figures taken for
    another version of the kernel are not reported."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2509_07690_amd", "csrc", "kernels.hip")).read()
    _, first, last = TRAFFIC_SOURCES[cls]
    a = src.index(first)
    b = src.index(last, a)
    return hashlib.sha1(src[a:b].encode()).hexdigest()[:16]


def _traffic(cls):
    """Measured HBM bytes per launch of a kernel class from the committed
    counter profile, when it was taken for the current kernel source."""
    if cls not in TRAFFIC_SOURCES:
        return None
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"traffic_json: (\{.*\})", txt)
    if not m:
        return None
    d = json.loads(m.group(1)).get(cls)
    if not d or d.get("source_hash") != _kernel_source_hash(cls):
        return None
    return d


def _timed(fn, steps, warmup):
    """Runs fn() warmup times, then times `steps` calls between two device
    synchronisations; returns ms per call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def _line(metric, value, unit, args, dtype, config, **extra):
    out = {"metric": metric, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(value, 4), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out))


def batch_leg(members, precision, steps, warmup, sn_dense=64, sn_inverse=1, sn_tile=0):
    """The uneven batch: `members` matrices (even: local circuits n ~ U{2000..
    50000}; odd: 9-point grids, side ~ U{32..160}) on one handle; a step
    refactorises every member with its fresh values (one graph) and solves one
    right-hand side each.  Launch shapes come from the autotuner (untimed)."""
    import torch
    from paper_2509_07690_amd import synth, hylu
    dev = torch.device("cuda:0")
    t0 = time.time()
    ws = [synth.batch_member(m) for m in range(members)]
    a0 = [w.extra["analyze_values"] for w in ws]
    log(f"batch: members {len(ws)} n={sum(w.A.n for w in ws)} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    hb = hylu.Handle.batch([(a.row_ptr, a.col, a.val) for a in a0], precision=precision, sn_dense=sn_dense,
                           sn_inverse=sn_inverse, sn_tile=sn_tile)
    t_an = time.time() - t0
    inf = hb.info()
    log(f"batch: analyze {t_an:.1f}s F={inf['flops']:.3e} levels={inf['n_levels']}")
    v0 = torch.from_numpy(np.concatenate([a.val for a in a0])).to(dev)
    v1 = torch.from_numpy(np.concatenate([w.A.val for w in ws])).to(dev)
    b = torch.from_numpy(np.concatenate([w.b[:, 0] for w in ws])).to(dev)
    x = torch.empty_like(b)
    hb.factorize(v0)
    t_def, t_tuned = hb.autotune(v1, reps=2)
    log(f"batch: autotune level time {t_def:.2f} ms with built-in shapes, {t_tuned:.2f} ms tuned")

    def step():
        hb.refactor(v1)
        hb.solve(b, out=x)
    ms = _timed(step, steps, warmup)
    t_ref = _timed(lambda: hb.refactor(v1), steps, 1)
    eta, res1 = hb.residual(b, x)
    prof = hb.profile(v1, b, torch.empty_like(b))
    kernels = {k["name"]: {"launches": k["launches"], "ms": round(k["ms"], 3)} for k in prof}
    roff, _ = hb.offsets()
    xs = x.cpu().numpy()
    err = max(float(np.abs(xs[roff[k]:roff[k + 1]] - w.x_true[:, 0]).max()) for k, w in enumerate(ws))
    info = hb.info()
    res = {"metric": f"batch refactor+solve ms ({len(ws)} uneven matrices, one handle)", "ms_per_step": round(ms, 4),
           "precision": precision, "steps": steps,
           "config": {"workload": f"uneven batch of {len(ws)}: circuits n~U[2000,50000] + 9-pt grids side~U[32,160]",
                      "members": len(ws), "n_total": hb.n, "nnz_total": hb.nnz},
           "refactor_ms": round(t_ref, 4), "factor_gflops": round(info["flops"] / (t_ref * 1e-3) / 1e9, 3),
           "flops": info["flops"], "autotune_level_ms": {"builtin": round(t_def, 3), "tuned": round(t_tuned, 3)},
           "backward_error": eta, "resid_1": res1, "max_abs_err_vs_x_true": err, "ir_iters": info["ir_iters"],
           "analyze_s": round(t_an, 2), "kernels": kernels}
    hb.close()
    res["symbolic"] = symbolic_compare(info, lambda: hylu.Handle.batch(
        [(a.row_ptr, a.col, a.val) for a in a0], precision=precision, sn_dense=sn_dense, sn_inverse=sn_inverse,
        sn_tile=sn_tile, gpu_symbolic=1))
    return res


def grid27_leg(side, precision, steps, warmup, dense_tail=0.5, sn_tile=0, sn_dense=64, sn_inverse=1, tail_sparse=1):
    """27-point 3D convection-diffusion on side^3 (nested dissection with
    multilevel separators), 8 RHS."""
    import torch
    from paper_2509_07690_amd import synth, hylu
    w = synth.convdiff3d_27pt(side)
    A = w.A
    t0 = time.time()
    h = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd_ml", precision=precision, dense_tail=dense_tail,
                    sn_tile=sn_tile, sn_dense=sn_dense, sn_inverse=sn_inverse, tail_sparse=tail_sparse)
    t_an = time.time() - t0
    log(f"grid27 {precision}: analyze {t_an:.1f}s F={h.info()['flops']:.3e} tail={h.info()['tail_rows']}")
    v = torch.from_numpy(A.val).cuda()
    B = torch.from_numpy(np.ascontiguousarray(w.b.T)).cuda()       # (8, n): column-major RHS
    X = torch.empty_like(B)
    t0 = time.time()
    h.factorize(v)
    torch.cuda.synchronize()
    log(f"grid27 {precision}: factorize {time.time() - t0:.2f}s")
    t0 = time.time()
    t_def, t_tuned = h.autotune(v, reps=1)      # launch shapes per level (untimed setup)
    tune = {"builtin": round(t_def, 3), "tuned": round(t_tuned, 3), "s": round(time.time() - t0, 2)}
    log(f"grid27 {precision}: autotune level time {t_def:.1f} ms with built-in shapes, {t_tuned:.1f} ms tuned "
        f"({tune['s']} s)")
    ms = _timed(lambda: (h.refactor(v), h.solve_cols(B, out=X)), steps, warmup)
    t_ref = _timed(lambda: h.refactor(v), steps, 1)
    h.solve_cols(B, out=X)
    eta, res1 = h.residual(B, X)
    prof = h.profile(v, B[0].contiguous(), torch.empty_like(B[0]))
    kernels = {k["name"]: {"launches": k["launches"], "ms": round(k["ms"], 3),
                           "TFLOPs": round(k["flops"] / max(k["ms"], 1e-9) / 1e9, 3)} for k in prof}
    info = h.info()
    res = {"metric": f"refactor+solve ms (27-pt grid {side}^3, 8 rhs)", "ms_per_step": round(ms, 4),
           "precision": precision, "steps": steps,
           "config": {"workload": f"convdiff3d_27pt side={side} n={A.n} nnz={A.nnz}, 8 rhs"},
           "refactor_ms": round(t_ref, 4), "factor_gflops": round(info["flops"] / (t_ref * 1e-3) / 1e9, 3),
           "flops": info["flops"], "flops_issued": info["flops_issued"], "backward_error": eta, "resid_1": res1,
           "ir_iters": info["ir_iters"], "analyze_s": round(t_an, 2), "tail_rows": info["tail_rows"],
           "autotune_level_ms": tune, "kernels_one_rhs": kernels}
    h.close()
    return res


def adjoint_leg(side, steps, warmup, dense_tail=0.15, sn_dense=64, sn_inverse=1, tail_sparse=1, sn_tile=0):
    """x = A^{-1} b and the gradient of 0.5||x - x_target||^2 with respect to
    the values of A and b, on the 7-point grid side^3 (ND): forward
    (refactor + solve) and backward (transposed solve + pattern gradient)."""
    import torch
    from paper_2509_07690_amd import synth, hylu
    w = synth.convdiff3d_7pt(side)
    A = w.A
    t0 = time.time()
    h = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd", dense_tail=dense_tail, sn_dense=sn_dense,
                    sn_inverse=sn_inverse, tail_sparse=tail_sparse, sn_tile=sn_tile)
    t_an = time.time() - t0
    v = torch.from_numpy(A.val).cuda()
    b = torch.from_numpy(np.ascontiguousarray(w.b[:, 0])).cuda()
    xt = torch.from_numpy(w.extra["x_target"]).cuda()
    h.factorize(v)
    t0 = time.time()
    t_def, t_tuned = h.autotune(v, reps=2)      # launch shapes per level (untimed setup)
    tune = {"builtin": round(t_def, 3), "tuned": round(t_tuned, 3), "s": round(time.time() - t0, 2)}

    def fwd():
        return hylu.sparse_solve(h, v, b)

    grads = {}

    def fwd_bwd():
        vv = v.clone().requires_grad_()
        bb = b.clone().requires_grad_()
        x = hylu.sparse_solve(h, vv, bb)
        (0.5 * ((x - xt) ** 2).sum()).backward()
        grads["x"], grads["lam"] = x.detach(), bb.grad
    t_f = _timed(fwd, steps, warmup)
    t_fb = _timed(fwd_bwd, steps, warmup)
    eta, _ = h.residual(b, grads["x"])
    eta_t, _ = h.residual((grads["x"] - xt).contiguous(), grads["lam"], transpose=True)
    res = {"metric": f"adjoint forward+backward ms (7-pt grid {side}^3)", "ms_per_step": round(t_fb, 4),
           "precision": "fp64", "steps": steps,
           "config": {"workload": f"convdiff3d_7pt side={side} n={A.n} nnz={A.nnz}, loss 0.5||x-x_target||^2"},
           "forward_ms": round(t_f, 4), "backward_ms": round(t_fb - t_f, 4), "flops": h.info()["flops"],
           "backward_error": eta, "backward_error_transposed": eta_t, "analyze_s": round(t_an, 2),
           "autotune_level_ms": tune}
    h.close()
    return res


def _print_leg(res, args):
    extra = {k: v for k, v in res.items() if k not in ("metric", "ms_per_step", "precision", "steps", "config")}
    _line(res["metric"], res["ms_per_step"], "ms", args, "f64" if res["precision"] == "fp64" else "f32+f64ir",
          dict(res["config"], precision=res["precision"]), **extra)


def bench_batch(args):
    _print_leg(batch_leg(args.members, args.precision, args.steps, args.warmup, args.sn_dense, args.sn_inverse,
                         args.sn_tile), args)


def bench_grid27(args):
    side = args.n if args.n != 200000 else 64
    _print_leg(grid27_leg(side, args.precision, args.steps, args.warmup, args.dense_tail if args.dense_tail != 0.15
                          else 0.5, args.sn_tile, args.sn_dense, args.sn_inverse, args.tail_sparse), args)


def bench_adjoint(args):
    side = args.n if args.n != 200000 else 48
    _print_leg(adjoint_leg(side, args.steps, args.warmup, args.dense_tail, args.sn_dense, args.sn_inverse,
                           args.tail_sparse, args.sn_tile), args)


def other_configs(args):
    """The other workloads, each briefly (a few steps): the 27-point 64^3 grid
    in FP64 and FP32 + refinement, the 256-member uneven batch in FP64 and FP32
    + refinement, and the adjoint on the 7-point 48^3 grid."""
    out = {}
    import torch
    for key, fn in (("grid27_64_fp64", lambda: grid27_leg(64, "fp64", 3, 1)),
                    ("grid27_64_fp32_ir", lambda: grid27_leg(64, "fp32", 3, 1)),
                    ("batch256_fp64", lambda: batch_leg(256, "fp64", 5, 1)),
                    ("batch256_fp32_ir", lambda: batch_leg(256, "fp32", 5, 1)),
                    ("adjoint_grid7_48", lambda: adjoint_leg(48, 5, 1))):
        t0 = time.time()
        out[key] = fn()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"{key}: {out[key]['ms_per_step']} ms per step ({time.time() - t0:.1f}s)")
    return out


def cpu_baseline(A0, base, h, nref, first):
    """The CPU oracle (plain single-threaded FP64 C) on a bounded sample of the
    same workload: `nref` refactor+solve steps with the same permutations and
    scalings, timed on the host (symbolic analysis excluded)."""
    import oracle
    sym = h.symbolic()
    o = oracle.Oracle(A0.n, A0.row_ptr, A0.col, A0.val, sym["perm_r"], sym["perm_c"], sym["dr"], sym["dc"])
    t = time.perf_counter()
    o.analyse()
    t_sym = time.perf_counter() - t
    tau = o.pivot_tau()                 # from the oracle's own B (analysed values)
    o.numeric(tau)
    piv = o.factors()[-1]
    times = []
    for r in range(nref):
        w = base.revalue(first + r + 1)
        o.set_values(w.A.val)
        t = time.perf_counter()
        o.numeric(tau, piv=piv)
        x = o.solve(w.b[:, 0])
        times.append(time.perf_counter() - t)
    err = float(np.abs(x - w.x_true[:, 0]).max())
    return {"value": round(1e3 * float(np.median(times)), 2), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"{nref} refactor+solve step(s) of the same n={A0.n} workload, FP64, single thread, "
                      f"symbolic ({t_sym:.1f}s) excluded", "max_abs_err_vs_x_true": err,
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "host_cpus_usable": len(os.sched_getaffinity(0))}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
