#!/usr/bin/env python3
"""Benchmark: effective TFLOP/s (2mkn/t) of recursive fast matrix multiplication on one
MI355X, beside the classical GEMM built the same way (same precision form, one leaf), with the
max-norm relative error of both against the long-double CPU reference.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--algo winograd] [--depth 1]
                    [--n 8192] [--precision f16x3] [--beside f32] [--scaling none]
                    [--dist uniform01] [--fuse auto] [--also none]

Default workload (the precision-form configuration): Strassen <2,2,2;7>, depth 2, cutoff 256,
n = 16384, N(0,1) entries, outside scaling (Algorithm 1, each factor the power of two nearest to
the row's or column's max-abs), leaves as FP16
MFMA products with FP32 accumulation in the two-limb split form (F16X3).  Beside it in the same
line: the classical GEMM built the same way (same precision form, same scaling, one leaf), the
same plan on plain FP32 MFMA, and the <4,2,4;26> rule at the same depth, size, scaling and
precision.  Prints one JSON line.  A step is one fastmm_gemm call (scaling reductions, operand
formation, products, W-combination) on inputs already resident in HBM.  The products kernel's
average duration comes from HIP events the library records on its launch stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "effective TFLOP/s (2mkn/t) and max-norm rel error vs FP64 oracle, fast vs classical"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "bf16x3": 2500.0, "f16x3": 2500.0,
               "bf16x6": 2500.0}
PEAK_TFLOPS_BY_DTYPE = {"float64": 78.6, "float32": 157.3, "float16": 2500.0, "bfloat16": 2500.0}
PRODUCTS = {"f64": 1, "f32": 1, "bf16": 1, "f16": 1, "bf16x3": 3, "f16x3": 3, "bf16x6": 6}
HBM_PEAK_GBS = 8000.0
ORACLE_NAME = {"strassen": "strassen", "winograd": "winograd", "f323": "f323", "f332": "f332", "f233": "f233",
               "f442": "f442", "f424": "f424", "f244": "f244", "laderman333": "laderman333"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--algo", default="strassen")
    ap.add_argument("--depth", type=int, default=2)
    ap.add_argument("--cutoff", type=int, default=256)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--precision", default="f16x3",
                    help="leaf arithmetic: f64, f32, or a split form (bf16, f16, bf16x3, f16x3, bf16x6)")
    ap.add_argument("--beside", default="f32",
                    help="also time the same plan in this precision (reported beside the headline; none = skip)")
    ap.add_argument("--scaling", default="outside")
    ap.add_argument("--scaling-steps", type=int, default=2)
    ap.add_argument("--o-round", default="nearest", choices=["up", "nearest"],
                    help="O-step factors: the nearest power of two to the max (default), or the smallest "
                         "one >= it")
    ap.add_argument("--per-level", action="store_true",
                    help="run the scaling steps at every inner node of the recursion, not only once")
    ap.add_argument("--dist", default="normal")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--err-rows", type=int, default=16)
    ap.add_argument("--cpu-n", type=int, default=8192,
                    help="size of the oracle timing sample (same algorithm, depth and distribution)")
    ap.add_argument("--also", default="f424",
                    help="also time this rule at the same depth, size, scaling and precision (none = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-classical", action="store_true")
    ap.add_argument("--fuse", default="auto", choices=["auto", "off", "always", "written"],
                    help="fusion mode of the plan (off: leaf products from composite source lists; "
                         "written: written-out leaf operands, never the fused kernel)")
    ap.add_argument("--no-vendor", action="store_true",
                    help="skip timing torch.bmm (hipBLASLt) on the leaf products' shape")
    ap.add_argument("--torch-ref", action="store_true",
                    help="also time torch.matmul (vendor BLAS) on the same operands, as context")
    ap.add_argument("--batch", type=int, default=0,
                    help="time a batch of this many rectangular problems (dims drawn from 512..8192) with "
                         "autotuned plans in one batched launch, instead of the single-product workload")
    ap.add_argument("--scaling-study", action="store_true",
                    help="the section 6.5 scaling study on the GPU (FP64 Strassen, L = 1..6, the seven "
                         "scaling schedules, the three distributions, componentwise error) instead of the "
                         "throughput workload")
    ap.add_argument("--study-n", type=int, default=2000)
    ap.add_argument("--study-pairs", type=int, default=5)
    ap.add_argument("--study-rows", type=int, default=32, help="sampled rows per product for the error")
    ap.add_argument("--study-dist", default="fig3", choices=["fig3", "badly"],
                    help="the three distributions of section 6.5, or D1 R D2 with diagonals 10^u, "
                         "u ~ U(-6, 6) per row / column")
    ap.add_argument("--study-max-depth", type=int, default=6)
    ap.add_argument("--study-precision", default="f64", help="f64, f32 or a split form")
    ap.add_argument("--tune-cache", default="", help="JSON cache of the autotuner's choices (batch mode)")
    ap.add_argument("--max-instability", type=float, default=16.0,
                    help="autotuner admission cap on (E/K0^2)^L (batch mode)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the product kernel's HBM bytes per launch for this workload into "
                         "profiles/traffic.json from two rocprofv3 counter runs (--pmc FETCH_SIZE, then "
                         "--pmc WRITE_SIZE) of this command with --no-classical --beside none --also none "
                         "--calib-copy-mb MB; runs on the host only")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB (calibrates rocprofv3 byte counters)")
    return ap.parse_args()


def time_steps(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def product_kernel(precision: str, path: str):
    """(kernel name, source file) of the launch that computes the products."""
    if path == "fused":
        return "fmm_node222", "node_fused.h"
    if path == "fused_loads":
        return "fmm_limb_fused", "limb_gemm.hip"
    if precision in ("f64", "f32"):  # leaf and written paths
        return "fmm_leaf_pipelined", "leaf_mfma.hip"
    return "fmm_limb_gemm", "limb_gemm.hip"


def kernel_source_hash(source: str) -> str:
    with open(os.path.join(ROOT, "paper_1507_00687_amd", "csrc", source), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload: str, source: str):
    """HBM bytes per product-kernel launch from committed rocprofv3 counter runs, if they were
    taken with the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except Exception:
        return None
    if not rec or rec.get("source") != source or rec.get("source_hash") != kernel_source_hash(source):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline_leg(args, A, B, rows):
    """Everything that touches the CPU oracle: the long-double reference rows for the error
    figures, and the oracle's own fast multiplication timed on a bounded sample."""
    import numpy as np

    from oracle import coeffs as C
    from oracle import fastmm_oracle as O
    from synth import make_pair

    A64 = A.astype(np.float64)
    B64 = B.astype(np.float64)
    ref = O.reference_rows(A64, B64, rows)
    out = {"ref": ref}
    if not args.no_cpu:
        n = args.cpu_n
        As, Bs = make_pair(args.dist, args.seed, n, n, n, dtype=np.float64)
        alg = C.get(ORACLE_NAME[args.algo]) if args.algo in ORACLE_NAME else None
        cutoff = min(args.cutoff, max(1, n // (2 ** args.depth)))
        t0 = time.perf_counter()
        if alg is None or args.depth == 0:
            alg, depth = C.get("strassen"), 0
        else:
            depth = args.depth
        if args.scaling != "none":
            O.scaled_fast(As, Bs, alg, depth, cutoff, mode=args.scaling, steps=args.scaling_steps,
                          o_round=args.o_round)
        else:
            O.fast(As, Bs, alg, depth, cutoff)
        dt = time.perf_counter() - t0
        sc = f", {args.scaling} scaling (power-of-two factors)" if args.scaling != "none" else ""
        out["cpu"] = {"value": 2.0 * n ** 3 / dt / 1e12, "unit": "TFLOP/s", "cores": O.num_threads(),
                      "kind": "oracle",
                      "sample": f"oracle fast FP64 ({args.algo}, depth {args.depth}{sc}) on one {n}^3 product "
                                f"of the same distribution, {dt:.2f} s; plain C classical leaves, "
                                f"sequential summation"}
    return out


def vendor_leaf_gemm(args, nleaves, mb, kb, nb, achieved):
    """The vendor library on the leaf products' shape, for context: torch.bmm (hipBLASLt) over
    nleaves independent mb x kb x nb products of N(0,1) data in the MFMA input type of the
    precision (fp16 for the fp16 limb forms, bf16 for the bf16 ones, else the precision itself).
    The MFMA rate depends on the data (operands of few significant bits draw less power and run
    at higher clocks), so the comparison uses full-mantissa values, as the limb planes are."""
    import torch

    dt = {"f16": torch.float16, "f16x3": torch.float16, "bf16": torch.bfloat16, "bf16x3": torch.bfloat16,
          "bf16x6": torch.bfloat16, "f32": torch.float32, "f64": torch.float64}[args.precision]
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    X = torch.randn((nleaves, mb, kb), dtype=torch.float32, device="cuda", generator=g).to(dt)
    Y = torch.randn((nleaves, kb, nb), dtype=torch.float32, device="cuda", generator=g).to(dt).contiguous()
    ms_v = time_steps(lambda: torch.bmm(X, Y), args.steps, args.warmup)
    v = 2.0 * nleaves * mb * kb * nb / (ms_v * 1e-3) / 1e12
    # its error on the first product (max-norm, relative to max|X| max|Y|) against FP64: shows
    # the arithmetic the library used (a reduced-precision internal type would show here)
    Z = torch.bmm(X[:1], Y[:1])[0].double()
    Zr = X[0].double() @ Y[0].double()
    err = ((Z - Zr).abs().max() / (X[0].double().abs().max() * Y[0].double().abs().max())).item()
    del X, Y, Z, Zr
    return {"what": f"torch.bmm {str(dt).replace('torch.', '')} (hipBLASLt), {nleaves} x {mb}x{kb}x{nb}, N(0,1)",
            "ms": ms_v, "value": v, "frac": v / PEAK_TFLOPS_BY_DTYPE[str(dt).replace("torch.", "")],
            "product_kernel_over_vendor": achieved / v, "first_product_error": err}


def leaf_flops(F, plan_algo, plan, m, k, n, precision):
    """Product flops one launch executes for a plan on (m, k, n): leaves x limb products x 2 mb kb nb."""
    L, Mp, Kp, Np = plan.shape(m, k, n)
    if plan_algo == "classical" or L == 0:
        return 2.0 * Mp * Kp * Np * PRODUCTS[precision]
    info = F.fastmm_algo_info(plan_algo)
    mb, kb, nb = Mp // info["M0"] ** L, Kp // info["K0"] ** L, Np // info["N0"] ** L
    return 2.0 * mb * kb * nb * info["R"] ** L * PRODUCTS[precision]


def batch_main(args):
    """A batch of rectangular problems (dims drawn from {512, ..., 8192}, tall-skinny included,
    N(0,1) entries from the seeded host generator), plans chosen per shape by the autotuner; a
    step is one training step of the batch: the forward products in one fastmm_gemm_batched call,
    then the gradients dA_i = G_i B_i^T, dB_i = A_i^T G_i of every problem in one
    fastmm_gemm_backward_batched call.  The same batch with classical plans beside."""
    import numpy as np
    import torch

    import paper_1507_00687_amd as F
    from paper_1507_00687_amd import tune as T
    from synth import make_pair
    from synth.gen import TAG_G, normal01

    torch.cuda.set_device(0)
    rng = np.random.default_rng(args.seed)
    dims = np.array([512, 1024, 2048, 4096, 8192])
    shapes = [tuple(int(x) for x in rng.choice(dims, 3)) for _ in range(args.batch)]
    ndt = np.float64 if args.precision == "f64" else np.float32
    t0 = time.perf_counter()
    hostA, hostB, hostG = [], [], []
    for i, (m, k, n) in enumerate(shapes):
        A, B = make_pair("normal", args.seed + i, m, k, n, dtype=ndt)
        hostA.append(A)
        hostB.append(B)
        hostG.append(normal01(args.seed + i, TAG_G, (m, n)).astype(ndt))
    gen_s = time.perf_counter() - t0
    As = [torch.from_numpy(X).cuda() for X in hostA]
    Bs = [torch.from_numpy(X).cuda() for X in hostB]
    Gs = [torch.from_numpy(X).cuda() for X in hostG]
    Cs = [torch.empty((m, n), dtype=As[0].dtype, device="cuda") for m, k, n in shapes]
    t0 = time.perf_counter()
    choices = T.tune(shapes, precision=args.precision, cache=args.tune_cache or None, max_depth=2,
                     cutoffs=(128, 256, 512), max_instability=args.max_instability, reps=2)
    tune_s = time.perf_counter() - t0
    plans = [choices[sh].plan(args.precision) for sh in shapes]
    cplans = [F.Plan("classical", 0, 1, precision=args.precision) for _ in shapes]
    ws = torch.empty(max(F.fastmm_batched_workspace_size(plans, As, Bs), 1), dtype=torch.uint8, device="cuda")
    cws = torch.empty(max(F.fastmm_batched_workspace_size(cplans, As, Bs), 1), dtype=torch.uint8, device="cuda")
    Cc = [torch.empty_like(c) for c in Cs]
    flops = sum(2.0 * m * k * n for m, k, n in shapes)
    fwd = lambda: F.fastmm_gemm_batched(plans, As, Bs, Cs, workspace=ws)
    grads = {}
    bwd = lambda: grads.__setitem__("fast", F.fastmm_gemm_backward_batched(plans, As, Bs, Gs))
    cbwd = lambda: grads.__setitem__("classical", F.fastmm_gemm_backward_batched(cplans, As, Bs, Gs))
    ms_cls = time_steps(lambda: F.fastmm_gemm_batched(cplans, As, Bs, Cc, workspace=cws), args.steps, args.warmup)
    ms_cls_b = time_steps(cbwd, args.steps, args.warmup)
    ms = time_steps(fwd, args.steps, args.warmup)
    ms_b = time_steps(bwd, args.steps, args.warmup)

    F.fastmm_profile_enable(True)
    F.fastmm_profile_read()
    for _ in range(args.steps):
        fwd()
    prof = F.fastmm_profile_read()
    for _ in range(args.steps):
        bwd()
    prof_b = F.fastmm_profile_read()
    F.fastmm_profile_enable(False)
    calls = max(prof["calls"], 1)
    calls_b = max(prof_b["calls"], 1)
    leaf_ms = prof["leaf_ms"] / calls
    executed = sum(leaf_flops(F, choices[sh].algo, p, *sh, args.precision) for sh, p in zip(shapes, plans))
    achieved = executed / (leaf_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]

    # errors of a few problems on sampled rows against the long-double reference (oracle leg):
    # C = A B, dA = G B^T, dB = A^T G
    from oracle import fastmm_oracle as O

    err = {"fast": 0.0, "classical": 0.0, "fast_dA": 0.0, "fast_dB": 0.0, "classical_dA": 0.0,
           "classical_dB": 0.0}
    sampled = np.unique(np.linspace(0, len(shapes) - 1, 4).astype(int))
    for i in sampled:
        m, k, n = shapes[i]
        A64, B64, G64 = (X.astype(np.float64) for X in (hostA[i], hostB[i], hostG[i]))
        rows = np.unique(np.linspace(0, m - 1, 4).astype(np.int64))
        ref = O.reference_rows(A64, B64, rows)
        err["fast"] = max(err["fast"], O.normwise_error(Cs[i].cpu().numpy(), ref, A64, B64, rows))
        err["classical"] = max(err["classical"], O.normwise_error(Cc[i].cpu().numpy(), ref, A64, B64, rows))
        Bt, At = np.ascontiguousarray(B64.T), np.ascontiguousarray(A64.T)
        rows_b = np.unique(np.linspace(0, k - 1, 4).astype(np.int64))
        ref_a = O.reference_rows(G64, Bt, rows)
        ref_b = O.reference_rows(At, G64, rows_b)
        for key in ("fast", "classical"):
            dA, dB = grads[key][i]
            err[key + "_dA"] = max(err[key + "_dA"], O.normwise_error(dA.cpu().numpy(), ref_a, G64, Bt, rows))
            err[key + "_dB"] = max(err[key + "_dB"], O.normwise_error(dB.cpu().numpy(), ref_b, At, G64, rows_b))
    # the oracle timed on the largest problems of the batch with their tuned plans, until about
    # 10 s of CPU work (at most 4 problems)
    cpu = None
    if not args.no_cpu:
        from oracle import coeffs as C

        order = sorted(range(len(shapes)), key=lambda j: -shapes[j][0] * shapes[j][1] * shapes[j][2])
        done, fl_cpu, dt_cpu = [], 0.0, 0.0
        for i in order[:4]:
            m, k, n = shapes[i]
            c = choices[shapes[i]]
            A64, B64 = hostA[i].astype(np.float64), hostB[i].astype(np.float64)
            t0 = time.perf_counter()
            if c.depth == 0 or c.algo == "classical" or c.levels:
                O.classical(A64, B64)
            else:
                O.fast(A64, B64, C.get(ORACLE_NAME.get(c.algo, c.algo)), c.depth, c.cutoff)
            dt_cpu += time.perf_counter() - t0
            fl_cpu += 2.0 * m * k * n
            done.append(f"{m}x{k}x{n} {c.algo} L={c.depth}")
            if dt_cpu >= 10.0:
                break
        cpu = {"value": fl_cpu / dt_cpu / 1e12, "unit": "TFLOP/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"oracle FP64 forward of the largest problems of the batch ({', '.join(done)}), "
                         f"{dt_cpu:.2f} s"}
    mix = {}
    for sh in shapes:
        c = choices[sh]
        key = f"{c.algo} L={c.depth}" if c.depth else "classical"
        mix[key] = mix.get(key, 0) + 1
    kname = "fmm_limb_gemm_batched" if args.precision in ("bf16", "f16", "bf16x3", "f16x3", "bf16x6") else \
        "fmm_leaf_batched"
    total = ms + ms_b
    line = {
        "metric": METRIC,
        "value": 3.0 * flops / (total * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"batch of {len(shapes)} problems, dims from 512..8192 (seed {args.seed}), "
                               f"autotuned plans, {args.precision}, N(0,1), forward + backward",
                   "problems": len(shapes), "flops_2mkn": flops, "plan_mix": mix, "generation_s": gen_s,
                   "tuning_s": tune_s, "max_instability": args.max_instability},
        "forward": {"ms_per_step": ms, "value": flops / (ms * 1e-3) / 1e12},
        "backward": {"ms_per_step": ms_b, "value": 2.0 * flops / (ms_b * 1e-3) / 1e12,
                     "launches": "one fastmm_gemm_backward_batched call (dA and dB of every problem, one "
                                 "products launch)"},
        "classical": {"ms_per_step": ms_cls + ms_cls_b, "forward_ms": ms_cls, "backward_ms": ms_cls_b,
                      "value": 3.0 * flops / ((ms_cls + ms_cls_b) * 1e-3) / 1e12},
        "speedup_vs_classical": (ms_cls + ms_cls_b) / total,
        "error": dict(err, problems_sampled=len(sampled), rows_per_problem=4,
                      reference="long double classical (oracle)"),
        "phases_ms": {"scaling": prof["scaling_ms"] / calls, "form": prof["form_ms"] / calls, "leaf": leaf_ms,
                      "combine": prof["combine_ms"] / calls},
        "phases_ms_backward": {"scaling": prof_b["scaling_ms"] / calls_b, "form": prof_b["form_ms"] / calls_b,
                               "leaf": prof_b["leaf_ms"] / calls_b, "combine": prof_b["combine_ms"] / calls_b},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": kname, "flops_per_launch": executed,
                     "launch": "forward products"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def scaling_study(args):
    """Componentwise error max_ij |c^_ij - c_ij| / |c_ij| (over sampled rows, maximum over the
    pairs) of Strassen's algorithm in FP64 on the GPU, L = 1..6, for the seven scaling schedules
    and the three input distributions of section 6.5 (with --per-level, also each schedule run at
    every inner node of the recursion); the long-double oracle gives c."""
    import numpy as np
    import torch

    import paper_1507_00687_amd as F
    from oracle import fastmm_oracle as O
    from synth.gen import badly_scaled, fig3_pair

    torch.cuda.set_device(0)
    n = args.study_n
    depths = list(range(1, args.study_max_depth + 1))
    prec = args.study_precision
    dt = np.float64 if prec == "f64" else np.float32
    # the three distributions of section 6.5, or the row/column-scaled D1 R D2 inputs
    dists = [("badly", lambda seed: badly_scaled(seed, n, n, n))] if args.study_dist == "badly" else \
        [(f"dist{d}", (lambda d: lambda seed: fig3_pair(seed, n, d))(d)) for d in (1, 2, 3)]
    schedules = [(m, s, False) for m, s in [("none", 2), ("outside", 2), ("inside", 2), ("out_in", 2),
                                              ("in_out", 2), ("repeated", 4), ("repeated", 20)]]
    if args.per_level:  # the same schedules run at every inner node as well
        schedules += [(m, s, True) for m, s, _ in schedules if m != "none"]
    rows = np.unique(np.linspace(0, n - 1, args.study_rows).astype(np.int64))
    table = {}
    t0 = time.perf_counter()
    gpu_ms = 0.0
    normwise = {}
    for name, gen in dists:
        pairs = [gen(1000 + p) for p in range(args.study_pairs)]
        refs = [O.reference_rows(A, B, rows) for A, B in pairs]
        dev = [(torch.from_numpy(A.astype(dt)).cuda(), torch.from_numpy(B.astype(dt)).cuda()) for A, B in pairs]
        for depth in depths:
            for mode, steps, every in schedules:
                key = (f"{mode}{steps}" if mode == "repeated" else mode) + ("_every_level" if every else "")
                plan = F.Plan("strassen", depth, 1, scaling=mode, steps=steps, precision=prec, per_level=every)
                err = errn = 0.0
                for (A, B), (tA, tB), ref in zip(pairs, dev, refs):
                    ta = time.perf_counter()
                    Cg = F.fastmm_gemm(plan, tA, tB)
                    torch.cuda.synchronize()
                    gpu_ms += (time.perf_counter() - ta) * 1e3
                    got = Cg[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
                    if not np.all(np.isfinite(got)):  # overflow (e.g. fp16 limbs of unscaled inputs)
                        err = errn = float("inf")
                        continue
                    err = max(err, O.componentwise_error(got, ref))
                    errn = max(errn, float(np.max(np.abs(got.astype(np.longdouble) - ref))) /
                               (float(np.max(np.abs(A))) * float(np.max(np.abs(B)))))
                table.setdefault(name, {}).setdefault(key, []).append(err)
                normwise.setdefault(name, {}).setdefault(key, []).append(errn)
        print(f"{name} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    line = {
        "metric": f"componentwise relative error of Strassen ({prec}, GPU) under the section 6.5 scaling "
                  "schedules, max over pairs and sampled rows; index = L - 1",
        "value": None,
        "unit": "relative error",
        "n_gpus": 1,
        "steps": None,
        "warmup": None,
        "ms_per_step": gpu_ms / (len(dists) * len(depths) * len(schedules) * args.study_pairs),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"scaling study: N={n}, {args.study_pairs} pairs per distribution, "
                               f"{len(rows)} sampled rows, Strassen L=1..{depths[-1]} (cutoff 1), "
                               f"inputs {args.study_dist}",
                   "schedules": [(f"{m}{s}" if m == "repeated" else m) + ("_every_level" if e else "")
                                 for m, s, e in schedules]},
        "errors": table,
        "normwise_errors": normwise,
    }
    print(json.dumps(line), flush=True)


def record_traffic(args):
    """Median FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the product kernel in two rocprofv3
    counter runs, each scaled by what the counter reads for the calibration copy of
    --calib-copy-mb MiB (its true bytes read and written), into profiles/traffic.json under this
    workload's key, with the hash of the kernel's source (bench lines report the bytes only while
    the source is unchanged)."""
    import csv
    import statistics

    import paper_1507_00687_amd as F

    if args.calib_copy_mb <= 0:
        sys.exit("--record-traffic needs --calib-copy-mb (the copy the counters are scaled by)")
    n = args.n
    plan = F.Plan(args.algo, args.depth, args.cutoff, scaling=args.scaling, steps=args.scaling_steps,
                  precision=args.precision, fuse=args.fuse, per_level=args.per_level, o_round=args.o_round)
    path = plan.path(n, n, n)
    kname, ksource = product_kernel(args.precision, path)
    workload = (f"{args.algo} L={args.depth} cutoff={args.cutoff} n={n} {args.precision} {args.dist} "
                f"scaling={args.scaling}{' per-level' if args.per_level else ''}"
                f"{' o-round=nearest' if args.o_round == 'nearest' and args.scaling != 'none' else ''} path={path}")
    calib_kib = (args.calib_copy_mb << 20) / 1024.0

    def per_dispatch(fname, counter):
        vals = {}
        copies = {}
        for r in csv.DictReader(open(fname)):
            if r["Counter_Name"] != counter:
                continue
            d, v = r["Dispatch_Id"], float(r["Counter_Value"])
            if r["Kernel_Name"].split("(")[0].split("<")[0].endswith(kname):
                vals[d] = vals.get(d, 0.0) + v
            elif "copyBuffer" in r["Kernel_Name"]:
                copies[d] = copies.get(d, 0.0) + v
        if not vals or not copies:
            sys.exit(f"{fname}: no {counter} rows for {kname} or for the calibration copy")
        return statistics.median(vals.values()), max(copies.values()), len(vals)

    fetch, fcopy, nd = per_dispatch(args.record_traffic[0], "FETCH_SIZE")
    write, wcopy, _ = per_dispatch(args.record_traffic[1], "WRITE_SIZE")
    fs, wsc = calib_kib / fcopy, calib_kib / wcopy
    rec = {"kernel": kname, "source": ksource, "source_hash": kernel_source_hash(ksource), "fetch_kib": fetch,
           "write_kib": write, "fetch_scale": round(fs, 3), "write_scale": round(wsc, 3),
           "bytes_per_launch": int((fetch * fs + write * wsc) * 1024), "dispatches": nd}
    path_json = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path_json)) if os.path.exists(path_json) else {}
    old = data.get(workload, {})
    if "summary" in old:
        rec["summary"] = old["summary"]
    data[workload] = rec
    with open(path_json, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")
    print(json.dumps({workload: rec}))


def main():
    args = parse()
    if args.record_traffic:
        record_traffic(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built",
              file=sys.stderr)
        sys.exit(2)
    if args.batch > 0:
        batch_main(args)
        return
    if args.scaling_study:
        scaling_study(args)
        return
    import numpy as np
    import torch

    import paper_1507_00687_amd as F
    from synth import make_pair

    torch.cuda.set_device(0)
    n = args.n
    m = k = n
    dt_np = np.float64 if args.precision == "f64" else np.float32
    A, B = make_pair(args.dist, args.seed, m, k, n, dtype=dt_np)
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    plan = F.Plan(args.algo, args.depth, args.cutoff, scaling=args.scaling, steps=args.scaling_steps,
                  precision=args.precision, fuse=args.fuse, per_level=args.per_level, o_round=args.o_round)
    L, Mp, Kp, Np = plan.shape(m, k, n)
    path = plan.path(m, k, n)
    kname, ksource = product_kernel(args.precision, path)
    ws = torch.empty(max(plan.workspace_size(m, k, n), 1), dtype=torch.uint8, device="cuda")
    Cf = torch.empty((m, n), dtype=tA.dtype, device="cuda")
    run_fast = lambda: F.fastmm_gemm(plan, tA, tB, C=Cf, workspace=ws)

    classical = None
    if not args.no_classical:
        cplan = F.Plan("classical", 0, 1, scaling=args.scaling, steps=args.scaling_steps, precision=args.precision,
                       o_round=args.o_round)
        cws = torch.empty(max(cplan.workspace_size(m, k, n), 1), dtype=torch.uint8, device="cuda")
        Cc = torch.empty((m, n), dtype=tA.dtype, device="cuda")
        run_cls = lambda: F.fastmm_gemm(cplan, tA, tB, C=Cc, workspace=cws)
        ms_cls = time_steps(run_cls, args.steps, args.warmup)
        classical = {"ms_per_step": ms_cls, "value": 2.0 * m * k * n / (ms_cls * 1e-3) / 1e12}

    beside = None
    if args.beside and args.beside != "none" and args.beside != args.precision:
        bdt = torch.float64 if args.beside == "f64" else torch.float32
        bA, bB = (tA, tB) if bdt == tA.dtype else (tA.to(bdt), tB.to(bdt))
        bplan = F.Plan(args.algo, args.depth, args.cutoff, scaling=args.scaling, steps=args.scaling_steps,
                       precision=args.beside, fuse=args.fuse, per_level=args.per_level, o_round=args.o_round)
        bws = torch.empty(max(bplan.workspace_size(m, k, n), 1), dtype=torch.uint8, device="cuda")
        Cb = torch.empty((m, n), dtype=bdt, device="cuda")
        ms_b = time_steps(lambda: F.fastmm_gemm(bplan, bA, bB, C=Cb, workspace=bws), args.steps, args.warmup)
        beside = {"precision": args.beside, "path": bplan.path(m, k, n), "ms_per_step": ms_b,
                  "value": 2.0 * m * k * n / (ms_b * 1e-3) / 1e12}

    also, also_rows = None, None
    if args.also and args.also != "none" and args.also != args.algo:
        aplan = F.Plan(args.also, args.depth, args.cutoff, scaling=args.scaling, steps=args.scaling_steps,
                       precision=args.precision, fuse=args.fuse, per_level=args.per_level, o_round=args.o_round)
        aws = torch.empty(max(aplan.workspace_size(m, k, n), 1), dtype=torch.uint8, device="cuda")
        Ca = torch.empty((m, n), dtype=tA.dtype, device="cuda")
        run_also = lambda: F.fastmm_gemm(aplan, tA, tB, C=Ca, workspace=aws)
        ms_a = time_steps(run_also, args.steps, args.warmup)
        F.fastmm_profile_enable(True)
        F.fastmm_profile_read()
        for _ in range(args.steps):
            run_also()
        aprof = F.fastmm_profile_read()
        F.fastmm_profile_enable(False)
        acalls = max(aprof["calls"], 1)
        also = {"algo": args.also, "path": aplan.path(m, k, n), "levels_used": aplan.shape(m, k, n)[0],
                "ms_per_step": ms_a, "value": 2.0 * m * k * n / (ms_a * 1e-3) / 1e12,
                "phases_ms": {"scaling": aprof["scaling_ms"] / acalls, "form": aprof["form_ms"] / acalls,
                              "leaf": aprof["leaf_ms"] / acalls, "combine": aprof["combine_ms"] / acalls}}
        also_rows = Ca  # sampled after the reference rows are chosen
        del aws

    # timed region: K steps between device synchronisations (one GPU: no barrier needed)
    ms = time_steps(run_fast, args.steps, args.warmup)
    value = 2.0 * m * k * n / (ms * 1e-3) / 1e12

    # product-kernel duration from the library's HIP events (same stream as the launches)
    F.fastmm_profile_enable(True)
    F.fastmm_profile_read()
    for _ in range(args.steps):
        run_fast()
    prof = F.fastmm_profile_read()
    F.fastmm_profile_enable(False)
    calls = max(prof["calls"], 1)
    leaf_ms = prof["leaf_ms"] / calls
    info = F.fastmm_algo_info(args.algo)
    nleaves = info["R"] ** L if args.algo != "classical" else 1
    mb, kb, nb = Mp // info["M0"] ** L, Kp // info["K0"] ** L, Np // info["N0"] ** L
    flops_per_launch = 2.0 * mb * kb * nb * nleaves * PRODUCTS[args.precision]
    # one recorded call per step, or (scaling at every level) one per node product of the
    # first level, each with its own products launch
    flops_per_launch *= args.steps / calls
    achieved = flops_per_launch / (leaf_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    workload = (f"{args.algo} L={args.depth} cutoff={args.cutoff} n={n} {args.precision} {args.dist} "
                f"scaling={args.scaling}{' per-level' if args.per_level else ''}"
                f"{' o-round=nearest' if args.o_round == 'nearest' and args.scaling != 'none' else ''} path={path}")

    torch_ref = None
    if args.torch_ref:
        ms_t = time_steps(lambda: torch.matmul(tA, tB), args.steps, args.warmup)
        torch_ref = {"ms_per_step": ms_t, "value": 2.0 * m * k * n / (ms_t * 1e-3) / 1e12}
    vendor = None
    if not args.no_vendor and L > 0 and path != "every_level":
        vendor = vendor_leaf_gemm(args, nleaves, mb, kb, nb, achieved)
    if args.calib_copy_mb > 0:
        nbytes = args.calib_copy_mb << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # errors on sampled rows against the long-double reference (oracle leg)
    rows = np.unique(np.linspace(0, m - 1, args.err_rows).astype(np.int64))
    Cf_rows = Cf[torch.from_numpy(rows).cuda()].cpu().numpy()
    leg = cpu_baseline_leg(args, A, B, rows)
    ref = leg["ref"]
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    den = float(np.max(np.abs(A64))) * float(np.max(np.abs(B64)))
    err_fast = float(np.max(np.abs(Cf_rows.astype(np.longdouble) - ref))) / den
    err = {"fast": err_fast, "rows_sampled": int(len(rows)), "reference": "long double classical (oracle)"}
    if classical is not None:
        Cc_rows = Cc[torch.from_numpy(rows).cuda()].cpu().numpy()
        err["classical"] = float(np.max(np.abs(Cc_rows.astype(np.longdouble) - ref))) / den
    if beside is not None:
        Cb_rows = Cb[torch.from_numpy(rows).cuda()].cpu().numpy()
        beside["error"] = float(np.max(np.abs(Cb_rows.astype(np.longdouble) - ref))) / den
    if also is not None:
        Ca_rows = also_rows[torch.from_numpy(rows).cuda()].cpu().numpy()
        also["error"] = float(np.max(np.abs(Ca_rows.astype(np.longdouble) - ref))) / den
        if classical is not None:
            also["speedup_vs_classical"] = classical["ms_per_step"] / also["ms_per_step"]

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": workload, "algo": args.algo, "depth": args.depth, "levels_used": L,
                   "cutoff": args.cutoff, "m": m, "k": k, "n": n, "padded": [Mp, Kp, Np],
                   "precision": args.precision, "scaling": args.scaling, "o_round": args.o_round, "dist": args.dist,
                   "path": path},
        "classical": classical,
        "beside": beside,
        "also": also,
        "torch_matmul": torch_ref,
        "vendor_leaf_gemm": vendor,
        "speedup_vs_classical": (classical["ms_per_step"] / ms) if classical else None,
        "error": err,
        "phases_ms": {"scaling": prof["scaling_ms"] / calls, "form": prof["form_ms"] / calls, "leaf": leaf_ms,
                      "combine": prof["combine_ms"] / calls},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": load_traffic(workload, ksource),
                     "kernel": kname, "flops_per_launch": flops_per_launch},
        "cpu_baseline": leg.get("cpu"),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
