"""Autotuner: choose a plan (rule, depth, cutoff and, for the split precisions, the limb GEMM's
output tile) per problem shape by measuring on the GPU.

Candidates are the built-in rules at depths 0..3 (depth 0 is the classical kernel).  A
candidate is admitted only if its growth factor relative to classical -- the E^L term of
Theorem 4.1 over the classical K0^L -- stays within `max_instability` (the relative
instability (E/K0^2)^L of section 5.3 is the same quantity up to the inner dimension); the
fastest admitted candidate wins; for a split precision timed alone, the winner is then timed
with the other output tile (128 x 128 against 256 x 256) and keeps the faster (a batched
launch runs all its problems on one tile, so batch tuning leaves the tile to the library).  Results are cached in a JSON file keyed by shape and
precision, so tuning can resume.  The timing itself runs the product through libfastmm.so.

By default a candidate is timed the way a batch runs it: as one fastmm_gemm_batched call over
enough copies of the shape to give the GPU several hundred output tiles, the time divided by
the copies.  (Timed alone, a small classical product leaves most compute units idle and the
extra leaves of a fast rule look like a gain that a full batch does not see.)
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass
from typing import Dict, Iterable, List, Optional, Tuple

RULES = ("strassen", "winograd", "f323", "f332", "f233", "f424", "f442", "f244", "laderman333")
SPLIT = ("bf16", "f16", "bf16x3", "f16x3", "bf16x6")
LIMBS = {"bf16": 1, "f16": 1, "bf16x3": 2, "f16x3": 2, "bf16x6": 3}


@dataclass
class Choice:
    algo: str
    depth: int
    cutoff: int
    ms: float
    instability: float  # product over the levels used of E / K0^2 (1 for classical)
    levels: Optional[List[str]] = None  # a rule per level (uniform non-stationary), else None
    tile: int = 0  # split precisions: limb-GEMM output tile (0: by the leaf-block shape)

    def plan(self, precision: str, **kw):
        from .fastmm import Plan

        p = Plan(self.algo, self.depth, self.cutoff, precision=precision, **kw)
        if self.levels:
            p.set_levels(self.levels)
        if self.tile:
            p.set_tile(self.tile)
        return p


def relative_instability(algo: str, levels: int) -> float:
    """(E / K0^2)^L: the factor by which the leading term of Theorem 4.1 exceeds classical's."""
    from .fastmm import fastmm_algo_stability

    if algo == "classical" or levels == 0:
        return 1.0
    return fastmm_algo_stability(algo, levels)["rel_instability"]


def candidates(max_depth: int = 3, cutoffs: Iterable[int] = (128, 256, 512), non_stationary: bool = False):
    """(rule, depth, cutoff, levels) tuples: classical, every rule stationary at depths
    1..max_depth and, with non_stationary, every ordered pair of distinct rules as two levels
    (section 3.3; shapes far from square are where mixed base cases pay)."""
    out = [("classical", 0, 1, None)]
    for a in RULES:
        for d in range(1, max_depth + 1):
            for c in cutoffs:
                out.append((a, d, c, None))
    if non_stationary and max_depth >= 2:
        for a in RULES:
            for b in RULES:
                if a != b:
                    for c in cutoffs:
                        out.append((a, 2, c, [a, b]))
    return out


def _time_plan(plan, A, B, C, ws, reps: int) -> float:
    import torch

    from .fastmm import fastmm_gemm

    fastmm_gemm(plan, A, B, C=C, workspace=ws)  # warm-up (uploads the task table)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        start.record()
        fastmm_gemm(plan, A, B, C=C, workspace=ws)
        stop.record()
        stop.synchronize()
        times.append(start.elapsed_time(stop))
    times.sort()
    return times[len(times) // 2]


def _time_plan_batched(plan, A, B, Cs, reps: int) -> float:
    """Milliseconds per problem of one batched call over len(Cs) copies of (A, B)."""
    import torch

    from .fastmm import fastmm_batched_workspace_size, fastmm_gemm_batched

    c = len(Cs)
    plans, As, Bs = [plan] * c, [A] * c, [B] * c
    ws = torch.empty(max(fastmm_batched_workspace_size(plans, As, Bs), 1), dtype=torch.uint8, device="cuda")
    fastmm_gemm_batched(plans, As, Bs, Cs, workspace=ws)  # warm-up (uploads the task table)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        start.record()
        fastmm_gemm_batched(plans, As, Bs, Cs, workspace=ws)
        stop.record()
        stop.synchronize()
        times.append(start.elapsed_time(stop))
    times.sort()
    return times[len(times) // 2] / c


def batch_copies(m: int, n: int, target_tiles: int = 512, max_copies: int = 32) -> int:
    """Copies of an m x n output that give about target_tiles output tiles of 256 x 256."""
    tiles = -(-m // 256) * -(-n // 256)
    return max(1, min(max_copies, -(-target_tiles // tiles)))


def _key(m, k, n, precision, in_batch=True):
    return f"{m}x{k}x{n}:{precision}" + (":batch" if in_batch else "")


def tune_shape(m: int, k: int, n: int, precision: str = "f32", max_depth: int = 3, cutoffs=(128, 256, 512),
               max_instability: float = float("inf"), reps: int = 3, A=None, B=None, in_batch: bool = True,
               non_stationary: bool = False) -> Choice:
    """Measure every admitted candidate on (m, k, n) and return the fastest (timed inside a
    batch of copies when in_batch, else alone)."""
    import torch

    from .fastmm import Plan

    dt = torch.float64 if precision == "f64" else torch.float32
    gen = torch.Generator(device="cuda").manual_seed(1234)
    if A is None:
        A = torch.randn((m, k), dtype=dt, device="cuda", generator=gen)
    if B is None:
        B = torch.randn((k, n), dtype=dt, device="cuda", generator=gen)
    C = torch.empty((m, n), dtype=dt, device="cuda")
    Cs = [torch.empty((m, n), dtype=dt, device="cuda") for _ in range(batch_copies(m, n))] if in_batch else None
    best: Optional[Choice] = None
    seen = set()
    for algo, depth, cutoff, lv in candidates(max_depth, cutoffs, non_stationary):
        plan = Plan(algo, depth, cutoff, precision=precision)
        if lv:
            plan.set_levels(lv)
        levels = plan.shape(m, k, n)[0]
        key = (tuple(lv[:levels]) if lv else (algo,) * levels)
        if key in seen or (levels == 0 and algo != "classical"):
            continue  # same computation as a candidate already measured
        seen.add(key)
        inst = 1.0
        for r in key:
            inst *= relative_instability(r, 1)
        if inst > max_instability:
            continue
        if in_batch:
            ms = _time_plan_batched(plan, A, B, Cs, reps)
        else:
            ws = torch.empty(max(plan.workspace_size(m, k, n), 1), dtype=torch.uint8, device="cuda")
            ms = _time_plan(plan, A, B, C, ws, reps)
        if best is None or ms < best.ms:
            best = Choice(algo, depth if levels else 0, cutoff, ms, inst, list(lv[:levels]) if (lv and levels) else None)
    assert best is not None
    if precision in SPLIT and LIMBS[precision] <= 2 and not in_batch:
        # the winner with the other output tile (the library picks one by the leaf-block shape);
        # not for batches: a batched launch runs all its problems on one tile (the smallest of
        # their plans'), so a per-shape tile would set it for the whole batch
        for tile in (128, 256):
            cand = Choice(best.algo, best.depth, best.cutoff, 0.0, best.instability, best.levels, tile)
            plan = cand.plan(precision)
            ws = torch.empty(max(plan.workspace_size(m, k, n), 1), dtype=torch.uint8, device="cuda")
            ms = _time_plan(plan, A, B, C, ws, reps)
            if ms < best.ms * 0.98:  # a clear gain only: both tiles compute the same products
                cand.ms = ms
                best = cand
    return best


def tune(shapes: Iterable[Tuple[int, int, int]], precision: str = "f32", cache: Optional[str] = None,
         **kw) -> Dict[Tuple[int, int, int], Choice]:
    """Tune every distinct shape (cached results are reused and new ones appended)."""
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
    out = {}
    for (m, k, n) in dict.fromkeys(tuple(s) for s in shapes):
        key = _key(m, k, n, precision, kw.get("in_batch", True))
        if key in store:
            out[(m, k, n)] = Choice(**store[key])
            continue
        ch = tune_shape(m, k, n, precision, **kw)
        out[(m, k, n)] = ch
        store[key] = asdict(ch)
        if cache:
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(store, f, indent=1)
            os.replace(tmp, cache)
    return out
