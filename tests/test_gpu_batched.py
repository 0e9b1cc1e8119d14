"""GPU tests of the batched persistent launch and of the autotuner."""
import numpy as np
import pytest

from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import np_dtype

pytestmark = pytest.mark.gpu

# (rule, depth, (m, k, n)): mixed rules, depths, ragged and tall-skinny shapes
BATCH = [
    ("classical", 0, (130, 70, 90)),
    ("strassen", 1, (256, 128, 512)),
    ("f323", 2, (198, 96, 180)),
    ("winograd", 2, (64, 512, 64)),
    ("f424", 1, (512, 64, 128)),
    ("laderman333", 1, (99, 99, 99)),
    ("strassen", 2, (17, 300, 41)),
    ("f332", 1, (300, 33, 260)),
]


def _run_batch(precision, dist, scaling="none"):
    import torch

    import paper_1507_00687_amd as F

    dt = np_dtype(precision)
    # the batched launch has no fused kernel: FP64 / FP32 problems take written leaf operands
    # where they apply, else the composite lists, as single launches in fusion mode "written"
    # do; compare with those (fused single launches round differently from depth 2 on)
    plans, leaf_plans, As, Bs, hostA, hostB = [], [], [], [], [], []
    for i, (name, depth, (m, k, n)) in enumerate(BATCH):
        A, B = make_pair(dist, 100 + i, m, k, n, dtype=dt)
        hostA.append(A)
        hostB.append(B)
        plans.append(F.Plan(name, depth, 1, precision=precision, scaling=scaling))
        leaf_plans.append(F.Plan(name, depth, 1, precision=precision, scaling=scaling, fuse="written"))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
    Cs = F.fastmm_gemm_batched(plans, As, Bs)
    singles = [F.fastmm_gemm(p, a, b) for p, a, b in zip(leaf_plans, As, Bs)]
    torch.cuda.synchronize()
    return hostA, hostB, [c.cpu().numpy() for c in Cs], [c.cpu().numpy() for c in singles]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batched_integer_exact_and_equal_to_single_launches(precision):
    A, B, Cb, Cs = _run_batch(precision, "int8")
    for a, b, cb, cs in zip(A, B, Cb, Cs):
        exact = (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64)
        assert np.array_equal(cb.astype(np.float64), exact)
        assert np.array_equal(cb, cs)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("scaling", ["none", "repeated"])
def test_batched_float_bitwise_equal_to_single_launches(precision, scaling):
    # every tile is computed by the same code in the same order as in a single launch
    A, B, Cb, Cs = _run_batch(precision, "normal", scaling)
    for a, b, cb, cs in zip(A, B, Cb, Cs):
        assert np.array_equal(cb, cs)
        ref = O.reference_rows(a.astype(np.float64), b.astype(np.float64))
        assert O.normwise_error(cb, ref, a, b) <= (1e-13 if precision == "f64" else 5e-5)


@pytest.mark.parametrize("precision", ["bf16x3", "f16x3"])
def test_batched_split_precision_exact_and_equal_to_single_launches(precision):
    # one limb-GEMM launch for the whole batch (tiles shared by all problems); the limb
    # products of every output element run in the same order as in single launches
    A, B, Cb, Cs = _run_batch(precision, "int8")
    for a, b, cb, cs in zip(A, B, Cb, Cs):
        exact = (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64)
        assert np.array_equal(cb.astype(np.float64), exact)
    A, B, Cb, Cs = _run_batch(precision, "normal")
    for a, b, cb, cs in zip(A, B, Cb, Cs):
        assert np.array_equal(cb, cs)


@pytest.mark.parametrize("precision", ["f32", "f64", "f16x3"])
def test_batched_mixed_scaling_and_output_modes(precision):
    # plans with and without outside scaling, classical (written straight to C) and fast
    # (leaf workspace, then the W-combination) in one batch: every mode's group of work items
    import torch

    import paper_1507_00687_amd as F

    dt = np_dtype(precision) if precision != "f16x3" else np.float32
    specs = [("classical", 0, "none", (130, 70, 90)), ("strassen", 1, "outside", (256, 128, 160)),
             ("classical", 0, "outside", (96, 200, 64)), ("winograd", 2, "none", (150, 260, 170)),
             ("f424", 1, "outside", (160, 96, 200)), ("strassen", 2, "none", (70, 300, 90))]
    plans, As, Bs, hostA, hostB = [], [], [], [], []
    for i, (name, depth, scaling, (m, k, n)) in enumerate(specs):
        A, B = make_pair("int8", 200 + i, m, k, n, dtype=dt)
        hostA.append(A)
        hostB.append(B)
        plans.append(F.Plan(name, depth, 1, precision=precision, scaling=scaling))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
    Cs = F.fastmm_gemm_batched(plans, As, Bs)
    torch.cuda.synchronize()
    for a, b, c in zip(hostA, hostB, Cs):
        exact = (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64)
        assert np.array_equal(c.cpu().numpy().astype(np.float64), exact)


def test_batched_repeat_is_deterministic():
    _, _, C1, _ = _run_batch("f32", "normal")
    _, _, C2, _ = _run_batch("f32", "normal")
    for a, b in zip(C1, C2):
        assert np.array_equal(a, b)


def test_batched_rejects_mixed_precision_and_aliasing():
    import torch

    import paper_1507_00687_amd as F

    a = torch.ones((32, 32), dtype=torch.float64, device="cuda")
    b = torch.ones((32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(F.FastmmError):
        F.fastmm_gemm_batched([F.Plan("strassen", 1, precision="f64"), F.Plan("strassen", 1, precision="f32")],
                              [a, b], [a, b])
    with pytest.raises(F.FastmmError):  # output aliases an input of another problem
        F.fastmm_gemm_batched([F.Plan("strassen", 1, precision="f64")] * 2, [a, a.clone()], [a.clone(), a.clone()],
                              Cs=[torch.empty_like(a), a])


def test_autotune_picks_a_valid_plan_and_caches(tmp_path):
    import torch

    import paper_1507_00687_amd as F
    from paper_1507_00687_amd import tune

    cache = str(tmp_path / "tune.json")
    shapes = [(256, 256, 256), (512, 128, 512)]
    res = tune.tune(shapes, precision="f32", cache=cache, max_depth=2, reps=2)
    assert set(res) == set(shapes)
    for (m, k, n), ch in res.items():
        A, B = make_pair("int8", 3, m, k, n, dtype=np.float32)
        C = F.fastmm_gemm(ch.plan("f32"), torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()).cpu().numpy()
        assert np.array_equal(C.astype(np.float64), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))
    again = tune.tune(shapes, precision="f32", cache=cache, max_depth=2, reps=2)
    assert {s: (c.algo, c.depth) for s, c in again.items()} == {s: (c.algo, c.depth) for s, c in res.items()}
    # a stability cap of 1 admits only the classical kernel
    capped = tune.tune([(256, 256, 256)], precision="f32", max_instability=1.0, max_depth=1, reps=1)
    assert capped[(256, 256, 256)].algo == "classical"


def test_autotune_with_per_level_rules():
    # Non-stationary candidates (a rule per level) join the search; the winner runs correctly.
    import torch

    import paper_1507_00687_amd as F
    from paper_1507_00687_amd import tune

    shape = (512, 256, 1024)
    res = tune.tune([shape], precision="f32", max_depth=2, reps=1, non_stationary=True)
    ch = res[shape]
    plan = ch.plan("f32")
    A, B = make_pair("int8", 90, *shape, dtype=np.float32)
    C = F.fastmm_gemm(plan, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()).cpu().numpy()
    assert np.array_equal(C.astype(np.float64), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))
    assert ch.levels is None or len(ch.levels) == ch.depth
    print(f"\n  chose {ch}", flush=True)


def test_output_tile_forced_and_tuned_split_precision(tmp_path):
    # the limb GEMM's 128 and 256 tiles give the same exact products, alone and in a batch with
    # mixed tile settings (the batch runs the smallest); the tuner returns a usable tile choice
    import torch

    import paper_1507_00687_amd as F
    from paper_1507_00687_amd import tune

    shape = (600, 520, 700)
    print(f"\n[tile] {shape} f16x3", flush=True)
    A, B = make_pair("int8", 5, *shape, dtype=np.float32)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    outs = []
    for tile in (0, 128, 256):
        p = F.Plan("strassen", 1, 1, precision="f16x3").set_tile(tile)
        outs.append(F.fastmm_gemm(p, tA, tB).cpu().numpy())
        assert np.array_equal(outs[-1].astype(np.float64), exact)
    plans = [F.Plan("strassen", 1, 1, precision="f16x3").set_tile(t) for t in (256, 128, 0)]
    Cs = F.fastmm_gemm_batched(plans, [tA] * 3, [tB] * 3)
    torch.cuda.synchronize()
    for c in Cs:
        assert np.array_equal(c.cpu().numpy().astype(np.float64), exact)
    res = tune.tune([shape], precision="f16x3", cache=str(tmp_path / "t.json"), max_depth=1, reps=1,
                    in_batch=False)
    ch = res[shape]
    assert ch.tile in (0, 128, 256)
    got = F.fastmm_gemm(ch.plan("f16x3"), tA, tB).cpu().numpy()
    assert np.array_equal(got.astype(np.float64), exact)
