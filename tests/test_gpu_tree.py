"""GPU tests of non-uniform recursion (section 3.4): the trees of the two non-uniform examples of section 5.2
(Examples 4.2 and 4.3 here) on the written path (FP64, FP32: each parent node's operands
formed with its own rule), the composite-list leaf path (fusion off) and the split-precision
path, single and batched, against the oracle's per-node recursion."""
import numpy as np
import pytest

from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import np_dtype, run_gpu
from tests.trees import dalberto_tree, f323_tree

pytestmark = pytest.mark.gpu

TREES = {"dalberto": (dalberto_tree, "strassen", (2, 2, 2)), "f323": (f323_tree, "f323", (3, 2, 3))}


def _tree_plan(F, tree, precision, cutoff=1):
    build, base, dims = TREES[tree]
    ids, rule = build(F)
    return F.Plan(base, 2, cutoff, precision=precision).set_tree(ids), rule, dims


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3"])
@pytest.mark.parametrize("tree,shape", [("dalberto", (256, 256, 256)), ("dalberto", (130, 70, 190)),
                                        ("f323", (200, 150, 220))])
def test_tree_integer_exact(precision, tree, shape):
    import paper_1507_00687_amd as F

    print(f"\n[tree-int] {tree} {shape} {precision}", flush=True)
    plan, _, _ = _tree_plan(F, tree, precision)
    A, B = make_pair("int8", 41, *shape, dtype=np.float64 if precision == "f64" else np.float32)
    got = run_gpu(plan, A, B)
    assert np.array_equal(got.astype(np.float64), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("tree", ["dalberto", "f323"])
def test_tree_float_against_oracle_tree(precision, tree):
    import paper_1507_00687_amd as F

    shape = (288, 200, 288)
    print(f"\n[tree-float] {tree} {shape} {precision}", flush=True)
    plan, rule, dims = _tree_plan(F, tree, precision)
    A, B = make_pair("normal", 42, *shape, dtype=np_dtype(precision))
    got = run_gpu(plan, A, B)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = O.reference_rows(A64, B64)
    err = O.normwise_error(got, ref, A64, B64)
    err_oracle = O.normwise_error(O.fast_tree(A, B, rule, [dims, dims]), ref, A64, B64)
    u = 2.0 ** -53 if precision == "f64" else 2.0 ** -24
    print(f"  error {err:.3e}, oracle's own {err_oracle:.3e}", flush=True)
    assert err <= 4 * err_oracle + 8 * u
    assert err <= (1e-13 if precision == "f64" else 5e-5)


def test_tree_in_a_batch_and_backward():
    import torch

    import paper_1507_00687_amd as F

    tplan, _, _ = _tree_plan(F, "dalberto", "f32")
    uplan = F.Plan("strassen", 2, 1, precision="f32")
    shapes = [(256, 128, 192), (100, 300, 60), (64, 64, 64)]
    plans = [tplan, uplan, tplan]
    host = [make_pair("int8", 50 + i, *s, dtype=np.float32) for i, s in enumerate(shapes)]
    As = [torch.from_numpy(a).cuda() for a, _ in host]
    Bs = [torch.from_numpy(b).cuda() for _, b in host]
    Cs = F.fastmm_gemm_batched(plans, As, Bs)
    torch.cuda.synchronize()
    for (a, b), c in zip(host, Cs):
        assert np.array_equal(c.cpu().numpy().astype(np.float64), (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64))
    # backward: every node's rule transposed and rotated alike (section 3.1), exact on integers,
    # single and batched
    from synth.gen import TAG_G, int_uniform

    i64 = lambda X: X.astype(np.int64)
    Gs = [int_uniform(60 + i, TAG_G, (s[0], s[2])).astype(np.float32) for i, s in enumerate(shapes)]
    tGs = [torch.from_numpy(g).cuda() for g in Gs]
    dA, dB = F.fastmm_gemm_backward(tplan, As[0], Bs[0], tGs[0])
    batched = F.fastmm_gemm_backward_batched(plans, As, Bs, tGs)
    torch.cuda.synchronize()
    a, b = host[0]
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), (i64(Gs[0]) @ i64(b).T).astype(np.float64))
    assert np.array_equal(dB.cpu().numpy().astype(np.float64), (i64(a).T @ i64(Gs[0])).astype(np.float64))
    for (a, b), g, (ga, gb) in zip(host, Gs, batched):
        assert np.array_equal(ga.cpu().numpy().astype(np.float64), (i64(g) @ i64(b).T).astype(np.float64))
        assert np.array_equal(gb.cpu().numpy().astype(np.float64), (i64(a).T @ i64(g)).astype(np.float64))


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("tree,shape", [("dalberto", (130, 70, 190)), ("f323", (200, 150, 220))])
def test_tree_written_and_list_paths_exact(precision, tree, shape):
    """Tree plans write their leaf operands by default, each parent node's children formed with
    that node's rule; on integers both that path and the composite-list path are exact."""
    import paper_1507_00687_amd as F

    print(f"\n[tree-written] {tree} {shape} {precision}", flush=True)
    build, base, _ = TREES[tree]
    ids, _ = build(F)
    written = F.Plan(base, 2, 1, precision=precision).set_tree(ids)
    listed = F.Plan(base, 2, 1, precision=precision, fuse="off").set_tree(ids)
    assert written.path(*shape) == "written" and listed.path(*shape) == "leaf"
    A, B = make_pair("int8", 42, *shape, dtype=np_dtype(precision))
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(run_gpu(written, A, B).astype(np.float64), exact)
    assert np.array_equal(run_gpu(listed, A, B).astype(np.float64), exact)
