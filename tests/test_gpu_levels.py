"""GPU tests of uniform non-stationary recursion (section 3.3, Theorem 4.2): a rule per level,
with different base shapes, on the written path (FP64, FP32: each level's node operands formed
with that level's rule), the composite-list leaf path (fusion off) and the split-precision path,
single, batched and through the backward pass (every level's rule rotated), against the
oracle's level-by-level recursion and Theorem 4.2."""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import np_dtype, run_gpu

pytestmark = pytest.mark.gpu

LEVELS = {"323-222": ["f323", "strassen"], "222-424": ["strassen", "f424"],
          "332-233-323": ["f332", "f233", "f323"]}


def _plan(F, key, precision, cutoff=1):
    lv = LEVELS[key]
    return F.Plan(lv[0], len(lv), cutoff, precision=precision).set_levels(lv)


def _exact(A, B):
    return (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3"])
@pytest.mark.parametrize("key,shape", [("323-222", (200, 130, 190)), ("222-424", (260, 100, 240)),
                                       ("332-233-323", (150, 120, 170))])
def test_levels_integer_exact(precision, key, shape):
    import paper_1507_00687_amd as F

    print(f"\n[levels-int] {key} {shape} {precision}", flush=True)
    A, B = make_pair("int8", 61, *shape, dtype=np.float64 if precision == "f64" else np.float32)
    got = run_gpu(_plan(F, key, precision), A, B)
    assert np.array_equal(got.astype(np.float64), _exact(A, B))


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("key", sorted(LEVELS))
def test_levels_float_against_oracle_and_theorem_4_2(precision, key):
    import paper_1507_00687_amd as F

    shape = (216, 180, 216)
    print(f"\n[levels-float] {key} {shape} {precision}", flush=True)
    rules = [C.get(a) for a in LEVELS[key]]
    dims = [(a.M0, a.K0, a.N0) for a in rules]
    A, B = make_pair("normal", 62, *shape, dtype=np_dtype(precision))
    got = run_gpu(_plan(F, key, precision), A, B)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = O.reference_rows(A64, B64)
    err = O.normwise_error(got, ref, A64, B64)
    err_oracle = O.normwise_error(O.fast_tree(A, B, lambda path: rules[len(path)], dims), ref, A64, B64)
    u = 2.0 ** -53 if precision == "f64" else 2.0 ** -24
    Kp = O.padded_dims(*shape, dims)[1]
    bound = O.thm42_bound(Kp, rules, u)
    print(f"  error {err:.3e}, oracle's own {err_oracle:.3e}, Theorem 4.2 {bound:.3e}", flush=True)
    assert err <= 4 * err_oracle + 8 * u
    assert err <= bound


def test_levels_batched_and_backward():
    import torch

    import paper_1507_00687_amd as F

    plans = [_plan(F, "323-222", "f64"), F.Plan("strassen", 2, 1, precision="f64"), _plan(F, "222-424", "f64")]
    shapes = [(90, 70, 110), (64, 128, 32), (120, 80, 100)]
    host = [make_pair("int8", 70 + i, *s) for i, s in enumerate(shapes)]
    As = [torch.from_numpy(a).cuda() for a, _ in host]
    Bs = [torch.from_numpy(b).cuda() for _, b in host]
    Cs = F.fastmm_gemm_batched(plans, As, Bs)
    torch.cuda.synchronize()
    for (a, b), c in zip(host, Cs):
        assert np.array_equal(c.cpu().numpy(), _exact(a, b))
    # backward through the rotated level rules: dA = G B^T, dB = A^T G, exact on integers
    for key in ("323-222", "332-233-323"):
        p = _plan(F, key, "f64")
        A, B = make_pair("int8", 80, 100, 90, 110)
        G = make_pair("int8", 81, 100, 110, 1)[0]
        tA, tB, tG = (torch.from_numpy(x).cuda() for x in (A, B, G))
        dA, dB = F.fastmm_gemm_backward(p, tA, tB, tG)
        torch.cuda.synchronize()
        assert np.array_equal(dA.cpu().numpy(), _exact(G, B.T))
        assert np.array_equal(dB.cpu().numpy(), _exact(A.T, G))


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("key,shape", [("323-222", (200, 130, 190)), ("222-424", (260, 100, 240)),
                                       ("332-233-323", (150, 120, 170))])
def test_levels_written_path_equals_leaf_path_on_integers(precision, key, shape):
    """Per-level rules take the written path by default (each level's node operands formed with
    its own U, V); on integers it is exact, like the composite-list leaf path."""
    import paper_1507_00687_amd as F

    print(f"\n[levels-written] {key} {shape} {precision}", flush=True)
    lv = LEVELS[key]
    written = _plan(F, key, precision)
    listed = F.Plan(lv[0], len(lv), 1, precision=precision, fuse="off").set_levels(lv)
    assert written.path(*shape) == "written" and listed.path(*shape) == "leaf"
    A, B = make_pair("int8", 63, *shape, dtype=np_dtype(precision))
    exact = _exact(A, B)
    assert np.array_equal(run_gpu(written, A, B).astype(np.float64), exact)
    assert np.array_equal(run_gpu(listed, A, B).astype(np.float64), exact)
