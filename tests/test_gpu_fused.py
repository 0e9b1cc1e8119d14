"""GPU tests of the fused one-level path for <2,2,2;7> rules (S/T formation, the seven
products and the W-sums of eq. (1) in one launch): exact on integers, equal to the leaf path
where both round identically, and within the error bounds of section 4 otherwise."""
import numpy as np
import pytest

from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import UNIT_ROUNDOFF, np_dtype, oracle_fast, run_gpu, theorem_bound

pytestmark = pytest.mark.gpu

# (depth, (m, k, n)): several tiles and ragged tails at every level; odd sizes reach the
# padded (virtual zero) rows and columns; (1, 64, 64) has one-row sub-blocks.
SHAPES = [
    (1, (256, 256, 256)),
    (1, (300, 200, 260)),
    (1, (1, 64, 64)),
    (1, (129, 33, 257)),
    (2, (17, 300, 41)),
    (2, (520, 136, 392)),
    (3, (1000, 520, 776)),
]


def _plan(name, depth, precision, fuse="always", scaling="none", cutoff=1):
    import paper_1507_00687_amd as F

    return F.Plan(name, depth, cutoff, precision=precision, scaling=scaling, fuse=fuse)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", ["strassen", "winograd"])
@pytest.mark.parametrize("depth,shape", SHAPES)
def test_fused_integer_inputs_bit_exact(precision, name, depth, shape):
    m, k, n = shape
    print(f"\n[fused-int] {name} L={depth} {precision} {shape}", flush=True)
    plan = _plan(name, depth, precision)
    assert plan.path(m, k, n) == "fused"
    A, B = make_pair("int8", 7, m, k, n, dtype=np_dtype(precision))
    Cg = run_gpu(plan, A, B)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(Cg.astype(np.float64), exact)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", ["strassen", "winograd"])
@pytest.mark.parametrize("scaling", ["none", "outside", "repeated"])
@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 200, 260)])
def test_fused_equals_leaf_path_at_depth_one(precision, name, scaling, shape):
    # At one level both paths form each S_r, T_r element with the same operations in the same
    # order, run the same MFMA sequence over k (the same k-interleave in every 16-k chunk) and
    # sum the W terms in ascending r: the results are bitwise equal.
    m, k, n = shape
    print(f"\n[fused=leaf] {name} {precision} {scaling} {shape}", flush=True)
    dist = "badly_scaled" if scaling != "none" else "normal"
    A, B = make_pair(dist, 11, m, k, n, dtype=np_dtype(precision))
    Cf = run_gpu(_plan(name, 1, precision, "always", scaling), A, B)
    Cl = run_gpu(_plan(name, 1, precision, "off", scaling), A, B)
    assert np.array_equal(Cf, Cl)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", ["strassen", "winograd"])
@pytest.mark.parametrize("depth,shape", [(2, (520, 136, 392)), (3, (1000, 520, 776)), (1, (300, 200, 260))])
def test_fused_float_error_against_oracle(precision, name, depth, shape):
    m, k, n = shape
    print(f"\n[fused-float] {name} L={depth} {precision} {shape}", flush=True)
    A, B = make_pair("normal", 5, m, k, n, dtype=np_dtype(precision))
    Cg = run_gpu(_plan(name, depth, precision), A, B)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = O.reference_rows(A64, B64)
    err = O.normwise_error(Cg, ref, A64, B64)
    u = UNIT_ROUNDOFF[precision]
    assert err <= theorem_bound(name, m, k, n, depth, 1, u)
    assert err <= (1e-13 if precision == "f64" else 5e-5)
    if precision == "f64":  # same order of error as the oracle's fast product (FP64 too)
        err_o = O.normwise_error(oracle_fast(name, A64, B64, depth, 1), ref, A64, B64)
        assert err <= 4 * err_o + 16 * u


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_strided_and_unaligned_operands(precision):
    # Row strides larger than the row and base pointers off 16-byte alignment take the
    # element-wise load path; results stay exact on integers.
    import torch

    import paper_1507_00687_amd as F

    m, k, n = 200, 150, 180
    A, B = make_pair("int8", 13, m, k, n, dtype=np_dtype(precision))
    bigA = np.zeros((m, k + 9), dtype=A.dtype)
    bigA[:, 1:k + 1] = A
    bigB = np.zeros((k, n + 5), dtype=B.dtype)
    bigB[:, 3:n + 3] = B
    plan = _plan("strassen", 2, precision)
    tA = torch.from_numpy(bigA).cuda()[:, 1:k + 1]
    tB = torch.from_numpy(bigB).cuda()[:, 3:n + 3]
    Cg = F.fastmm_gemm_ex(plan, tA, False, tB, False).cpu().numpy()
    assert np.array_equal(Cg.astype(np.float64), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


def test_fused_repeat_is_deterministic():
    A, B = make_pair("normal", 2, 384, 320, 352, dtype=np.float32)
    plan = _plan("winograd", 2, "f32")
    C1 = run_gpu(plan, A, B)
    C2 = run_gpu(plan, A, B)
    assert np.array_equal(C1, C2)


@pytest.mark.parametrize("name", ["strassen", "winograd"])
def test_fused_gradients_integer_exact(name):
    # The backward pass runs the transposes of the rotated rules (compiled patterns of the
    # fused kernel), the transposed operand copied row-major first, so it takes the fused path
    # too.
    import torch

    import paper_1507_00687_amd as F
    from synth.gen import TAG_G, int_uniform

    m, k, n = 160, 96, 224
    A, B = make_pair("int8", 4, m, k, n, dtype=np.float32)
    G = int_uniform(4, TAG_G, (m, n)).astype(np.float32)
    plan = _plan(name, 2, "f32")
    tA = torch.from_numpy(A).cuda().requires_grad_(True)
    tB = torch.from_numpy(B).cuda().requires_grad_(True)
    F.fast_matmul(tA, tB, plan).backward(torch.from_numpy(G).cuda())
    i64 = lambda X: X.astype(np.int64)
    assert np.array_equal(tA.grad.cpu().numpy().astype(np.float64), (i64(G) @ i64(B).T).astype(np.float64))
    assert np.array_equal(tB.grad.cpu().numpy().astype(np.float64), (i64(A).T @ i64(G)).astype(np.float64))
