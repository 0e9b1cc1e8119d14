"""The FP64 / FP32 path with written-out leaf operands (from depth 1, every plan with one rule
that the FP32 fused kernel does not take): every S_r and T_r formed level by level by eq. (2),
the first level scaled, then one launch over the written-out leaves and the W-combination of
the composite destination lists.

Integer inputs must be bit-exact (every partial sum is an integer well inside the mantissa);
floating-point results within Theorem 4.1 and within 4x the oracle's own error for the same
rule and depth (the S/T sums follow the oracle's level-by-level order; the leaf products and
the W-sums are summed in other orders)."""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import UNIT_ROUNDOFF, np_dtype, oracle_fast, run_gpu, theorem_bound

pytestmark = pytest.mark.gpu

CASES = [  # rule, depth, shape (ragged: padding on every side)
    ("f424", 2, (200, 40, 180)),
    ("f424", 2, (256, 128, 256)),
    ("f442", 2, (150, 100, 60)),
    ("f244", 2, (70, 180, 150)),
    ("f323", 2, (200, 150, 220)),
    ("laderman333", 2, (135, 100, 81)),
    ("f424", 3, (260, 70, 300)),
    ("f424", 1, (200, 40, 180)),
    ("laderman333", 1, (100, 81, 135)),
]
CASES_F64 = [("strassen", 1, (300, 200, 100)), ("strassen", 2, (257, 300, 129)), ("winograd", 3, (200, 264, 300))]


def _plan(name, depth, precision, scaling="none", steps=2):
    import paper_1507_00687_amd as F

    return F.Plan(name, depth, 1, scaling=scaling, steps=steps, precision=precision)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,depth,shape", CASES)
def test_written_integer_exact(precision, name, depth, shape):
    print(f"\n[written-int] {name} L={depth} {shape} {precision}", flush=True)
    p = _plan(name, depth, precision)
    assert p.path(*shape) == "written"
    A, B = make_pair("int8", 50, *shape, dtype=np_dtype(precision))
    got = run_gpu(p, A, B)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(got.astype(np.float64), exact)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,depth,shape", CASES[:6])
def test_written_float_against_oracle(precision, name, depth, shape):
    print(f"\n[written-float] {name} L={depth} {shape} {precision}", flush=True)
    A, B = make_pair("normal", 51, *shape, dtype=np_dtype(precision))
    got = run_gpu(_plan(name, depth, precision), A, B)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = O.reference_rows(A64, B64)
    err = O.normwise_error(got, ref, A64, B64)
    u = UNIT_ROUNDOFF[precision]
    assert err <= theorem_bound(name, *shape, depth, 1, u)
    err_or = O.normwise_error(oracle_fast(name, A, B, depth, 1), ref, A64, B64)
    assert err <= 4 * err_or + 4 * u


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("scaling,steps", [("outside", 1), ("inside", 1), ("out_in", 2), ("repeated", 4)])
def test_written_scaled_against_oracle(precision, scaling, steps):
    """Badly scaled inputs: the error of the scaled written path entry by entry relative to
    r_i s_j ||A'|| ||B'|| (the scaled-error bound of section 6.3), within Theorem 4.1 and within 4x the oracle's own
    scaled product in the same precision; integers times powers of two stay bit-exact."""
    name, depth, shape = "f424", 2, (160, 96, 200)
    print(f"\n[written-scaled] {name} L={depth} {shape} {precision} {scaling}", flush=True)
    p = _plan(name, depth, precision, scaling, steps)
    assert p.path(*shape) == "written"
    dt = np_dtype(precision)
    A, B = make_pair("badly_scaled", 52, *shape, dtype=dt)
    got = run_gpu(p, A, B)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = O.reference_rows(A64, B64)
    sc = O.scale(A64, B64, O.schedule_for(scaling, steps), pow2=True)
    bound_mat = np.outer(sc.r, sc.s) * O.maxabs(sc.A) * O.maxabs(sc.B)
    rel = float(np.max(np.abs(got.astype(np.longdouble) - ref) / bound_mat))
    u = UNIT_ROUNDOFF[precision]
    assert rel <= theorem_bound(name, *shape, depth, 1, u)
    Cor = O.scaled_fast(A, B, C.get(name), depth, 1, mode=scaling, steps=steps)
    rel_or = float(np.max(np.abs(Cor.astype(np.longdouble) - ref) / bound_mat))
    assert rel <= 4 * rel_or + 4 * u
    # integers times powers of two (rows and columns): after an O step every scaled value, sum
    # and product is exact (the O step takes the row and column factors out again, so the S/T
    # sums mix entries of one scale); inside steps alone leave the factors in, and FP32 sums of
    # entries 2^8 apart need more than 24 bits, so there only FP64 is exact
    if precision == "f32" and "O" not in O.schedule_for(scaling, steps):
        return
    Ai, Bi = make_pair("int8", 53, *shape)
    Ai = (Ai * np.exp2(np.arange(shape[0]) % 9)[:, None]).astype(dt)
    Bi = (Bi * np.exp2(-(np.arange(shape[2]) % 7))[None, :]).astype(dt)
    got = run_gpu(p, Ai, Bi)
    assert np.array_equal(got.astype(np.float64), Ai.astype(np.float64) @ Bi.astype(np.float64))


@pytest.mark.parametrize("name,depth,shape", CASES_F64)
def test_written_f64_strassen_exact_and_against_oracle(name, depth, shape):
    """FP64 <2,2,2> rules take the written path by default: exact on integers, and within
    Theorem 4.1 and 4x the oracle's own error on N(0,1) inputs."""
    print(f"\n[written-f64] {name} L={depth} {shape}", flush=True)
    p = _plan(name, depth, "f64")
    assert p.path(*shape) == "written"
    A, B = make_pair("int8", 7, *shape)
    got = run_gpu(p, A.astype(np.float64), B.astype(np.float64))
    assert np.array_equal(got, (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))
    A, B = make_pair("normal", 8, *shape)
    got = run_gpu(p, A, B)
    ref = O.reference_rows(A, B)
    err = O.normwise_error(got, ref, A, B)
    assert err <= theorem_bound(name, *shape, depth, 1, UNIT_ROUNDOFF["f64"])
    err_or = O.normwise_error(oracle_fast(name, A, B, depth, 1), ref, A, B)
    assert err <= 4 * err_or + 4 * UNIT_ROUNDOFF["f64"]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,depth,shape", [("f424", 2, (200, 40, 180)), ("f323", 1, (150, 100, 120)),
                                              ("strassen", 2, (130, 200, 90))])
def test_written_transposed_operands_bitwise_equal(precision, name, depth, shape):
    """Transposed operands are read through the LDS-staged formation at the first level,
    row-major ones by the register-only formation; both form every S_r, T_r element with the
    same operations in the same order, so the products are bitwise equal."""
    print(f"\n[written-trans] {name} L={depth} {shape} {precision}", flush=True)
    import paper_1507_00687_amd as F

    p = F.Plan(name, depth, 1, precision=precision, fuse="written")
    m, k, n = shape
    assert p.path(m, k, n) == "written" and p.path(m, k, n, True, True) == "written"
    A, B = make_pair("normal", 9, m, k, n, dtype=np_dtype(precision))
    plain = run_gpu(p, A, B)
    trans = run_gpu(p, np.ascontiguousarray(A.T), np.ascontiguousarray(B.T), transA=True, transB=True)
    assert np.array_equal(plain, trans)
