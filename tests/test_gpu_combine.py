"""GPU tests of the W-combination forms: the register forms for one and two levels of
<2,K0,2> rules and for one level of a 16-block rule, against the exact product (integer
inputs) and the oracle (floats), on shapes that take the 16-byte and the element-wise paths
(n a multiple of 4 or not, ragged m), with and without outside scaling; the two-level form's
level-by-level sums on FP64 inputs within the oracle's own error (same association)."""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import run_gpu

pytestmark = pytest.mark.gpu

CASES = [("strassen", 1), ("winograd", 1), ("strassen", 2), ("winograd", 2), ("f424", 1)]
SHAPES = [(200, 96, 240), (131, 70, 190), (97, 64, 101)]


def _plan(name, depth, precision, scaling="none", fuse="off"):
    import paper_1507_00687_amd as F

    return F.Plan(name, depth, 1, scaling=scaling, precision=precision, fuse=fuse)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3"])
@pytest.mark.parametrize("scaling", ["none", "outside"])
@pytest.mark.parametrize("name,depth", CASES)
@pytest.mark.parametrize("shape", SHAPES)
def test_combination_integer_exact(precision, scaling, name, depth, shape):
    print(f"\n[combine-int] {name} L={depth} {shape} {precision} {scaling}", flush=True)
    A, B = make_pair("int8", 90, *shape, dtype=np.float64 if precision == "f64" else np.float32)
    got = run_gpu(_plan(name, depth, precision, scaling), A, B)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(got.astype(np.float64), exact)


@pytest.mark.parametrize("name,depth", CASES)
def test_combination_float_within_oracle(name, depth):
    shape = (256, 192, 256)
    print(f"\n[combine-float] {name} L={depth} {shape} f64", flush=True)
    A, B = make_pair("normal", 91, *shape)
    got = run_gpu(_plan(name, depth, "f64"), A, B)
    ref = O.reference_rows(A, B)
    err = O.normwise_error(got, ref, A, B)
    err_oracle = O.normwise_error(O.fast(A, B, C.get(name), depth), ref, A, B)
    print(f"  error {err:.3e}, oracle's own {err_oracle:.3e}", flush=True)
    assert err <= 4 * err_oracle + 8 * 2.0 ** -53


@pytest.mark.parametrize("precision", ["f64", "f16x3"])
@pytest.mark.parametrize("name,depth", CASES)
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (9, 4, 17)])
def test_combination_tiny_shapes(precision, name, depth, shape):
    print(f"\n[combine-tiny] {name} L={depth} {shape} {precision}", flush=True)
    A, B = make_pair("int8", 92, *shape, dtype=np.float64 if precision == "f64" else np.float32)
    got = run_gpu(_plan(name, depth, precision), A, B)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(got.astype(np.float64), exact)
