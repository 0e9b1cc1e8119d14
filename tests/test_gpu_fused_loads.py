"""The split-precision path with the innermost level formed in the limb GEMM's tile loads
(`fused_loads`, taken with fusion mode "always"): S_r = sum_i u_ir A_i and T_r^T =
sum_j v_jr B_j^T (eq. (1)) are summed in FP32
from the loaded tiles of the node operands, split into limbs in registers and staged in LDS;
no limb planes are written.

Integer inputs are exact: every entry, sum, limb, product and partial sum is an integer inside
FP32's 24 bits.  Floating-point results are held to Theorem 4.1 with the two-limb unit roundoff
and to the same plan through limb planes (fusion off: same sums, same limbs, only the MFMA
accumulation order differs), and to the oracle's own fast product in FP64.
"""
import numpy as np
import pytest

from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import oracle_fast, run_gpu, theorem_bound

pytestmark = pytest.mark.gpu

U_EFF = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "bf16x3": 2.0 ** -16, "f16x3": 2.0 ** -22}

# (rule, depth, shape): 256-wide leaf blocks or more; ragged m, n; k a multiple of 8 or not
CASES = [
    ("classical", 0, (512, 512, 512)),
    ("classical", 0, (600, 520, 300)),
    ("strassen", 1, (512, 512, 512)),
    ("strassen", 1, (520, 1032, 600)),
    ("strassen", 1, (512, 517, 512)),
    ("strassen", 2, (1024, 1024, 1024)),
    ("strassen", 2, (1100, 1040, 1030)),
]


def _plan(name, depth, precision, scaling="none", fuse="always"):
    import paper_1507_00687_amd as F

    return F.Plan(name, depth, 1, scaling=scaling, precision=precision, fuse=fuse)


@pytest.mark.parametrize("precision", ["f16x3", "bf16x3", "f16"])
@pytest.mark.parametrize("name,depth,shape", CASES)
@pytest.mark.parametrize("scaling", ["none", "outside", "out_in"])
def test_fused_loads_integer_exact(precision, name, depth, shape, scaling):
    print(f"\n[fused-loads-int] {name} L={depth} {shape} {precision} {scaling}", flush=True)
    p = _plan(name, depth, precision, scaling)
    assert p.path(*shape) == "fused_loads"
    A, B = make_pair("int8", 60, *shape, dtype=np.float32)
    got = run_gpu(p, A, B)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.array_equal(got.astype(np.float64), exact)


@pytest.mark.parametrize("precision", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("name,depth,shape", CASES)
def test_fused_loads_float_against_planes_and_oracle(precision, name, depth, shape):
    print(f"\n[fused-loads-float] {name} L={depth} {shape} {precision}", flush=True)
    A, B = make_pair("normal", 61, *shape, dtype=np.float32)
    got = run_gpu(_plan(name, depth, precision), A, B)
    planes = run_gpu(_plan(name, depth, precision, fuse="off"), A, B)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    rows = np.unique(np.linspace(0, shape[0] - 1, 24).astype(np.int64))
    ref = O.reference_rows(A64, B64, rows)
    err = O.normwise_error(got, ref, A64, B64, rows)
    err_planes = O.normwise_error(planes, ref, A64, B64, rows)
    assert err <= theorem_bound(name, *shape, depth, 1, U_EFF[precision])
    assert err <= 1.5 * err_planes
    err_or = O.normwise_error(oracle_fast(name, A64, B64, depth, 1)[rows], ref, A64, B64, None)
    print(f"  error fused {err:.3e} planes {err_planes:.3e} oracle fp64 {err_or:.3e}", flush=True)


@pytest.mark.parametrize("transA,transB", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("depth", [1, 2])
def test_fused_loads_transposed_operands(transA, transB, depth):
    m, k, n = 1024, 1024, 1040
    print(f"\n[fused-loads-trans] strassen L={depth} transA={transA} transB={transB}", flush=True)
    p = _plan("strassen", depth, "f16x3", "outside")
    assert p.path(m, k, n, transA, transB) == "fused_loads"
    A, B = make_pair("int8", 62, m, k, n, dtype=np.float32)
    As = np.ascontiguousarray(A.T) if transA else A
    Bs = np.ascontiguousarray(B.T) if transB else B
    got = run_gpu(p, As, Bs, transA, transB)
    assert np.array_equal(got.astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))


def test_fused_loads_badly_scaled_outside():
    """Rows and columns 10^u apart: outside scaling keeps every fp16 limb in range; the fused
    path's componentwise error stays within 2x that of the limb-plane path."""
    shape = (1024, 1024, 1024)
    print("\n[fused-loads-badly] strassen L=2 f16x3 outside", flush=True)
    A, B = make_pair("badly_scaled", 63, *shape, dtype=np.float32)
    got = run_gpu(_plan("strassen", 2, "f16x3", "outside"), A, B)
    planes = run_gpu(_plan("strassen", 2, "f16x3", "outside", fuse="off"), A, B)
    assert np.all(np.isfinite(got))
    rows = np.unique(np.linspace(0, shape[0] - 1, 16).astype(np.int64))
    ref = O.reference_rows(A.astype(np.float64), B.astype(np.float64), rows)
    e_got = O.componentwise_error(got[rows], ref)
    e_pl = O.componentwise_error(planes[rows], ref)
    print(f"  componentwise fused {e_got:.3e} planes {e_pl:.3e}", flush=True)
    assert e_got <= 2.0 * e_pl + 1e-6
