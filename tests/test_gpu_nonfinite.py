"""Non-finite inputs and the range of fp16 limbs.

Non-finite entries are not errors: they propagate as IEEE arithmetic does, and a row or column
whose maximum is not finite (NaN or infinity) gets scaling factor 1, like an all-zero one
(the oracle's rule for Algorithms 1-3).  The set of non-finite outputs depends only on which
inputs reach which outputs through S_r, T_r, M_r and the W-sums (eq. (2)), so the GPU and the
oracle running the same rule must agree on it exactly; for FP64 and FP32 they must also agree on
NaN against +-infinity.  Split precisions turn an infinite entry into a NaN low limb (inf - inf),
so there only the non-finite set is compared.  Finite outputs are held to the oracle's own
fast product within the usual factor.

Also: inside scaling alone leaves entries of any size, so F16/F16X3 limbs must not be moved up
by the 2^8 offset that follows an O step (it would overflow fp16 for entries above 256).
"""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair
from tests.gpu_util import np_dtype, run_gpu

pytestmark = pytest.mark.gpu


def _plan(precision, scaling, depth=1, name="strassen", steps=4):
    import paper_1507_00687_amd as F

    return F.Plan(name, depth, 16, scaling=scaling, steps=steps, precision=precision)


def _inputs(dtype, n=128):
    A, B = make_pair("normal", 31, n, n, n)
    A[5, 17] = np.nan          # one NaN in A
    A[70, 3] = np.inf          # +inf in A
    B[40, 99] = -np.inf        # -inf in B
    B[:, 120] = 0.0            # an all-zero column of B (factor 1 as well)
    return A.astype(dtype), B.astype(dtype)


def _oracle(A, B, scaling, depth=1):
    alg = C.strassen()
    if scaling == "none":
        return O.fast(A, B, alg, depth, 16)
    return O.scaled_fast(A, B, alg, depth, 16, mode=scaling)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3", "bf16x3"])
@pytest.mark.parametrize("scaling", ["none", "outside", "out_in"])
def test_nonfinite_propagation_matches_oracle(precision, scaling):
    print(f"\n[nonfinite] strassen L=1 n=128 {precision} scaling={scaling}", flush=True)
    dt = np_dtype(precision)
    A, B = _inputs(dt)
    got = run_gpu(_plan(precision, scaling), A, B).astype(np.float64)
    want = _oracle(A.astype(np.float64), B.astype(np.float64), scaling)
    bad_g, bad_w = ~np.isfinite(got), ~np.isfinite(want)
    assert bad_w.any()
    assert np.array_equal(bad_g, bad_w)
    if precision in ("f64", "f32"):
        assert np.array_equal(np.isnan(got), np.isnan(want))
        inf = np.isinf(want)
        assert np.array_equal(np.sign(got[inf]), np.sign(want[inf]))
    # finite outputs: within the precision's reach of the oracle's FP64 product
    ok = ~bad_w
    Af, Bf = np.where(np.isfinite(A), A, 0.0), np.where(np.isfinite(B), B, 0.0)
    den = float(np.max(np.abs(Af))) * float(np.max(np.abs(Bf)))
    tol = {"f64": 1e-13, "f32": 1e-5, "f16x3": 1e-5, "bf16x3": 2e-4}[precision]
    assert np.max(np.abs(got[ok] - want[ok])) / den <= tol


@pytest.mark.parametrize("scaling", ["outside", "out_in", "repeated"])
def test_nonfinite_scaling_exponents_match_oracle(scaling):
    """Rows / columns with a NaN or infinite maximum keep factor 1 (exponent 0 from their
    steps), bit-exact against the oracle's power-of-two factors."""
    import torch

    import paper_1507_00687_amd as F

    print(f"\n[nonfinite-exps] n=128 f32 scaling={scaling}", flush=True)
    A, B = _inputs(np.float32)
    plan = _plan("f32", scaling)
    ea, eb, ep = F.fastmm_scaling_exponents(plan, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    sc = O.scale(A.astype(np.float64), B.astype(np.float64), O.schedule_for(scaling, 4))
    assert np.array_equal(ea.cpu().numpy(), np.log2(sc.r).astype(np.int64))
    assert np.array_equal(eb.cpu().numpy(), np.log2(sc.s).astype(np.int64))
    assert np.array_equal(ep.cpu().numpy(), np.log2(sc.p).astype(np.int64))


@pytest.mark.parametrize("precision", ["f16", "f16x3"])
@pytest.mark.parametrize("depth", [0, 1])
def test_inside_scaling_large_entries_fp16_no_overflow(precision, depth):
    """Integers times 2^7 (entries up to 1024): inside scaling keeps them at that size, the fp16
    limbs hold them exactly, and every product and partial sum stays an exact FP32 value, so
    the result must be the exact product (an offset of 2^8 would overflow fp16 here)."""
    n = 256
    print(f"\n[inside-fp16] strassen L={depth} n={n} {precision} entries up to 1024", flush=True)
    A, B = make_pair("int8", 32, n, n, n)
    A, B = (A * 128.0).astype(np.float32), (B * 128.0).astype(np.float32)
    got = run_gpu(_plan(precision, "inside", depth), A, B)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got.astype(np.float64), exact)
