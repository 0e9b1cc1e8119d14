"""fastmm_gemm_noalloc against fastmm_gemm, through the C ABI.

The no-allocation entry point runs the same kernels on the library's fixed scratch array, so its
result must equal fastmm_gemm's bit for bit.  Two calls in a row, the second on a smaller
input, so the second runs on the array the first left behind.  Also: a product needing more
workspace than the array holds is refused before any launch, and a plan whose task tables are
not on the device yet is refused instead of uploading them.
"""
import ctypes

import numpy as np
import pytest

from synth import make_pair

pytestmark = pytest.mark.gpu

CASES = [  # (algo, depth, cutoff, precision, scaling, first n, second n)
    ("strassen", 1, 64, "f16x3", "outside", 1024, 520),
    ("strassen", 2, 64, "f32", "none", 1024, 384),
    ("strassen", 2, 64, "f64", "out_in", 768, 256),
    ("f424", 1, 64, "bf16x3", "none", 1024, 300),
    ("strassen", 2, 64, "f16x3", "repeated", 1024, 640),
]


def _noalloc(F, plan, A, B, C):
    """The C-ABI call on torch's current stream; returns its status."""
    import torch

    return F.lib().fastmm_gemm_noalloc(plan.handle, A.data_ptr(), B.data_ptr(), C.data_ptr(), A.shape[0],
                                       A.shape[1], B.shape[1], int(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("algo,depth,cutoff,precision,scaling,n1,n2", CASES)
def test_noalloc_equals_gemm_twice(algo, depth, cutoff, precision, scaling, n1, n2):
    import torch

    import paper_1507_00687_amd as F

    print(f"\n[noalloc] {algo} L={depth} {precision} scaling={scaling} n={n1} then n={n2}", flush=True)
    plan = F.Plan(algo, depth, cutoff, scaling=scaling, precision=precision)
    dt = np.float64 if precision == "f64" else np.float32
    for i, n in enumerate((n1, n2)):
        A, B = make_pair("normal", 40 + i, n, n + 8, n - 4, dtype=dt)
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        want = F.fastmm_gemm(plan, tA, tB)  # also uploads the plan's tables for this depth
        torch.cuda.synchronize()
        got = torch.full_like(want, float("nan"))
        st = _noalloc(F, plan, tA, tB, got)
        assert st == 0, F.lib().fastmm_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"call {i + 1}: results differ"


def test_noalloc_rejects_oversized_and_unprepared():
    import torch

    import paper_1507_00687_amd as F

    print("\n[noalloc] oversized and unprepared plans", flush=True)
    n = 8192  # F16X3 Strassen depth 1: limb planes and products far above the array
    plan = F.Plan("strassen", 1, 64, precision="f16x3")
    need = plan.workspace_size(n, n, n)
    limit = 256 << 20
    assert need > limit
    A = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    C = torch.full((n, n), 7.0, dtype=torch.float32, device="cuda")
    st = _noalloc(F, plan, A, A, C)
    assert st == -8  # FASTMM_EWORKSPACE
    assert str(limit) in F.lib().fastmm_last_error().decode()
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())  # nothing launched
    # a fresh plan has no task tables on the device: refused, nothing launched
    plan2 = F.Plan("winograd", 1, 16, precision="f32")
    A2 = torch.ones((256, 256), dtype=torch.float32, device="cuda")
    C2 = torch.full((256, 256), 7.0, dtype=torch.float32, device="cuda")
    st = _noalloc(F, plan2, A2, A2, C2)
    assert st == -6  # FASTMM_EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((C2 == 7.0).all())
    # after one fastmm_gemm call the same plan runs without allocating
    want = F.fastmm_gemm(plan2, A2, A2)
    assert _noalloc(F, plan2, A2, A2, C2) == 0
    torch.cuda.synchronize()
    assert torch.equal(C2, want)
