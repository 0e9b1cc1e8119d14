"""GPU tests of the backward products dA = G B^T and dB = A^T G (section 3.1: the transposes of
the rotated rules, transposed operands read through the transpose flags), single and batched
(fastmm_gemm_backward_batched: every gradient product of the batch in one launch), and of the
strided / transposed batched forward (fastmm_gemm_batched_ex).

Integer inputs are exact in every precision.  Float gradients are held to Theorem 4.1 for the
gradient products (same Q and E as the plan's rule: transposition and rotation only relabel the
products) with the precision's unit roundoff, and to the oracle's classical gradients.
"""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair
from synth.gen import TAG_G, int_uniform, normal01
from tests.gpu_util import np_dtype

pytestmark = pytest.mark.gpu

U_EFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16x3": 2.0 ** -16, "f16x3": 2.0 ** -22}


def _inputs(dist, seed, m, k, n, precision):
    dt = np_dtype(precision)
    A, B = make_pair(dist, seed, m, k, n, dtype=dt)
    G = (int_uniform(seed, TAG_G, (m, n)) if dist == "int8" else normal01(seed, TAG_G, (m, n))).astype(dt)
    return A, B, G


def _single(plan, A, B, G):
    import torch

    import paper_1507_00687_amd as F

    tA, tB, tG = (torch.from_numpy(X).cuda() for X in (A, B, G))
    dA, dB = F.fastmm_gemm_backward(plan, tA, tB, tG)
    torch.cuda.synchronize()
    return dA.cpu().numpy(), dB.cpu().numpy()


def _bound(name, depth, inner, u):
    a = C.get(name)
    q = C.quantities(a)
    Kp = O.padded_dims(1, inner, 1, [(a.N0, a.N0, a.N0)] * depth)[1]  # inner dimension of dA (n) padded by N0^L
    return O.thm41_bound(Kp, a.N0, depth, q.Q, q.E, u)


@pytest.mark.parametrize("precision", ["f32", "f16x3", "bf16x3"])
@pytest.mark.parametrize("name,depth", [("strassen", 1), ("strassen", 2), ("winograd", 2)])
@pytest.mark.parametrize("scaling", ["none", "outside"])
def test_gradients_float_against_oracle(precision, name, depth, scaling):
    """dA and dB on N(0,1) inputs against the classical gradients in long double: normwise error
    within Theorem 4.1 with the precision's unit roundoff (for <2,2,2> rules every index is
    split by 2, so the padded inner dimensions of dA (n) and dB (m) follow the same rule)."""
    import paper_1507_00687_amd as F

    m, k, n = 520, 388, 456
    print(f"\n[grad-float] {name} L={depth} {precision} {scaling}", flush=True)
    A, B, G = _inputs("normal", 21, m, k, n, precision)
    plan = F.Plan(name, depth, 1, precision=precision, scaling=scaling)
    dA, dB = _single(plan, A, B, G)
    A64, B64, G64 = (X.astype(np.float64) for X in (A, B, G))
    rows_a = np.unique(np.linspace(0, m - 1, 24).astype(np.int64))
    rows_b = np.unique(np.linspace(0, k - 1, 24).astype(np.int64))
    refA = O.reference_rows(G64, np.ascontiguousarray(B64.T), rows_a)
    refB = O.reference_rows(np.ascontiguousarray(A64.T), G64, rows_b)
    errA = O.normwise_error(dA.astype(np.float64), refA, G64, np.ascontiguousarray(B64.T), rows_a)
    errB = O.normwise_error(dB.astype(np.float64), refB, np.ascontiguousarray(A64.T), G64, rows_b)
    u = U_EFF[precision]
    print(f"  error dA {errA:.3e} dB {errB:.3e} bound {_bound(name, depth, n, u):.3e}", flush=True)
    assert errA <= _bound(name, depth, n, u)
    assert errB <= _bound(name, depth, m, u)
    # and against the oracle's gradients (classical, FP64) on the same rows
    dA_o, dB_o = O.gradients(A64, B64, G64)
    tol = 64 * u * max(n, m)
    assert np.max(np.abs(dA[rows_a] - dA_o[rows_a])) <= tol * np.max(np.abs(G64)) * np.max(np.abs(B64)) * 1.0
    assert np.max(np.abs(dB[rows_b] - dB_o[rows_b])) <= tol * np.max(np.abs(A64)) * np.max(np.abs(G64)) * 1.0


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3"])
def test_gradients_empty_inner_dimension_is_zero(precision):
    """m = 0: dB = A^T G sums over nothing and comes back zero (likewise dA for n = 0)."""
    import torch

    import paper_1507_00687_amd as F

    plan = F.Plan("strassen", 1, 1, precision=precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    A = torch.empty((0, 24), dtype=dt, device="cuda")
    B = torch.ones((24, 40), dtype=dt, device="cuda")
    G = torch.empty((0, 40), dtype=dt, device="cuda")
    dA, dB = F.fastmm_gemm_backward(plan, A, B, G)
    assert dA.shape == (0, 24) and dB.shape == (24, 40)
    assert torch.count_nonzero(dB).item() == 0
    A2 = torch.ones((16, 24), dtype=dt, device="cuda")
    B2 = torch.empty((24, 0), dtype=dt, device="cuda")
    G2 = torch.empty((16, 0), dtype=dt, device="cuda")
    dA2, dB2 = F.fastmm_gemm_backward(plan, A2, B2, G2)
    assert dA2.shape == (16, 24) and torch.count_nonzero(dA2).item() == 0


# (rule, depth, (m, k, n)): mixed rules, depths, ragged shapes
BATCH = [
    ("classical", 0, (130, 70, 90)),
    ("strassen", 1, (256, 128, 512)),
    ("f323", 1, (198, 96, 180)),
    ("winograd", 2, (64, 512, 96)),
    ("f424", 1, (512, 64, 128)),
    ("strassen", 2, (260, 300, 140)),
]


def _batch(precision, dist, scaling="none"):
    import torch

    import paper_1507_00687_amd as F

    plans, leaf_plans, host, dev = [], [], [], []
    for i, (name, depth, (m, k, n)) in enumerate(BATCH):
        A, B, G = _inputs(dist, 200 + i, m, k, n, precision)
        host.append((A, B, G))
        dev.append(tuple(torch.from_numpy(X).cuda() for X in (A, B, G)))
        plans.append(F.Plan(name, depth, 1, precision=precision, scaling=scaling))
        # the batched launch's path for FP64 / FP32 (no fused kernel): single launches on it
        leaf_plans.append(F.Plan(name, depth, 1, precision=precision, scaling=scaling, fuse="written"))
    got = F.fastmm_gemm_backward_batched(plans, [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev])
    singles = [F.fastmm_gemm_backward(p, *d) for p, d in zip(leaf_plans, dev)]
    torch.cuda.synchronize()
    cpu = lambda pair: tuple(x.cpu().numpy() for x in pair)
    return host, [cpu(g) for g in got], [cpu(s) for s in singles]


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3", "bf16x3"])
def test_batched_backward_integer_exact_and_equal_to_single(precision):
    print(f"\n[grad-batched-int] {precision}", flush=True)
    host, got, singles = _batch(precision, "int8")
    i64 = lambda X: X.astype(np.int64)
    for (A, B, G), (dA, dB), (sA, sB) in zip(host, got, singles):
        assert np.array_equal(dA.astype(np.float64), (i64(G) @ i64(B).T).astype(np.float64))
        assert np.array_equal(dB.astype(np.float64), (i64(A).T @ i64(G)).astype(np.float64))
        assert np.array_equal(dA, sA) and np.array_equal(dB, sB)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3"])
@pytest.mark.parametrize("scaling", ["none", "outside"])
def test_batched_backward_float_equal_to_single(precision, scaling):
    """Every tile of the batched launch is computed by the same code in the same order as in a
    single launch on the same path: bitwise equal."""
    print(f"\n[grad-batched-float] {precision} {scaling}", flush=True)
    host, got, singles = _batch(precision, "normal", scaling)
    for (dA, dB), (sA, sB) in zip(got, singles):
        assert np.array_equal(dA, sA) and np.array_equal(dB, sB)


def test_batched_backward_only_one_gradient():
    import torch

    import paper_1507_00687_amd as F

    A, B, G = _inputs("int8", 5, 96, 64, 80, "f32")
    plan = F.Plan("strassen", 1, 1, precision="f32")
    tA, tB, tG = (torch.from_numpy(X).cuda() for X in (A, B, G))
    (dA, dB), = F.fastmm_gemm_backward_batched([plan], [tA], [tB], [tG], need_dA=True, need_dB=False)
    assert dB is None
    i64 = lambda X: X.astype(np.int64)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), (i64(G) @ i64(B).T).astype(np.float64))


@pytest.mark.parametrize("precision", ["f64", "f32", "f16x3"])
def test_batched_ex_transposed_and_strided_operands(precision):
    """fastmm_gemm_batched_ex with every transpose combination and row-strided views: exact on
    integers and bitwise equal to fastmm_gemm_ex on the same path."""
    import torch

    import paper_1507_00687_amd as F

    dt = np_dtype(precision)
    cases = [("strassen", 1, (200, 136, 264), False, False), ("strassen", 2, (260, 300, 140), True, False),
             ("f424", 1, (256, 96, 192), False, True), ("winograd", 2, (130, 260, 70), True, True),
             ("classical", 0, (64, 40, 72), True, True)]
    plans, leaf_plans, As, Bs, tAs, tBs, exact = [], [], [], [], [], [], []
    for i, (name, depth, (m, k, n), ta, tb) in enumerate(cases):
        A, B = make_pair("int8", 300 + i, m, k, n, dtype=dt)
        exact.append((A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))
        SA = np.ascontiguousarray(A.T) if ta else A
        SB = np.ascontiguousarray(B.T) if tb else B
        # stored inside a wider buffer: row stride 8 elements beyond the row length
        wa = torch.zeros((SA.shape[0], SA.shape[1] + 8), dtype=torch.from_numpy(SA).dtype, device="cuda")
        wb = torch.zeros((SB.shape[0], SB.shape[1] + 8), dtype=torch.from_numpy(SB).dtype, device="cuda")
        wa[:, :SA.shape[1]] = torch.from_numpy(SA).cuda()
        wb[:, :SB.shape[1]] = torch.from_numpy(SB).cuda()
        As.append(wa[:, :SA.shape[1]])
        Bs.append(wb[:, :SB.shape[1]])
        tAs.append(ta)
        tBs.append(tb)
        plans.append(F.Plan(name, depth, 1, precision=precision))
        leaf_plans.append(F.Plan(name, depth, 1, precision=precision, fuse="written"))
    print(f"\n[batched-ex] {precision}", flush=True)
    got = F.fastmm_gemm_batched_ex(plans, As, Bs, tAs, tBs)
    singles = [F.fastmm_gemm_ex(p, a.contiguous(), ta, b.contiguous(), tb)
               for p, a, b, ta, tb in zip(leaf_plans, As, Bs, tAs, tBs)]
    torch.cuda.synchronize()
    for g, s, e in zip(got, singles, exact):
        assert np.array_equal(g.cpu().numpy().astype(np.float64), e)
        assert np.array_equal(g.cpu().numpy(), s.cpu().numpy())
