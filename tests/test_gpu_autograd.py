"""GPU tests of the differentiable path: dA = G B^T and dB = A^T G through the rotated fast
algorithms, against exact products, the oracle's gradients and finite differences."""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair
from synth.gen import TAG_G, int_uniform, normal01
from tests.gpu_util import np_dtype

pytestmark = pytest.mark.gpu

ROTATED = {  # rule of the plan -> (rule computing dA^T = B G^T, rule computing dB^T = G^T A)
    "strassen": ("strassen", "strassen"),
    "f323": ("f233", "f332"),
    "f424": ("f442", "f244"),
}


def _grad_case(name, depth, precision, m, k, n, dist="int8", seed=0):
    import torch

    import paper_1507_00687_amd as F

    dt = np_dtype(precision)
    A, B = make_pair(dist, seed, m, k, n, dtype=dt)
    G = (int_uniform(seed, TAG_G, (m, n)) if dist == "int8" else normal01(seed, TAG_G, (m, n))).astype(dt)
    plan = F.Plan(name, depth, 1, precision=precision)
    tA = torch.from_numpy(A).cuda().requires_grad_(True)
    tB = torch.from_numpy(B).cuda().requires_grad_(True)
    Cg = F.fast_matmul(tA, tB, plan)
    Cg.backward(torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    return A, B, G, Cg.detach().cpu().numpy(), tA.grad.cpu().numpy(), tB.grad.cpu().numpy()


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("name,depth", [("strassen", 2), ("f323", 1), ("f424", 1), ("winograd", 1)])
def test_gradients_integer_bit_exact(precision, name, depth):
    print(f"\n[grad-int] {name} L={depth} {precision}", flush=True)
    m, k, n = 96, 80, 112
    A, B, G, Cg, dA, dB = _grad_case(name, depth, precision, m, k, n)
    i64 = lambda X: X.astype(np.int64)
    assert np.array_equal(Cg.astype(np.float64), (i64(A) @ i64(B)).astype(np.float64))
    assert np.array_equal(dA.astype(np.float64), (i64(G) @ i64(B).T).astype(np.float64))
    assert np.array_equal(dB.astype(np.float64), (i64(A).T @ i64(G)).astype(np.float64))


@pytest.mark.parametrize("name", ["strassen", "f323", "f424"])
def test_gradients_float_against_oracle(name):
    m, k, n = 144, 128, 160
    A, B, G, Cg, dA, dB = _grad_case(name, 1, "f64", m, k, n, dist="normal", seed=3)
    dA_o, dB_o = O.gradients(A, B, G)
    refA = O.reference_rows(G, np.ascontiguousarray(B.T))
    refB = O.reference_rows(np.ascontiguousarray(A.T), G)
    errA = O.normwise_error(dA, refA, G, B)
    errB = O.normwise_error(dB, refB, A, G)
    rotA, rotB = (C.get(x) for x in ROTATED[name])
    qa, qb = C.quantities(rotA), C.quantities(rotB)
    u = 2.0 ** -53
    # dA^T = B G^T is a product with inner dimension n, dB^T = G^T A with inner dimension m
    assert errA <= O.thm41_bound(O.padded_dims(k, n, m, [(rotA.M0, rotA.K0, rotA.N0)])[1], rotA.K0, 1, qa.Q, qa.E, u)
    assert errB <= O.thm41_bound(O.padded_dims(n, m, k, [(rotB.M0, rotB.K0, rotB.N0)])[1], rotB.K0, 1, qb.Q, qb.E, u)
    assert errA <= 1e-13 and errB <= 1e-13
    assert np.allclose(dA, dA_o, rtol=0, atol=1e-12 * np.max(np.abs(dA_o)))
    assert np.allclose(dB, dB_o, rtol=0, atol=1e-12 * np.max(np.abs(dB_o)))


def test_gradients_match_finite_differences():
    # loss = <G, fast(A, B)> is linear in A and in B: with integer data and step 1 every
    # quantity is an exactly representable integer, so the central difference equals the
    # gradient exactly.
    import torch

    import paper_1507_00687_amd as F

    m, k, n = 40, 36, 44
    A, B = make_pair("int8", 8, m, k, n)
    G = int_uniform(8, TAG_G, (m, n))
    plan = F.Plan("f323", 1, 1, precision="f64")
    tG = torch.from_numpy(G).cuda()

    def loss(Ah, Bh):
        return float(torch.sum(tG * F.fastmm_gemm(plan, torch.from_numpy(Ah).cuda(), torch.from_numpy(Bh).cuda())))

    _, _, _, _, dA, dB = _grad_case("f323", 1, "f64", m, k, n, seed=8)
    for (i, j) in [(0, 0), (17, 5), (39, 35)]:
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += 1.0
        Am[i, j] -= 1.0
        assert (loss(Ap, B) - loss(Am, B)) / 2.0 == dA[i, j]
    for (i, j) in [(0, 0), (20, 43), (35, 1)]:
        Bp, Bm = B.copy(), B.copy()
        Bp[i, j] += 1.0
        Bm[i, j] -= 1.0
        assert (loss(A, Bp) - loss(A, Bm)) / 2.0 == dB[i, j]


def test_torch_gradcheck():
    import torch

    import paper_1507_00687_amd as F

    plan = F.Plan("strassen", 2, 1, precision="f64")
    # finite differences with step 1e-6 carry ~u |C| / 1e-6 ~ 1e-9 noise
    An, Bn = make_pair("normal", 12, 9, 7, 11)
    A = torch.from_numpy(An).cuda().requires_grad_(True)
    B = torch.from_numpy(Bn).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: F.fast_matmul(a, b, plan), (A, B), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_backward_only_one_input_needs_grad():
    import torch

    import paper_1507_00687_amd as F

    A, B = make_pair("int8", 1, 64, 48, 56)
    plan = F.Plan("strassen", 1, 1, precision="f64")
    tA = torch.from_numpy(A).cuda().requires_grad_(True)
    tB = torch.from_numpy(B).cuda()
    F.fast_matmul(tA, tB, plan).sum().backward()
    assert tB.grad is None
    assert np.array_equal(tA.grad.cpu().numpy(), np.ones((64, 56)) @ B.T)
