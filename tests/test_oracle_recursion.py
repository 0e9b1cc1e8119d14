"""Pins for the oracle's recursion (eq. (2)), planning rules, reference and error bounds
(sections 3.2-3.4, 4.2-4.4).  CPU only."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair

ALGS = ["strassen", "winograd", "f323", "f332", "f424", "f442", "laderman333"]


def _int_exact(A, B):
    return (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)


@pytest.mark.parametrize("name", ALGS)
@pytest.mark.parametrize("L", [1, 2])
def test_integer_inputs_exact(name, L):
    # In exact arithmetic every valid [U,V,W] at any depth gives AB (eq. (2)); on small
    # integers every intermediate is an integer below 2^53, so FP64 is exact.  A wrong index
    # convention, sign or dropped term changes the result.
    alg = C.get(name)
    m, k, n = alg.M0 ** L * 3, alg.K0 ** L * 2, alg.N0 ** L * 3
    A, B = make_pair("int8", 7, m, k, n)
    assert np.array_equal(O.fast(A, B, alg, L), _int_exact(A, B))


@pytest.mark.parametrize("name", ["strassen", "f323", "f424"])
@pytest.mark.parametrize("shape", [(37, 29, 41), (1, 17, 5), (64, 1, 9), (65, 64, 63)])
def test_ragged_shapes_padding(name, shape):
    # Zero padding to multiples of the base sizes, then cropping (section 3.2).
    alg = C.get(name)
    A, B = make_pair("int8", 3, *shape)
    assert np.array_equal(O.fast(A, B, alg, 2), _int_exact(A, B))


@pytest.mark.parametrize("name", ["strassen", "winograd"])
def test_brute_force_one_level_exhaustive_small_entries(name):
    # Every pair A, B in {-1,0,1}^{2x2} (all 81 x 81 pairs): one level of the rule equals the
    # exact product.  A wrong sign, index or dropped term of [U,V,W] shows on some pair.
    alg = C.get(name)
    vals = [-1.0, 0.0, 1.0]
    combos = np.array(list(itertools.product(vals, repeat=4)))
    for a in combos:
        A = a.reshape(2, 2)
        for b in combos:
            B = b.reshape(2, 2)
            assert np.array_equal(O.fast(A, B, alg, 1), A @ B), (a, b)


def test_one_level_matches_eq1_scalar_formula():
    # Base-size inputs: the block recursion at depth 1 is eq. (1) on scalars.
    for name in ALGS:
        alg = C.get(name)
        A, B = make_pair("int8", 11, alg.M0, alg.K0, alg.N0)
        a = [A[i % alg.M0, i // alg.M0] for i in range(alg.M0 * alg.K0)]
        b = [B[j % alg.K0, j // alg.K0] for j in range(alg.K0 * alg.N0)]
        Cs = np.zeros((alg.M0, alg.N0))
        for kk in range(alg.M0 * alg.N0):
            tot = Fraction(0)
            for r in range(alg.R):
                S = sum((alg.U[i][r] * Fraction(a[i]) for i in range(len(a))), Fraction(0))
                T = sum((alg.V[j][r] * Fraction(b[j]) for j in range(len(b))), Fraction(0))
                tot += alg.W[kk][r] * S * T
            Cs[kk // alg.N0, kk % alg.N0] = float(tot)
        assert np.array_equal(O.fast(A, B, alg, 1), Cs)
        assert np.array_equal(Cs, _int_exact(A, B))


def test_uniform_nonstationary_tree_exact():
    # A different rule per level (section 3.3): <2,2,2> then <3,2,3>.
    levels = [C.strassen(), C.f323()]
    A, B = make_pair("int8", 5, 2 * 3 * 4, 2 * 2 * 3, 2 * 3 * 5)
    got = O.fast_tree(A, B, lambda path: levels[len(path)], [(2, 2, 2), (3, 2, 3)])
    assert np.array_equal(got, _int_exact(A, B))


def test_nonuniform_tree_exact():
    # D'Alberto's non-uniform Strassen (Example 4.2) computes AB.
    s = C.strassen()
    P = [[0, 1], [1, 0]]
    I2 = [[1, 0], [0, 1]]
    var = C.kron_perm_variant(s, list(range(4)), C.kron_index_perm(P, I2), C.kron_index_perm(I2, P), "v")
    A, B = make_pair("int8", 9, 16, 16, 16)
    got = O.fast_tree(A, B, lambda path: var if (len(path) == 1 and path[0] in (0, 2, 3)) else s,
                      [(2, 2, 2), (2, 2, 2)])
    assert np.array_equal(got, _int_exact(A, B))


def test_effective_depth_cutoff():
    d = [(2, 2, 2)] * 3
    assert O.effective_depth(256, 256, 256, d[:2], 64) == 2  # 64^3 leaves at n=256, L=2
    assert O.effective_depth(256, 256, 256, d, 64) == 2  # a third level would give 32 < 64
    assert O.effective_depth(256, 256, 256, d, 1) == 3
    assert O.effective_depth(100, 256, 256, d, 64) == 0  # ceil(100/2)=50 < 64
    assert O.effective_depth(4096, 4096, 4096, [(3, 2, 3)] * 3, 256) == 2  # ceil(4096/27)=152


def test_long_double_reference_against_exact_rationals():
    A, B = make_pair("uniform11", 2, 6, 40, 5)
    ref = O.reference_rows(A, B)
    for i in range(6):
        for j in range(5):
            exact = sum((Fraction(A[i, p]) * Fraction(B[p, j]) for p in range(40)), Fraction(0))
            bound = 40 * 2.0 ** -63 * float(sum(abs(A[i, p] * B[p, j]) for p in range(40)))
            assert abs(Fraction(float(ref[i, j])) - exact) <= Fraction(bound) + Fraction(2.0 ** -52) * abs(exact)


def test_classical_sequential_within_textbook_bound():
    A, B = make_pair("uniform01", 1, 16, 300, 12)
    Cc = O.classical(A, B)
    ref = O.reference_rows(A, B)
    u = 2.0 ** -53
    # |c^ - c| <= K u sum|a||b| (first order), per entry.
    absprod = np.abs(A) @ np.abs(B)
    assert np.all(np.abs(Cc.astype(np.longdouble) - ref) <= 300 * u * absprod * 1.01)


def test_thm42_bound_equals_thm41_for_identical_levels():
    # Theorem 4.2 with the same rule at every level is Theorem 4.1: sum of the levels' Q is
    # Q L, the product of their E is E^L and of their K0 is K0^L.
    for name in ["strassen", "winograd", "f323", "f424", "laderman333"]:
        alg = C.get(name)
        q = C.quantities(alg)
        for L in (1, 2, 3):
            K = 4 * alg.K0 ** L
            assert O.thm42_bound(K, [alg] * L, 2.0 ** -53) == O.thm41_bound(K, alg.K0, L, q.Q, q.E, 2.0 ** -53)


def test_thm42_bound_hand_value():
    # Strassen (Q 8, E 12, K0 2) above <3,2,3> (Q 10, E 20, K0 2), K = 64 (Table 1's values):
    # (64/4 + 8 + 10) (64/4) (12 * 20) u = 34 * 16 * 240 u = 130560 u.  A slip such as the
    # largest Q instead of the sum (26 * 16 * 240), K over one level's K0 (50 * 32 * 240) or
    # the sum of E instead of the product fails.
    u = 2.0 ** -53
    assert O.thm42_bound(64, [C.strassen(), C.f323()], u) == 130560 * u
    assert O.thm42_bound(64, [C.f323(), C.strassen()], u) == 130560 * u
    assert O.thm42_bound(64, [], u) == 64 * 64 * u  # no level: the classical K^2 bound


def test_two_level_nonstationary_error_within_thm42():
    levels = [C.strassen(), C.f323()]
    dims = [(2, 2, 2), (3, 2, 3)]
    for dist in ("uniform01", "normal"):
        A, B = make_pair(dist, 6, 6 * 40, 4 * 60, 6 * 40)
        got = O.fast_tree(A, B, lambda path: levels[len(path)], dims)
        err = O.normwise_error(got, O.reference_rows(A, B), A, B)
        assert 0 < err <= O.thm42_bound(4 * 60, levels, 2.0 ** -53)


def test_normwise_error_hand_value():
    # max |C^ - C| / (max|A| max|B|): one entry off by 1/2, max|A| = 2, max|B| = 3 -> 1/12.
    A = np.array([[1.0, -2.0], [0.0, 1.0]])
    B = np.array([[3.0, 0.0], [1.0, -1.0]])
    Cref = np.array([[1.0, 2.0], [3.0, 4.0]], dtype=np.longdouble)
    Chat = np.array([[1.0, 2.0], [3.0, 4.5]])
    assert O.normwise_error(Chat, Cref, A, B) == pytest.approx(1.0 / 12.0, rel=1e-15)
    # sampled rows: Cref holds only the sampled row
    assert O.normwise_error(Chat, Cref[[1]], A, B, rows=[1]) == pytest.approx(1.0 / 12.0, rel=1e-15)
    assert O.normwise_error(Chat, Cref[[0]], A, B, rows=[0]) == 0.0
    # the sign of the difference does not matter; the denominator uses max-abs, not max
    assert O.normwise_error(-Chat, -Cref, -A, -B) == pytest.approx(1.0 / 12.0, rel=1e-15)


def test_componentwise_error_hand_value():
    # max |c^ - c| / |c| over nonzero c: entries (0,0) off by 1/2 of 1, (1,1) by 1 of 5.
    Cref = np.array([[1.0, 2.0], [0.0, -5.0]], dtype=np.longdouble)
    Chat = np.array([[1.5, 2.0], [7.0, -4.0]])  # (1,0) has c = 0 and is skipped
    assert O.componentwise_error(Chat, Cref) == pytest.approx(0.5, rel=1e-15)
    assert O.componentwise_error(Chat, Cref[[1]], rows=[1]) == pytest.approx(0.2, rel=1e-15)


def test_thm41_special_cases():
    # L = 0: the classical K^2 bound (end of section 4.3).
    assert O.thm41_bound(1024, 2, 0, 8, 12, 1.0) == 1024.0 ** 2
    # Full recursion L = log_K0 K: (1 + Q L) E^L.
    assert O.thm41_bound(64, 2, 6, 8, 12, 1.0) == pytest.approx((1 + 8 * 6) * 12.0 ** 6)


@pytest.mark.parametrize("name", ["strassen", "winograd", "f323", "f424", "laderman333"])
@pytest.mark.parametrize("dist", ["uniform01", "normal"])
def test_measured_error_within_theorem_4_1(name, dist):
    alg = C.get(name)
    q = C.quantities(alg)
    n = 216 if alg.K0 == 3 else 256
    A, B = make_pair(dist, 0, n, n, n)
    ref = O.reference_rows(A, B)
    for L in (1, 2):
        Cf = O.fast(A, B, alg, L)
        Kp = O.padded_dims(n, n, n, [(alg.M0, alg.K0, alg.N0)] * L)[1]
        err = O.normwise_error(Cf, ref, A, B)
        assert err <= O.thm41_bound(Kp, alg.K0, L, q.Q, q.E, 2.0 ** -53)


def test_error_grows_with_depth_uniform01():
    # Section 5.1: the observed error increases with the number of recursive levels.
    A, B = make_pair("uniform01", 0, 512, 512, 512)
    ref = O.reference_rows(A, B)
    errs = [O.normwise_error(O.fast(A, B, C.strassen(), L), ref, A, B) for L in range(4)]
    assert errs[0] < errs[1] < errs[2] < errs[3]


def test_float32_recursion_and_classical():
    A, B = make_pair("normal", 4, 64, 64, 64, dtype=np.float32)
    C32 = O.fast(A, B, C.strassen(), 2)
    assert C32.dtype == np.float32
    ref = O.reference_rows(A.astype(np.float64), B.astype(np.float64))
    err = O.normwise_error(C32, ref, A, B)
    assert err <= O.thm41_bound(64, 2, 2, 8, 12, 2.0 ** -24)
    assert err > 1e-9  # single precision really was used


def test_gradients_match_finite_differences():
    # The loss <G, AB> is linear in A, so a central difference is exact up to rounding.
    A, B = make_pair("normal", 1, 5, 7, 6)
    G = make_pair("normal", 2, 5, 6, 6)[0]
    dA, dB = O.gradients(A, B, G)
    h = 0.5
    for (i, j) in [(0, 0), (3, 6), (4, 2)]:
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (np.sum(G * O.classical(Ap, B)) - np.sum(G * O.classical(Am, B))) / (2 * h)
        assert fd == pytest.approx(dA[i, j], rel=1e-12, abs=1e-12)
    for (i, j) in [(0, 0), (6, 5)]:
        Bp, Bm = B.copy(), B.copy()
        Bp[i, j] += h
        Bm[i, j] -= h
        fd = (np.sum(G * O.classical(A, Bp)) - np.sum(G * O.classical(A, Bm))) / (2 * h)
        assert fd == pytest.approx(dB[i, j], rel=1e-12, abs=1e-12)
