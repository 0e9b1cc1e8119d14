"""Pins for the oracle's diagonal scaling: Algorithms 1-3, the worked 2x2 examples of section 6
(numbered 6.1-6.5 here in the paper's order: outside scaling, inside scaling, inside-outside
against outside-inside (two), scaling not always enough), the invariants of Lemma D.1, the
closed form of Lemma D.5 (Appendix D) and the stopping-criterion theorem of section 6.3.  CPU only.  The symbolic small entry z of the examples is a power of two here so
that the power-of-two variant and the exact variant coincide."""
import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import badly_scaled
from tests.dyadic import dyadic_pair, exact_product

Z = 2.0 ** -20
SZ = 2.0 ** -10  # sqrt(Z)


@pytest.mark.parametrize("pow2", [True, False])
def test_example_6_1_outside(pow2):
    A = np.ones((2, 2))
    B = np.array([[Z, 1.0], [Z, 1.0]])
    sc = O.scale(A, B, "O", pow2=pow2)
    assert np.array_equal(sc.A, np.ones((2, 2)))
    assert np.array_equal(sc.B, np.ones((2, 2)))
    assert np.array_equal(sc.r, [1.0, 1.0]) and np.array_equal(sc.s, [Z, 1.0])
    Cp = O.fast(sc.A, sc.B, C.strassen(), 1)
    assert np.array_equal(Cp, 2 * np.ones((2, 2)))
    assert np.array_equal(sc.r[:, None] * Cp * sc.s[None, :], A @ B)


@pytest.mark.parametrize("pow2", [True, False])
def test_example_6_2_inside(pow2):
    A = np.array([[1.0, Z], [1.0, Z]])
    B = np.array([[Z, Z], [1.0, 1.0]])
    so = O.scale(A, B, "O", pow2=pow2)  # outside scaling is a no-op here
    assert np.array_equal(so.A, A) and np.array_equal(so.B, B)
    si = O.scale(A, B, "I", pow2=pow2)
    assert np.array_equal(si.factors[0][0], [SZ, 1.0 / SZ])
    assert np.array_equal(si.A, SZ * np.ones((2, 2)))
    assert np.array_equal(si.B, SZ * np.ones((2, 2)))


@pytest.mark.parametrize("pow2", [True, False])
def test_example_6_3_out_in_and_in_out(pow2):
    A = np.array([[1.0, 1.0 / Z], [1.0, 1.0]])
    B = np.array([[Z, 1.0], [Z, 1.0]])
    oi = O.scale(A, B, "OI", pow2=pow2)
    assert np.array_equal(oi.A, [[Z, 1.0], [1.0, 1.0]])
    assert np.array_equal(oi.B, np.ones((2, 2)))
    assert np.array_equal(oi.A @ oi.B, [[1 + Z, 1 + Z], [2.0, 2.0]])
    io = O.scale(A, B, "IO", pow2=pow2)
    assert np.array_equal(io.A, [[SZ, 1.0], [1.0, SZ]])
    assert np.array_equal(io.B, [[SZ, SZ], [1.0, 1.0]])
    # The (2,1) entry of C' is 2 z^{1/2} (the printed (1,1) entry "1 + z^{1/4}" is read as
    # 1 + z, which is what A' B' gives).
    assert np.array_equal(io.A @ io.B, [[1 + Z, 1 + Z], [2 * SZ, 2 * SZ]])
    for sc in (oi, io):
        Cp = O.fast(sc.A, sc.B, C.strassen(), 1)
        assert np.allclose(sc.r[:, None] * Cp * sc.s[None, :], A @ B, rtol=1e-15, atol=0)


@pytest.mark.parametrize("pow2", [True, False])
def test_example_6_4_in_out(pow2):
    A = np.array([[1.0, Z], [Z, Z]])
    B = np.array([[Z, 1.0], [1.0, 1.0 / Z]])
    io = O.scale(A, B, "IO", pow2=pow2)
    assert np.array_equal(io.A, [[1.0, 1.0], [Z, 1.0]])
    assert np.array_equal(io.B, np.ones((2, 2)))
    assert np.array_equal(io.A @ io.B, [[2.0, 2.0], [1 + Z, 1 + Z]])


@pytest.mark.parametrize("sched", ["O", "I", "OI", "IO", "OIOI"])
def test_example_6_5_scaling_is_a_no_op(sched):
    A = np.array([[1.0, Z], [Z, 1.0]])
    sc = O.scale(A, A.copy(), sched)
    assert np.array_equal(sc.A, A) and np.array_equal(sc.B, A)
    assert np.array_equal(sc.r, [1, 1]) and np.array_equal(sc.s, [1, 1])


def _lemma_d5(v):
    A = np.array([[1.0, 0.0], [1.0, 2.0 ** -(2 ** v)]])
    return A, np.eye(2)


@pytest.mark.parametrize("pow2", [True, False])
def test_lemma_d5_closed_form(pow2):
    # Starting with an O step (t0), for t = t0 + 2j: A^(t)_22 = 2^{-2^{v-j}},
    # s^(t)_2 = 2^{-2^v (1 - 2^{-j})}, B^(t) = I, r^(t) = 1; after the next I step
    # A_22 = B_22 = 2^{-2^{v-j-1}}.  Exact in both variants while the factors are powers of 2.
    v = 4
    A, B = _lemma_d5(v)
    for j in range(v):
        sc = O.scale(A, B, "OI" * j + "O", pow2=pow2)
        assert sc.A[1, 1] == 2.0 ** -(2 ** (v - j))
        assert sc.A[0, 0] == 1 and sc.A[1, 0] == 1 and sc.A[0, 1] == 0
        assert np.array_equal(sc.B, np.eye(2))
        assert np.array_equal(sc.r, [1.0, 1.0])
        assert sc.s[1] == 2.0 ** (-(2 ** v) * (1 - 2.0 ** -j))
        si = O.scale(A, B, "OI" * j + "OI", pow2=pow2)
        assert si.A[1, 1] == 2.0 ** -(2 ** (v - j - 1)) and si.B[1, 1] == 2.0 ** -(2 ** (v - j - 1))


def test_lemma_d5_linear_rate_one_half():
    # mu_22^(t) = 2^{2^{v-(t-t0)/2}} - 1 and mu^(t+2)/mu^(t) -> 1/2 (exact variant).
    v = 4
    A, B = _lemma_d5(v)
    limit = 2.0 ** -(2 ** v)  # r*_2 s*_2 ||A*|| ||B*||
    mus = []
    for j in range(v + 6):
        sc = O.scale(A, B, "OI" * j + "O", pow2=False)
        val = sc.r[1] * sc.s[1] * O.maxabs(sc.A) * O.maxabs(sc.B)
        mu = abs(val - limit) / limit
        assert mu == pytest.approx(2.0 ** (2.0 ** (v - j)) - 1, rel=1e-9)
        mus.append(mu)
    ratios = [mus[i + 1] / mus[i] for i in range(len(mus) - 1)]
    assert ratios[-1] == pytest.approx(0.5, abs=0.01)
    assert all(ratios[i + 1] >= ratios[i] - 1e-12 for i in range(len(ratios) - 1))


def test_stopping_criterion_guarantee_on_lemma_d5():
    # Stopping-criterion theorem (section 6.3): when the test passes after step t+1 (I) or t+2 (O), the relative distance
    # to the limit is at most tau.  Checked against the closed-form limit of Lemma D.5.
    v = 4
    A, B = _lemma_d5(v)
    limit = 2.0 ** -(2 ** v)
    for tau in (1.0, 0.1, 1e-3):
        sc = O.scale(A, B, "OI" * 40, tau=tau, pow2=False)
        assert sc.stopped_early
        val = sc.r[1] * sc.s[1] * O.maxabs(sc.A) * O.maxabs(sc.B)
        assert abs(val - limit) / limit <= tau * (1 + 1e-9)
        # the test is not vacuous: the iteration ran past the first O and I steps, and a
        # smaller tau needs more steps
        assert len(sc.steps) > 2
    n1 = len(O.scale(A, B, "OI" * 40, tau=1.0, pow2=False).steps)
    n2 = len(O.scale(A, B, "OI" * 40, tau=1e-3, pow2=False).steps)
    assert n2 > n1


def test_lemma_d1_invariants_and_monotonicity():
    A, B = badly_scaled(3, 24, 20, 28, span=4.0)
    sched = "OIOIOIOI"
    prev = None
    for t in range(1, len(sched) + 1):
        sc = O.scale(A, B, sched[:t], pow2=False)
        if sched[t - 1] == "O":
            assert O.maxabs(sc.A) == pytest.approx(1.0, rel=1e-15)
            assert O.maxabs(sc.B) == pytest.approx(1.0, rel=1e-15)
            assert np.allclose(np.max(np.abs(sc.A), axis=1), 1.0, rtol=1e-15)
        else:
            # after an I step every column of A' has the norm of the matching row of B'
            assert np.allclose(np.max(np.abs(sc.A), axis=0), np.max(np.abs(sc.B), axis=1), rtol=1e-14)
        cur = np.outer(sc.r, sc.s) * O.maxabs(sc.A) * O.maxabs(sc.B)
        if prev is not None:
            assert np.all(cur <= prev * (1 + 1e-13))
        prev = cur


def test_pow2_variant_is_exact_round_trip():
    A, B = badly_scaled(5, 33, 17, 21)
    sc = O.scale(A, B, "OIOI", pow2=True)
    # every factor is a power of two, so unscaling recovers the inputs bit for bit
    for x in list(sc.r) + list(sc.s) + list(sc.p):
        assert np.frexp(x)[0] == 0.5
    assert np.array_equal(sc.r[:, None] * sc.A / sc.p[None, :], A)
    assert np.array_equal(sc.p[:, None] * sc.B * sc.s[None, :], B)
    # the column factors of the I steps cancel between A' and B'
    Cref = A @ B
    Cs = sc.r[:, None] * (sc.A @ sc.B) * sc.s[None, :]
    assert np.allclose(Cs, Cref, rtol=1e-12, atol=0)
    # O step: scaled rows have max in (1/2, 1]
    so = O.scale(A, B, "O", pow2=True)
    rm = np.max(np.abs(so.A), axis=1)
    assert np.all((rm > 0.5) & (rm <= 1.0))


def test_pow2_round_ties_to_even_and_nearest():
    a = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 3.0, 1.0])
    b = np.array([2.0, 8.0, 4.0, 2.9, 3.0, 1.0, 0.5])
    # sqrt ratios: 1.414 (tie, log=1/2 -> 0), 2.83 (tie 3/2 -> 2), 2, 1.70 (log .77 -> 1),
    # 1.73 (.79 -> 1), 0.577 (-.79 -> -1), 0.707 (tie -1/2 -> 0)
    got = O.pow2_sqrt_ratio(b, a)
    assert np.array_equal(got, [1.0, 4.0, 2.0, 2.0, 2.0, 0.5, 1.0])
    assert np.array_equal(O.pow2_ceil(np.array([1.0, 0.75, 0.5, 3.0, 2.0 ** -30 * 1.5])),
                          [1.0, 1.0, 0.5, 4.0, 2.0 ** -29])


def test_zero_rows_and_columns_get_unit_factors():
    A = np.array([[0.0, 0.0], [2.0, 4.0]])
    B = np.array([[0.0, 3.0], [0.0, 5.0]])
    sc = O.scale(A, B, "OI")
    assert sc.r[0] == 1.0 and sc.s[0] == 1.0
    Cs = sc.r[:, None] * O.fast(sc.A, sc.B, C.strassen(), 1) * sc.s[None, :]
    assert np.array_equal(Cs, A @ B)


def test_scaling_improves_componentwise_error_on_example_6_1_pattern():
    # Section 6.1: columns of B far smaller than the rest give O(eps/z) relative errors in
    # those columns of C without scaling, and O(eps) with outside scaling.  Random entries
    # stand in for the small independent perturbations the paper mentions.
    from synth import make_pair

    n = 64
    A, B = make_pair("uniform01", 8, n, n, n)
    A = A + 1.0
    B[:, : n // 2] *= 2.0 ** -40
    ref = O.reference_rows(A, B)
    e_none = O.componentwise_error(O.fast(A, B, C.strassen(), 3), ref)
    e_out = O.componentwise_error(O.scaled_fast(A, B, C.strassen(), 3, mode="outside"), ref)
    assert e_out < 1e-13 < e_none


# ---- scaling at every level (a reading: the paper scales once; here every inner node of the
# recursion runs the same steps on its own operands and unscales its product)

@pytest.mark.parametrize("mode,steps", [("outside", 2), ("inside", 2), ("out_in", 2), ("repeated", 4)])
@pytest.mark.parametrize("rules,shape", [((C.strassen(),) * 2, (24, 20, 28)), ((C.strassen(),) * 3, (32, 16, 40)),
                                         ((C.f323(), C.strassen()), (30, 14, 27))])
def test_every_level_scaling_is_exact_on_dyadic_inputs(mode, steps, rules, shape):
    A, B = dyadic_pair(5, *shape)
    got = O.scaled_fast_every_level(A, B, list(rules), 1, mode, steps)
    assert np.array_equal(got, exact_product(A, B))


@pytest.mark.parametrize("mode,steps", [("outside", 2), ("out_in", 2), ("in_out", 2), ("repeated", 20)])
def test_every_level_scaling_at_depth_one_is_scaling_once(mode, steps):
    A, B = badly_scaled(7, 22, 18, 26)
    once = O.scaled_fast(A, B, C.strassen(), 1, 1, mode, steps)
    every = O.scaled_fast_every_level(A, B, [C.strassen()], 1, mode, steps)
    assert np.array_equal(once, every)


@pytest.mark.parametrize("sched_mode", ["outside", "out_in", "repeated"])
def test_every_inner_node_is_scaled(sched_mode):
    # depth 3 Strassen: 1 + 7 + 49 inner nodes, visited depth first; after the node's last O
    # step its operands have row (A) and column (B) maxima in (1/2, 1] (zero lines excepted);
    # after a last I step every column of the node's A' has the maximum of the matching row
    # of B' to within a factor 2 (power-of-two factors, Lemma D.5)
    A, B = badly_scaled(9, 40, 48, 56)
    trace = []
    O.scaled_fast_every_level(A, B, [C.strassen()] * 3, 1, sched_mode, 3, trace=trace)
    assert [lv for lv, _ in trace].count(0) == 1
    assert [lv for lv, _ in trace].count(1) == 7
    assert [lv for lv, _ in trace].count(2) == 49
    assert [lv for lv, _ in trace][:3] == [0, 1, 2]
    for lv, sc in trace:
        assert sc.A.shape == (40 // 2 ** lv, 48 // 2 ** lv) and sc.B.shape == (48 // 2 ** lv, 56 // 2 ** lv)
        if sc.steps[-1] == "O":
            for mx in (np.max(np.abs(sc.A), axis=1), np.max(np.abs(sc.B), axis=0)):
                nz = mx[mx > 0]
                assert np.all((nz > 0.5) & (nz <= 1.0))
        else:
            ca, rb = np.max(np.abs(sc.A), axis=0), np.max(np.abs(sc.B), axis=1)
            ok = (ca > 0) & (rb > 0)
            ratio = ca[ok] / rb[ok]
            assert np.all((ratio >= 0.5) & (ratio <= 2.0))


def test_every_level_scaling_with_cutoff_and_no_levels():
    A, B = badly_scaled(11, 20, 12, 18)
    # cutoff 8 stops Strassen after one level on k = 12 (12/2 = 6 < 8 at the first level)
    assert O.effective_depth(20, 12, 18, [(2, 2, 2)] * 3, 8) == 0
    got = O.scaled_fast_every_level(A, B, [C.strassen()] * 3, 8, "out_in")
    sc = O.scale(A, B, "OI")
    want = (sc.r[:, None] * O.classical(sc.A, sc.B)) * sc.s[None, :]
    assert np.array_equal(got, want)
    ref = O.reference_rows(A, B)
    assert O.componentwise_error(got, ref) < 1e-13


def test_pow2_nearest_hand_values_and_boundary():
    from fractions import Fraction

    above = float.fromhex("0x1.6a09e667f3bcdp-1")  # smallest double above 2^-1/2
    below = float(np.nextafter(above, 0.0))
    assert Fraction(below) ** 2 < Fraction(1, 2) < Fraction(above) ** 2  # exact
    x = np.array([1.0, 0.75, 0.7, 3.0, 2.8, 1.5, 1.4, above, below, 4.0 * above, 4.0 * below, 2.0 ** -30 * 1.5])
    want = [1.0, 1.0, 0.5, 4.0, 2.0, 2.0, 1.0, 1.0, 0.5, 4.0, 2.0, 2.0 ** -29]
    assert np.array_equal(O.pow2_nearest(x), want)


def test_pow2_nearest_against_log2_rounding():
    """Brute force over many magnitudes, away from the half-way points where float log2 could
    round either way."""
    rng = np.random.default_rng(11)
    x = 2.0 ** rng.uniform(-60, 60, 20000)
    l2 = np.log2(x)
    keep = np.abs(l2 - np.floor(l2) - 0.5) > 1e-9
    assert np.array_equal(O.pow2_nearest(x[keep]), 2.0 ** np.round(l2[keep]))


def test_outside_nearest_rounding_range_and_exact_round_trip():
    A, B = badly_scaled(6, 40, 24, 36)
    so = O.scale(A, B, "O", pow2=True, o_round="nearest")
    rm = np.max(np.abs(so.A), axis=1)
    cm = np.max(np.abs(so.B), axis=0)
    for m_ in (rm, cm):
        assert np.all((m_ >= 2.0 ** -0.5) & (m_ < 2.0 ** 0.5))
    for x in list(so.r) + list(so.s):
        assert np.frexp(x)[0] == 0.5
    assert np.array_equal(so.r[:, None] * so.A, A)
    assert np.array_equal(so.B * so.s[None, :], B)
    # exact on dyadic inputs through a fast rule, like the other rounding
    Ad, Bd = dyadic_pair(3, 48, 40, 56)
    got = O.scaled_fast(Ad, Bd, C.strassen(), 2, 1, "out_in", o_round="nearest")
    assert np.array_equal(got, exact_product(Ad, Bd))


def test_outside_rounding_and_the_cancelling_terms():
    """Why the O-step rounding matters for a fast rule: rows whose maxima straddle a rounding
    boundary get factors a ratio 2 apart, and Strassen's cancelling cross-block terms (e.g. the
    A22 terms of M1 and M4 in C11) then carry rounding errors up to twice their unscaled size
    after the product is unscaled.  Row and column maxima spread over [3, 5]: rounding up
    splits them at 4 (factors 4 and 8); the nearest power of two puts them all on 4 (the
    boundaries are 2^1.5 and 2^2.5), a uniform exact scaling, so the error equals the unscaled
    one.  FP32 arithmetic, Strassen depth 2, n = 256."""
    n = 256
    errs = {"none": [], "up": [], "nearest": []}
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        A = rng.standard_normal((n, n))
        B = rng.standard_normal((n, n))
        A = (A / np.abs(A).max(1)[:, None] * rng.uniform(3, 5, n)[:, None]).astype(np.float32)
        B = (B / np.abs(B).max(0)[None, :] * rng.uniform(3, 5, n)[None, :]).astype(np.float32)
        A64, B64 = A.astype(np.float64), B.astype(np.float64)
        ref = O.reference_rows(A64, B64)
        err = lambda X: O.normwise_error(X.astype(np.float64), ref, A64, B64)
        errs["none"].append(err(O.fast(A, B, C.strassen(), 2)))
        for r in ("up", "nearest"):
            errs[r].append(err(O.scaled_fast(A, B, C.strassen(), 2, 1, "outside", o_round=r)))
    assert errs["nearest"] == errs["none"]
    assert np.mean(errs["up"]) >= 1.4 * np.mean(errs["none"])
