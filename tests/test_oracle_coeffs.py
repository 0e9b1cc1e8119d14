"""Pins for the oracle's coefficient tables and principal quantities (sections 3.1, 4.1, 5.2,
Table 1, Examples 4.1-4.3, Appendices A-C).  CPU only."""
import os
from fractions import Fraction

import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(fname):
    out = []
    for line in open(os.path.join(GOLD, fname)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


@pytest.mark.parametrize("name", sorted(C.ALGORITHMS))
def test_brent_equations_hold(name):
    # Eq. (1) computes C = AB for all A, B iff the trilinear tensor of [U,V,W] equals the
    # matrix-multiplication tensor under the stated index conventions (section 3.1).
    assert C.brent_violations(C.get(name)) == 0


def test_printed_tables_need_relabelling():
    # Appendix A as printed is an algorithm only with A, B row-major and C column-major.
    sp = C.strassen_as_printed()
    assert C.brent_violations(sp) > 0
    assert C.brent_violations(sp, ("row", "row", "col")) == 0
    # Appendix C as printed fails under every pure row/column-major convention.
    fp = C.f442_as_printed()
    for conv in [(a, b, c) for a in ("row", "col") for b in ("row", "col") for c in ("row", "col")]:
        assert C.brent_violations(fp, conv) > 0


def test_a_wrong_sign_breaks_brent():
    # The check is sensitive to a single flipped coefficient.
    alg = C.strassen()
    alg.W[0][0] = -alg.W[0][0]
    assert C.brent_violations(alg) > 0


@pytest.mark.parametrize("row", _rows("table1.txt"), ids=lambda r: r[0])
def test_table1_quantities(row):
    key, M0, K0, N0, R, nnz, Q, E = row[:8]
    alg = C.get(key)
    q = C.quantities(alg)
    assert (alg.M0, alg.K0, alg.N0, alg.R) == (int(M0), int(K0), int(N0), int(R))
    assert q.nnz == int(nnz)
    assert q.Q == Fraction(Q)
    assert q.E == Fraction(E)


@pytest.mark.parametrize("row", _rows("stability_vectors.txt"), ids=lambda r: r[0])
def test_stability_vectors(row):
    key, order, vals = row[0], row[1], [Fraction(x) for x in row[2:-1]]
    alg = C.get(key)
    e = C.quantities(alg).e
    if order == "col-major":
        e = [e[p * alg.N0 + s] for s in range(alg.N0) for p in range(alg.M0)]
    assert e == vals


def test_example_4_1_structure_only_factor():
    gold = {r[0]: Fraction(r[1]) for r in _rows("two_level_E.txt")}
    assert C.quantities(C.f442()).E == 89
    assert C.structure_only_E(C.f442()) == gold["f442_structure_only_E"]


def test_rotation_244_factor_and_rotation_invariants():
    gold = {r[0]: Fraction(r[1]) for r in _rows("two_level_E.txt")}
    assert C.quantities(C.f244()).E == gold["f244_plain_rotation_E"]
    # Strassen is cyclic-invariant (Appendix A): rotations keep Q and E.
    s = C.strassen()
    for a in (C.rotate(s), C.rotate(C.rotate(s))):
        q = C.quantities(a)
        assert (q.Q, q.E) == (8, 12)
        assert C.brent_violations(a) == 0


def test_two_level_stationary_E_is_square():
    gold = {r[0]: Fraction(r[1]) for r in _rows("two_level_E.txt")}
    assert max(O.stationary_stability_vector(C.strassen(), 2)) == gold["strassen_stationary"]
    assert max(O.stationary_stability_vector(C.f323(), 2)) == gold["f323_stationary"]


def _swap2():
    return [[0, 1], [1, 0]]


def _eye(n):
    return [[1 if i == j else 0 for j in range(n)] for i in range(n)]


def test_example_4_2_dalberto_nonuniform():
    # [U, (P x I) V, (I x P) W] at nodes [2,1], [2,3], [2,4]; original elsewhere.
    gold = {r[0]: Fraction(r[1]) for r in _rows("two_level_E.txt")}
    s = C.strassen()
    P = _swap2()
    var = C.kron_perm_variant(s, list(range(4)), C.kron_index_perm(P, _eye(2)),
                              C.kron_index_perm(_eye(2), P), "dalberto")
    assert C.brent_violations(var) == 0
    nodes = {0, 2, 3}  # 1-based r1 = 1, 3, 4
    xi = O.nonuniform_two_level_xi(s, lambda r1: var if r1 in nodes else s)
    assert max(xi) == gold["strassen_dalberto_nonuniform"]
    # With the original rule everywhere the formula reduces to the stationary e (x) e.
    xi0 = O.nonuniform_two_level_xi(s, lambda r1: s)
    assert xi0 == O.stationary_stability_vector(s, 2)


def test_example_4_3_f323_nonuniform():
    gold = {r[0]: Fraction(r[1]) for r in _rows("two_level_E.txt")}
    a = C.f323()
    P1 = [[1, 0, 0], [0, 0, 1], [0, 1, 0]]
    P2 = [[0, 1, 0], [0, 0, 1], [1, 0, 0]]

    def variant(P, name):
        return C.kron_perm_variant(a, C.kron_index_perm(_eye(2), P), C.kron_index_perm(P, _eye(2)),
                                   C.kron_index_perm(P, P), name)

    v1, v2 = variant(P1, "v1"), variant(P2, "v2")
    assert C.brent_violations(v1) == 0 and C.brent_violations(v2) == 0
    n1 = {r - 1 for r in (1, 3, 10, 11)}
    n2 = {r - 1 for r in (4, 5, 7, 9, 12, 13)}
    xi = O.nonuniform_two_level_xi(a, lambda r1: v1 if r1 in n1 else (v2 if r1 in n2 else a))
    assert max(xi) == gold["f323_nonuniform_3variants"]


def test_winograd_flat_quantities():
    # Not printed in the paper; the paper says its stability factor is slightly larger than
    # Strassen's (Example 4.2).  Flat-form values by Definitions 4.1/4.2.
    q = C.quantities(C.winograd())
    assert (q.nnz, q.Q, q.E) == (42, 10, 18)
    assert q.E > C.quantities(C.strassen()).E


def test_classical_rule_quantities_match_table1_for_any_base():
    # The classical <2,2,2> row of Table 1 (Q=4, E=2) and its general form Q = 2 + K0,
    # E = K0 per output entry for <M0,K0,N0> with R = M0 K0 N0.
    for (m0, k0, n0) in [(2, 2, 2), (3, 2, 3), (2, 3, 4)]:
        q = C.quantities(C.classical(m0, k0, n0))
        assert q.E == k0
        assert q.Q == k0 + 2
        assert C.brent_violations(C.classical(m0, k0, n0)) == 0
