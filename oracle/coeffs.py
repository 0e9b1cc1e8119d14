"""Oracle: bilinear base-case algorithms [U, V, W] in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY. Nothing under oracle/ is part of the product path; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.

Conventions (section 3.1, eq. (1)): U is M0K0 x R, V is K0N0 x R, W is M0N0 x R, and
    C_k = sum_r W[k,r] * (sum_i U[i,r] A_i) * (sum_j V[j,r] B_j).
Single indices of A (M0 x K0) and B (K0 x N0) are column-major, single indices of C
(M0 x N0) are row-major.  All indices in this module are 0-based:
    A entry (p, q) <-> i = p + q*M0,   B entry (q, s) <-> j = q + s*K0,
    C entry (p, s) <-> k = p*N0 + s.

Tables are given as printed in the paper's appendices (rows in printed order), followed by
the row relabelling that makes each one satisfy the Brent equations under the convention
above.  The relabellings only permute rows, so nnz, Q and E (Table 1) are unchanged:
  * Strassen (Appendix A): the printed table is valid with A and B row-major and C
    column-major; swapping rows 2 and 3 (1-based) of U, V and W converts it.
  * <3,2,3;15> (Appendix B): valid as printed.
  * <4,4,2;26> (Appendix C): U as printed; V takes printed rows [1,5,2,6,3,7,4,8] and W takes
    printed rows [1,3,5,7,2,4,6,8] (1-based).
Coefficients not printed in the paper come from the literature and are pinned only by the
Brent equations: Winograd's variant of Strassen's algorithm (the 7-product, 15-addition
form) and Laderman's rank-23 algorithm for <3,3,3> (a stand-in: Smirnov's rank-23 table
that the paper's Table 1 row refers to is not printed).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Sequence


Matrix = List[List[Fraction]]


@dataclass
class Bilinear:
    """One base-case rule <M0,K0,N0;R> given by exact [U, V, W]."""

    name: str
    M0: int
    K0: int
    N0: int
    U: Matrix
    V: Matrix
    W: Matrix
    notes: str = field(default="")

    @property
    def R(self) -> int:
        return len(self.U[0])

    def as_float(self):
        import numpy as np

        return (
            np.array([[float(x) for x in row] for row in self.U]),
            np.array([[float(x) for x in row] for row in self.V]),
            np.array([[float(x) for x in row] for row in self.W]),
        )


def _parse(text: str, den: int = 1) -> Matrix:
    rows = []
    for line in text.strip().splitlines():
        line = line.strip()
        if not line:
            continue
        rows.append([Fraction(int(tok), den) for tok in line.split()])
    width = {len(r) for r in rows}
    assert len(width) == 1, "ragged table"
    return rows


def _permute_rows(mat: Matrix, order_1based: Sequence[int]) -> Matrix:
    return [list(mat[i - 1]) for i in order_1based]


# ---------------------------------------------------------------- Appendix A (as printed)
_STRASSEN_U = """
 1  0  1  0  1 -1  0
 0  0  0  0  1  0  1
 0  1  0  0  0  1  0
 1  1  0  1  0  0 -1
"""
_STRASSEN_V = """
 1  1  0 -1  0  1  0
 0  0  1  0  0  1  0
 0  0  0  1  0  0  1
 1  0 -1  0  1  0  1
"""
_STRASSEN_W = """
 1  0  0  1 -1  0  1
 0  1  0  1  0  0  0
 0  0  1  0  1  0  0
 1 -1  1  0  0  1  0
"""

# ---------------------------------------------------------------- Appendix B (as printed)
_F323_U = """
 0  1  0  0 -1  1  1  0  0  0 -1  0  0  0 -1
 0  1  0  0  0  0  0 -1  0 -1  0  0  1 -1  0
 0  0  0  1  0  0  0 -1  0 -1  1  0  0 -1  0
-1  0  1  0  1  0  0  0  0  0  1  0  0  0  1
-1  0  0  0  0  1  0  1  0  1  0  1 -1  0  0
 0  0 -1  0  0  0  0  1  1  0 -1  0  0  0 -1
"""
_F323_V = """
 0  0  1  1  0  0  0  0  0  0  1  0  0  1  1
 0  0  1  0  0  0  0 -1  1 -1  0  0  0  1  0
 0 -1  0  0  0  1  0  0  0  1  0  1  1 -1  0
-1  0  0  0  0  0  0  1  0  1  0  1  0 -1  0
 0  1  1  0  0  0  1  0  0  0  1  0  0  0  1
 1  0  1  0  1  1  1  0  0  0  0  0  0  0  1
"""
_F323_W = """
 0  0  1  0  0  0 -1  0  1  0  0  0  0  0 -1
 1  0  0  0  1  1  0  0  0  0  0 -1  0  0  0
 0  0  0  0  1  0  1  0  0  0  0  0  0  0  0
 0  0  0 -1  0  0  0  0  0 -1  0  1  0 -1  0
 0  0  0  0  0  0  0  0  0  0  0  1  1  0  0
 0  1  0  0  0  1 -1  0  0  0  0  0  1  0  0
 0  0  0  1  0  0  0  0  1  0  0  0  0  0  0
 0  0  0  0  0  0  0  1  1 -1  0  0 -1  0  0
 0  0  0 -1  1  0  0  0  0  0  1  0  0  0 -1
"""

# ---------------------------------------------------------------- Appendix C (as printed)
# U and V are printed as (1/2) * integer matrix; W has integer entries.
_F442_U2 = """
 2  0  0 -2  0  0  0  0 -2  0  0  0  0 -2  0  0  0  0  0  0  0  0  0  0  0  0
 0  0  0  0  0 -2  0  0  0  0  2  2  2  0  0  0  0  0  0  0  0  0  0  0  0  0
 0  0  2  0  0 -2  0  0  0  0  2  2  2 -2  0  0  0  0  0  0 -2  0  0  2  0  0
 0  0  0  0  0  0  0  0  0  0  0 -2  0  2  0  0  0  0  0  0  0  0  0  0  0  0
 0  2  0  0  0  0  0  1  0  0  0  0  0  0  0  0  0  0 -1  0  0  0  0  0  0  2
 0  2  0  0  0  0  0  0  0  0  0  0 -2  0  0  1  0  0  0  1  0 -2  0  2 -2  0
 0  2  0  0  0  0  0  1  0  0  0  0  0  0  0  0  0  0 -1  0  0 -2  0  0  0  0
 0  0  0  1  2  0 -1 -1  0 -1 -2  2  0 -2 -2  0  0  1  0  0  1  0  0  0  0  0
 0  0  0  0  0  0  0  1  0  0  0  0  0  0  0 -1  1  1  0  0  0  0  0  0  0  0
 0  2  0  0 -2  0  0  0  0  0  0  0  0  0  0  1  0  0  0  1  0 -2  2  0  2  0
 0  2  0  0 -2  0  0  1  0  0  0  0  0  0  0  0  0  1  0  0  0 -2  2  0  2  0
 0  0  0  1  0  0 -1 -1  0  1  0  0  0  0  0  0  0 -1  0  0 -1  0  0  0  0  0
 0 -2  0  0  0  0  0  0  2  0  0  0  0  0  0  1 -1 -1  1  0  0  0  0  0  0 -2
 0  0  0  0  2  0  0  0  0  0  0  0  2  0  0  0  0  0  0  0  0  0  0  0  0  0
 0  0  0  0  2  0  0  0  0  0  0  0  0  0  0  0  0 -1  1  0  0  0  0  0 -2  0
 0  0  0  0 -2  0  0  0  0  0  2  0  0  2  2  0  0  0  0  0  0  0  0  0  0  0
"""
_F442_V2 = """
 2  0 -2  0  0 -2  0  0  0  0 -2  0  0 -2 -2  0  0  0  0  0  0  0  0  0  0  0
 2  1  2  2  0  0  0  2  2  0  0  0  0  0  0  0  2 -2 -2  2  2  0  0 -2  1  0
-2  0 -2 -2  0 -2 -2  0  0 -2  0 -2  0  0  0  0  0  0  0  0 -2  0  0  0  0  0
-2  0  2 -2  0  0 -2  0 -2  2  0  0  0  0  0 -2 -2  0  0  2  2  0 -2 -2  0  0
 2  1 -2  2  0  0  0  2  2  0  0  0  0  0  0  2  0  2  2  0 -2  0  0  2 -1  2
 2  1 -2  2  0  2  0  2  2  0  2  0 -2  0  2  2  0  2 -2  0 -2  0  0  2 -1  0
-2 -2 -2 -2  0  0 -2  0 -2 -2  0  0  0  0  0  0  0  0  0  0 -2  2  2  2  0 -2
-2  0 -2 -2 -2  2 -2  0 -2 -2  2  0 -2  0  0  0  0  0  0  0 -2  0 -2  2 -2  0
"""
_F442_W = """
 1 -1  0  1  0  0  1  1  0  0  0  0  0  0  0  1  1  0  0  1  0  1  0  0  0  1
 0  1 -1  0  0  0  0  0  0 -1  0  0  0  0  0 -1 -1 -1 -1 -1 -1 -1  0  0  0 -1
 0 -1  0  1  0  0  1  1 -1  0  0  0  0  0  0  1 -1  0  0  1  0  1  0  0  0  0
 0  0  0  0  0  0  0  0  0  1  0  0  0  0  0  1  1  1  0 -1  1 -1 -1 -1  1  0
 0  0  1  0  1  0  0  0  0  1 -1  0 -1  0  1  1  1  1  0  1  1  0  0  0  1  0
 1  0 -1  1  0  0  1  0  0 -1  0  0  0 -1  1  0  0  0  0  0 -1  0  0  0  0  0
 0  0  0  0 -1  1  0  0  0 -1  1  0  0  0 -1 -1 -1 -1  0  1 -1  0  0  1 -1  0
 0  0  0  0  0  1  1  0  0  1  1  1  0  0 -1  0  0  0  0  0  0  0  0  0  0  0
"""


def strassen_as_printed() -> Bilinear:
    return Bilinear("strassen_printed", 2, 2, 2, _parse(_STRASSEN_U), _parse(_STRASSEN_V),
                    _parse(_STRASSEN_W), "Appendix A exactly as printed")


def strassen() -> Bilinear:
    p = strassen_as_printed()
    order = [1, 3, 2, 4]
    return Bilinear("strassen", 2, 2, 2, _permute_rows(p.U, order), _permute_rows(p.V, order),
                    _permute_rows(p.W, order), "Appendix A, rows 2 and 3 swapped")


def f323() -> Bilinear:
    return Bilinear("f323", 3, 2, 3, _parse(_F323_U), _parse(_F323_V), _parse(_F323_W),
                    "Appendix B as printed")


def f442_as_printed() -> Bilinear:
    return Bilinear("f442_printed", 4, 4, 2, _parse(_F442_U2, 2), _parse(_F442_V2, 2),
                    _parse(_F442_W), "Appendix C exactly as printed")


def f442() -> Bilinear:
    p = f442_as_printed()
    return Bilinear("f442", 4, 4, 2, [list(r) for r in p.U],
                    _permute_rows(p.V, [1, 5, 2, 6, 3, 7, 4, 8]),
                    _permute_rows(p.W, [1, 3, 5, 7, 2, 4, 6, 8]),
                    "Appendix C with V and W rows relabelled")


def rotate(alg: Bilinear, name: str | None = None) -> Bilinear:
    """[U,V,W] for <M0,K0,N0> -> [W,U,V], an algorithm for <N0,M0,K0> (cyclic rotation of the
    trilinear form; the stated index conventions make the relabelling the identity)."""
    return Bilinear(name or f"rot({alg.name})", alg.N0, alg.M0, alg.K0,
                    [list(r) for r in alg.W], [list(r) for r in alg.U], [list(r) for r in alg.V],
                    f"[W,U,V] of {alg.name}")


def f424() -> Bilinear:
    """<4,2,4;26>: the rotation [V,W,U] of the (relabelled) Appendix C algorithm."""
    return rotate(rotate(f442()), "f424")


def f244() -> Bilinear:
    """<2,4,4;26>: the rotation [W,U,V] of the (relabelled) Appendix C algorithm."""
    return rotate(f442(), "f244")


def classical(M0: int, K0: int, N0: int) -> Bilinear:
    """The classical rule: one product per (p, q, s), R = M0*K0*N0."""
    R = M0 * K0 * N0
    U = [[Fraction(0)] * R for _ in range(M0 * K0)]
    V = [[Fraction(0)] * R for _ in range(K0 * N0)]
    W = [[Fraction(0)] * R for _ in range(M0 * N0)]
    r = 0
    for p in range(M0):
        for s in range(N0):
            for q in range(K0):
                U[p + q * M0][r] = Fraction(1)
                V[q + s * K0][r] = Fraction(1)
                W[p * N0 + s][r] = Fraction(1)
                r += 1
    return Bilinear(f"classical{M0}{K0}{N0}", M0, K0, N0, U, V, W, "classical")


def _from_products(name, M0, K0, N0, products, outputs, notes) -> Bilinear:
    """Build [U,V,W] from named block expressions.

    products: list of (dict A-entry->coef, dict B-entry->coef) with entries like 'a12' (1-based
    row/col); outputs: dict 'c12' -> dict product-index(1-based)->coef.
    """
    R = len(products)
    U = [[Fraction(0)] * R for _ in range(M0 * K0)]
    V = [[Fraction(0)] * R for _ in range(K0 * N0)]
    W = [[Fraction(0)] * R for _ in range(M0 * N0)]
    for r, (sa, tb) in enumerate(products):
        for ent, c in sa.items():
            p, q = int(ent[1]) - 1, int(ent[2]) - 1
            U[p + q * M0][r] += Fraction(c)
        for ent, c in tb.items():
            q, s = int(ent[1]) - 1, int(ent[2]) - 1
            V[q + s * K0][r] += Fraction(c)
    for ent, terms in outputs.items():
        p, s = int(ent[1]) - 1, int(ent[2]) - 1
        for r1, c in terms.items():
            W[p * N0 + s][r1 - 1] += Fraction(c)
    return Bilinear(name, M0, K0, N0, U, V, W, notes)


def winograd() -> Bilinear:
    """Winograd's variant of Strassen's algorithm written out as a flat bilinear algorithm.

    With s1 = a21+a22, s2 = s1-a11, s3 = a11-a21, s4 = a12-s2, t1 = b12-b11, t2 = b22-t1,
    t3 = b22-b12, t4 = t2-b21 the products are p1 = a11 b11, p2 = a12 b21, p3 = s4 b22,
    p4 = a22 t4, p5 = s1 t1, p6 = s2 t2, p7 = s3 t3, and
    c11 = p1+p2, c12 = p1+p6+p5+p3, c21 = p1+p6+p7-p4, c22 = p1+p6+p7+p5.
    """
    products = [
        ({"a11": 1}, {"b11": 1}),
        ({"a12": 1}, {"b21": 1}),
        ({"a11": 1, "a12": 1, "a21": -1, "a22": -1}, {"b22": 1}),
        ({"a22": 1}, {"b11": 1, "b12": -1, "b21": -1, "b22": 1}),
        ({"a21": 1, "a22": 1}, {"b12": 1, "b11": -1}),
        ({"a21": 1, "a22": 1, "a11": -1}, {"b22": 1, "b12": -1, "b11": 1}),
        ({"a11": 1, "a21": -1}, {"b22": 1, "b12": -1}),
    ]
    outputs = {
        "c11": {1: 1, 2: 1},
        "c12": {1: 1, 6: 1, 5: 1, 3: 1},
        "c21": {1: 1, 6: 1, 7: 1, 4: -1},
        "c22": {1: 1, 6: 1, 7: 1, 5: 1},
    }
    return _from_products("winograd", 2, 2, 2, products, outputs,
                          "Winograd's variant (literature; not printed in the paper)")


def laderman333() -> Bilinear:
    """Laderman's rank-23 algorithm for <3,3,3> (J. Laderman, Bull. AMS 82, 1976)."""
    P = [
        ({"a11": 1, "a12": 1, "a13": 1, "a21": -1, "a22": -1, "a32": -1, "a33": -1}, {"b22": 1}),
        ({"a11": 1, "a21": -1}, {"b12": -1, "b22": 1}),
        ({"a22": 1}, {"b11": -1, "b12": 1, "b21": 1, "b22": -1, "b23": -1, "b31": -1, "b33": 1}),
        ({"a11": -1, "a21": 1, "a22": 1}, {"b11": 1, "b12": -1, "b22": 1}),
        ({"a21": 1, "a22": 1}, {"b11": -1, "b12": 1}),
        ({"a11": 1}, {"b11": 1}),
        ({"a11": -1, "a31": 1, "a32": 1}, {"b11": 1, "b13": -1, "b23": 1}),
        ({"a11": -1, "a31": 1}, {"b13": 1, "b23": -1}),
        ({"a31": 1, "a32": 1}, {"b11": -1, "b13": 1}),
        ({"a11": 1, "a12": 1, "a13": 1, "a22": -1, "a23": -1, "a31": -1, "a32": -1}, {"b23": 1}),
        ({"a32": 1}, {"b11": -1, "b13": 1, "b21": 1, "b22": -1, "b23": -1, "b31": -1, "b32": 1}),
        ({"a13": -1, "a32": 1, "a33": 1}, {"b22": 1, "b31": 1, "b32": -1}),
        ({"a13": 1, "a33": -1}, {"b22": 1, "b32": -1}),
        ({"a13": 1}, {"b31": 1}),
        ({"a32": 1, "a33": 1}, {"b31": -1, "b32": 1}),
        ({"a13": -1, "a22": 1, "a23": 1}, {"b23": 1, "b31": 1, "b33": -1}),
        ({"a13": 1, "a23": -1}, {"b23": 1, "b33": -1}),
        ({"a22": 1, "a23": 1}, {"b31": -1, "b33": 1}),
        ({"a12": 1}, {"b21": 1}),
        ({"a23": 1}, {"b32": 1}),
        ({"a21": 1}, {"b13": 1}),
        ({"a31": 1}, {"b12": 1}),
        ({"a33": 1}, {"b33": 1}),
    ]
    out = {
        "c11": {6: 1, 14: 1, 19: 1},
        "c12": {1: 1, 4: 1, 5: 1, 6: 1, 12: 1, 14: 1, 15: 1},
        "c13": {6: 1, 7: 1, 9: 1, 10: 1, 14: 1, 16: 1, 18: 1},
        "c21": {2: 1, 3: 1, 4: 1, 6: 1, 14: 1, 16: 1, 17: 1},
        "c22": {2: 1, 4: 1, 5: 1, 6: 1, 20: 1},
        "c23": {14: 1, 16: 1, 17: 1, 18: 1, 21: 1},
        "c31": {6: 1, 7: 1, 8: 1, 11: 1, 12: 1, 13: 1, 14: 1},
        "c32": {12: 1, 13: 1, 14: 1, 15: 1, 22: 1},
        "c33": {6: 1, 7: 1, 8: 1, 9: 1, 23: 1},
    }
    return _from_products("laderman333", 3, 3, 3, P, out,
                          "Laderman 1976 (stand-in for the unprinted Smirnov <3,3,3;23>)")


# ------------------------------------------------------------------------ exact algebra
def brent_violations(alg: Bilinear, conv=("col", "col", "row")) -> int:
    """Number of (a, b, c) triples where sum_r U[a,r] V[b,r] W[c,r] differs from the
    matrix-multiplication tensor delta(p=p') delta(q=q') delta(s=s')."""
    M0, K0, N0, R = alg.M0, alg.K0, alg.N0, alg.R

    def ia(p, q):
        return p + q * M0 if conv[0] == "col" else p * K0 + q

    def ib(q, s):
        return q + s * K0 if conv[1] == "col" else q * N0 + s

    def ic(p, s):
        return p * N0 + s if conv[2] == "row" else p + s * M0

    bad = 0
    for p in range(M0):
        for q in range(K0):
            for q2 in range(K0):
                for s in range(N0):
                    for p2 in range(M0):
                        for s2 in range(N0):
                            a, b, c = ia(p, q), ib(q2, s), ic(p2, s2)
                            t = sum((alg.U[a][r] * alg.V[b][r] * alg.W[c][r] for r in range(R)),
                                    Fraction(0))
                            want = 1 if (p == p2 and q == q2 and s == s2) else 0
                            if t != want:
                                bad += 1
    return bad


@dataclass
class Quantities:
    nnz: int
    alpha: list
    beta: list
    gamma: list
    a: list
    b: list
    q: list
    e: list
    Q: Fraction
    E: Fraction


def quantities(alg: Bilinear) -> Quantities:
    """Principal quantities of section 4.1: eqs. (abg), (ab), Definitions 4.1 and 4.2."""
    R = alg.R
    alpha = [sum(1 for i in range(len(alg.U)) if alg.U[i][r] != 0) for r in range(R)]
    beta = [sum(1 for j in range(len(alg.V)) if alg.V[j][r] != 0) for r in range(R)]
    gamma = [sum(1 for r in range(R) if alg.W[k][r] != 0) for k in range(len(alg.W))]
    a = [sum((abs(alg.U[i][r]) for i in range(len(alg.U))), Fraction(0)) for r in range(R)]
    b = [sum((abs(alg.V[j][r]) for j in range(len(alg.V))), Fraction(0)) for r in range(R)]
    q = []
    e = []
    for k in range(len(alg.W)):
        mx = max([alpha[r] + beta[r] for r in range(R) if alg.W[k][r] != 0], default=0)
        q.append(gamma[k] + mx)
        e.append(sum((a[r] * b[r] * abs(alg.W[k][r]) for r in range(R)), Fraction(0)))
    nnz = sum(alpha) + sum(beta) + sum(gamma)
    return Quantities(nnz, alpha, beta, gamma, a, b, q, e, Fraction(max(q)), max(e))


def structure_only_E(alg: Bilinear) -> int:
    """The earlier (Bini-Lotti style) stability factor that sees only the nonzero structure:
    max_k sum_r alpha_r beta_r [W_kr != 0]."""
    qt = quantities(alg)
    return max(sum(qt.alpha[r] * qt.beta[r] for r in range(alg.R) if alg.W[k][r] != 0)
               for k in range(len(alg.W)))


def kron_perm_variant(alg: Bilinear, PU, PV, PW, name: str) -> Bilinear:
    """[PU U, PV V, PW W] for permutation matrices given as 0-based index maps
    (row i of the result is row perm[i] of the input)."""
    return Bilinear(name, alg.M0, alg.K0, alg.N0,
                    [list(alg.U[PU[i]]) for i in range(len(alg.U))],
                    [list(alg.V[PV[i]]) for i in range(len(alg.V))],
                    [list(alg.W[PW[i]]) for i in range(len(alg.W))], f"variant of {alg.name}")


def kron_index_perm(P_outer: Sequence[Sequence[int]], P_inner: Sequence[Sequence[int]]):
    """Row map of the permutation matrix P_outer (x) P_inner (Kronecker product of 0/1
    permutation matrices given densely): returns perm with (P v)[i] = v[perm[i]]."""
    no, ni = len(P_outer), len(P_inner)
    perm = []
    for io in range(no):
        jo = [j for j in range(no) if P_outer[io][j]][0]
        for ii in range(ni):
            ji = [j for j in range(ni) if P_inner[ii][j]][0]
            perm.append(jo * ni + ji)
    return perm


ALGORITHMS = {
    "strassen": strassen,
    "winograd": winograd,
    "f323": f323,
    "f332": lambda: rotate(f323(), "f332"),
    "f233": lambda: rotate(rotate(f323()), "f233"),
    "f442": f442,
    "f424": f424,
    "f244": f244,
    "laderman333": laderman333,
    "classical222": lambda: classical(2, 2, 2),
}


def get(name: str) -> Bilinear:
    return ALGORITHMS[name]()
