"""Recursion trees of section 3.4 used by the tests: the non-uniform Strassen tree of Example
4.2 and the three-variant <3,2,3;15> tree of Example 4.3, registered with the library as user
rules (exact Brent check) from the oracle's coefficient tables."""
import numpy as np

from oracle import coeffs as C


def _int_rows(M):
    return np.array([[int(x) for x in r] for r in M], dtype=np.int64)


def _swap(n, perm):
    return [[1 if perm[i] == j else 0 for j in range(n)] for i in range(n)]


def dalberto_tree(F):
    """Example 4.2: Strassen's rule with D'Alberto's variant [U, (P x I) V, (I x P) W] at the
    nodes [2,1], [2,3], [2,4]; returns (node ids breadth first, oracle rule per path)."""
    s = C.strassen()
    P, I2 = _swap(2, [1, 0]), _swap(2, [0, 1])
    var = C.kron_perm_variant(s, list(range(4)), C.kron_index_perm(P, I2), C.kron_index_perm(I2, P), "dalberto")
    vid = F.fastmm_algo_register(2, 2, 2, 7, _int_rows(var.U), _int_rows(var.V), _int_rows(var.W), 0)
    nodes = {0, 2, 3}
    ids = [F.ALGOS["strassen"]] + [vid if r in nodes else F.ALGOS["strassen"] for r in range(7)]
    return ids, (lambda path: var if (len(path) == 1 and path[0] in nodes) else s)


def f323_tree(F):
    """Example 4.3: <3,2,3;15> with its two variants [(I x P) U, (P x I) V, (P x P) W] at the
    nodes listed there (1-based r1 = 1, 3, 10, 11 and 4, 5, 7, 9, 12, 13)."""
    a = C.f323()
    I2 = _swap(2, [0, 1])
    P1, P2 = _swap(3, [0, 2, 1]), _swap(3, [1, 2, 0])

    def variant(P, name):
        return C.kron_perm_variant(a, C.kron_index_perm(I2, P), C.kron_index_perm(P, I2), C.kron_index_perm(P, P),
                                   name)

    v1, v2 = variant(P1, "v1"), variant(P2, "v2")
    i1 = F.fastmm_algo_register(3, 2, 3, 15, _int_rows(v1.U), _int_rows(v1.V), _int_rows(v1.W), 0)
    i2 = F.fastmm_algo_register(3, 2, 3, 15, _int_rows(v2.U), _int_rows(v2.V), _int_rows(v2.W), 0)
    n1, n2 = {0, 2, 9, 10}, {3, 4, 6, 8, 11, 12}
    base = F.ALGOS["f323"]
    ids = [base] + [i1 if r in n1 else (i2 if r in n2 else base) for r in range(15)]
    rule = lambda path: (v1 if path[0] in n1 else (v2 if path[0] in n2 else a)) if len(path) == 1 else a
    return ids, rule


