"""Recursion trees of section 3.4 used by the tests: the non-uniform Strassen tree and the
three-variant <3,2,3;15> tree of the two non-uniform examples of section 5.2 (numbered 4.2 and
4.3 in these tests), registered with the library as user rules (exact Brent check) from the
oracle's coefficient tables."""
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




def composites(rule_at, dims, L):
    """Per leaf (r_1 .. r_L) in odometer order (r_1 most significant): the sets of composite A
    sources, B sources and (output block, coefficient) destinations of eq. (2) unrolled, with
    rule_at(path) the rule at the node reached by path = (r_1 .. r_{l-1}) and dims[l] its
    <M0,K0,N0> (A, B blocks column-major, C row-major; blocks indexed level 1 most significant)."""
    out = []

    def rec(l, path, a_terms, b_terms, c_terms):
        if l == L:
            out.append(({(br, bc, float(c)) for br, bc, c in a_terms}, {(br, bc, float(c)) for br, bc, c in b_terms},
                        {(br, bc, float(c)) for br, bc, c in c_terms}))
            return
        alg = rule_at(path)
        M0, K0, N0 = dims[l]
        for r in range(alg.R):
            na = [(br * M0 + i % M0, bc * K0 + i // M0, c * alg.U[i][r]) for br, bc, c in a_terms
                  for i in range(M0 * K0) if alg.U[i][r] != 0]
            nb = [(br * K0 + j % K0, bc * N0 + j // K0, c * alg.V[j][r]) for br, bc, c in b_terms
                  for j in range(K0 * N0) if alg.V[j][r] != 0]
            nc = [(br * M0 + k // N0, bc * N0 + k % N0, c * alg.W[k][r]) for br, bc, c in c_terms
                  for k in range(M0 * N0) if alg.W[k][r] != 0]
            rec(l + 1, path + (r,), na, nb, nc)

    rec(0, (), [(0, 0, 1)], [(0, 0, 1)], [(0, 0, 1)])
    return out


def table_composites(tab, NB):
    """The same sets read back from a library task table (NB: output block columns)."""
    dest_of = {}
    for b, (d0, dc) in enumerate(tab["bdest"]):
        for i in range(d0, d0 + dc):
            dest_of.setdefault(int(tab["dest_leaf"][i]), set()).add((b // NB, b % NB, float(tab["dest_coef"][i])))
    out = []
    for leaf, (a0, ac, b0, bc) in enumerate(tab["leaves"]):
        ga = {(int(tab["asrc"][i][0]), int(tab["asrc"][i][1]), float(tab["acoef"][i])) for i in range(a0, a0 + ac)}
        gb = {(int(tab["bsrc"][i][0]), int(tab["bsrc"][i][1]), float(tab["bcoef"][i])) for i in range(b0, b0 + bc)}
        out.append((ga, gb, dest_of.get(leaf, set())))
    return out
