"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and its host-side
logic (coefficient tables, quantities, planning rules, argument checks) agrees with the oracle.
No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import coeffs as C
from oracle import fastmm_oracle as O
from synth import make_pair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastmm.h")


@pytest.fixture(scope="module")
def F():
    import paper_1507_00687_amd as F

    if not os.path.exists(F.fastmm.LIB_PATH):
        from paper_1507_00687_amd import build

        build.build()
    return F


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:fastmm_status|const char|int)\s*\*?\s*(fastmm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol(F):
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(F.fastmm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


ORACLE_NAME = {
    "strassen": "strassen", "winograd": "winograd", "f323": "f323", "f332": "f332", "f233": "f233",
    "f442": "f442", "f424": "f424", "f244": "f244", "laderman333": "laderman333",
}


@pytest.mark.parametrize("name", sorted(ORACLE_NAME))
def test_library_tables_equal_oracle_tables(F, name):
    # Two independent transcriptions of the same rule must agree entry for entry.
    U, V, W = F.fastmm_algo_coeffs(name)
    Uo, Vo, Wo = C.get(ORACLE_NAME[name]).as_float()
    assert np.array_equal(U, Uo) and np.array_equal(V, Vo) and np.array_equal(W, Wo)
    info = F.fastmm_algo_info(name)
    q = C.quantities(C.get(ORACLE_NAME[name]))
    assert (info["nnz"], info["Q"], info["E"]) == (q.nnz, float(q.Q), float(q.E))


@pytest.mark.parametrize("name,depth,cutoff,shape", [
    ("strassen", 2, 64, (256, 256, 256)),
    ("strassen", 3, 64, (256, 256, 256)),
    ("f323", 3, 256, (4096, 4096, 4096)),
    ("f424", 2, 1, (37, 29, 41)),
    ("laderman333", 2, 1, (100, 1, 7)),
    ("winograd", 4, 1, (1, 1, 1)),
])
def test_plan_shape_matches_oracle_rules(F, name, depth, cutoff, shape):
    p = F.Plan(name, depth, cutoff)
    a = C.get(ORACLE_NAME[name])
    dims = [(a.M0, a.K0, a.N0)] * depth
    L = O.effective_depth(*shape, dims, cutoff)
    assert p.shape(*shape) == (L, *aligned_pads(shape, dims[:L]))


def aligned_pads(shape, dims):
    """The planner's padding: the oracle's (minimal) leaf block, rounded up to a multiple of 8
    elements when there is a level, times the product of the base sizes."""
    minimal = O.padded_dims(*shape, dims)
    if not dims:
        return minimal
    out = []
    for i, d in enumerate(shape):
        prod = int(np.prod([x[i] for x in dims]))
        b = -(-d // prod)
        out.append(-(-b // 8) * 8 * prod)
    assert all(o >= mn for o, mn in zip(out, minimal))
    return tuple(out)


def test_register_rejects_non_brent(F):
    a = C.strassen()
    U = np.array([[int(x) for x in r] for r in a.U])
    V = np.array([[int(x) for x in r] for r in a.V])
    W = np.array([[int(x) for x in r] for r in a.W])
    new_id = F.fastmm_algo_register(2, 2, 2, 7, U, V, W, 0)
    assert new_id >= 64
    assert F.fastmm_algo_info(new_id)["E"] == 12.0
    W2 = W.copy()
    W2[0, 0] = -W2[0, 0]
    with pytest.raises(F.FastmmError) as ei:
        F.fastmm_algo_register(2, 2, 2, 7, U, V, W2, 0)
    assert ei.value.status == -2  # FASTMM_EBRENT
    # the printed (unrelabelled) Strassen table is rejected as well
    sp = C.strassen_as_printed()
    with pytest.raises(F.FastmmError):
        F.fastmm_algo_register(2, 2, 2, 7, *[np.array([[int(x) for x in r] for r in M]) for M in (sp.U, sp.V, sp.W)], 0)


def test_plan_argument_errors(F):
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", -1)
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", 1, cutoff=0)
    with pytest.raises(F.FastmmError):
        F.Plan(77, 1)
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", 1, scaling="repeated", steps=0)


def test_gemm_argument_errors_before_launch(F):
    lib = F.lib()
    p = F.Plan("strassen", 1)
    # null plan, negative sizes, bad leading dims, aliasing: all rejected on the host
    assert lib.fastmm_gemm(None, 8, 8, 8, 4, 4, 4, None, 0, None) == -1
    assert lib.fastmm_gemm(p.handle, 8, 8, 8, -1, 4, 4, None, 0, None) == -1
    assert lib.fastmm_gemm_ex(p.handle, 8, 2, 0, 8, 4, 0, 4096, 4, 4, 4, 4, None, 0, None) == -3
    base = 1 << 20
    # C overlapping A
    assert lib.fastmm_gemm(p.handle, base, base + 100000, base + 64, 4, 4, 4, None, 0, None) in (-7, -8)
    # workspace too small (shape needs one at depth 1)
    assert p.workspace_size(64, 64, 64) > 0
    assert lib.fastmm_gemm(p.handle, base, base + 100000, base + 200000, 64, 64, 64, None, 0, None) == -8
    # empty products are no-ops
    assert lib.fastmm_gemm(p.handle, 0, 0, 0, 0, 5, 5, None, 0, None) == 0


def _int_rows(M):
    return np.array([[int(x) for x in r] for r in M], dtype=np.int64)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_path_selection(F, precision):
    P = lambda name, depth, cutoff=1, **kw: F.Plan(name, depth, cutoff, precision=precision, **kw)
    # FP32 <2,2,2> rules take the fused kernel from depth 3; below that, and for FP64, plans
    # write their leaf operands unless fusion is forced
    fused = "fused" if precision == "f32" else "written"
    assert P("strassen", 1).path(256, 256, 256) == "written"
    assert P("strassen", 2).path(256, 256, 256) == "written"
    assert P("strassen", 1, fuse="always").path(256, 256, 256) == "fused"
    assert P("strassen", 2, fuse="always").path(256, 256, 256) == "fused"
    assert P("winograd", 3).path(300, 200, 100) == fused
    assert P("strassen", 3).path(17, 300, 41) == fused
    # transposed operands are copied to row-major and take the fused kernel too; no level and
    # cutoff stopping at depth 0 take the leaf path; other rules write their leaf operands
    assert P("strassen", 3).path(256, 256, 256, transB=True) == fused
    assert P("strassen", 3).path(256, 256, 256, transA=True) == fused
    assert P("strassen", 0).path(256, 256, 256) == "leaf"
    assert P("strassen", 2, 512).path(256, 256, 256) == "leaf"
    assert P("f323", 1).path(300, 200, 300) == "written"
    assert P("laderman333", 1).path(300, 300, 300) == "written"
    assert P("strassen", 2, fuse=False).path(256, 256, 256) == "leaf"
    assert P("strassen", 2, fuse="off").path(256, 256, 256) == "leaf"
    # "written": the batched call's path, never the fused kernel
    assert P("strassen", 1, fuse="written").path(256, 256, 256) == "written"
    assert P("strassen", 0, fuse="written").path(256, 256, 256) == "leaf"
    plan = P("strassen", 1)
    with pytest.raises(F.FastmmError):
        F.fastmm._check(F.fastmm.lib().fastmm_plan_set_fusion(plan.handle, 4))
    assert F.Plan("strassen", 1, 1, precision="bf16x3").path(256, 256, 256) == "leaf"


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_written_path_selection(F, precision):
    """From depth 1, FP32/FP64 plans with one rule write their leaf operands out level by level
    (FP32 <2,2,2> rules keep the fused kernel); split precisions form limb planes instead;
    depth 0, fusion off and trees stay on the leaf path."""
    P = lambda name, depth, cutoff=1, **kw: F.Plan(name, depth, cutoff, precision=precision, **kw)
    assert P("f424", 2).path(256, 128, 256) == "written"
    assert P("f323", 2).path(198, 200, 180) == "written"
    assert P("laderman333", 2).path(135, 100, 81) == "written"
    assert P("f424", 2).path(256, 128, 256, transA=True, transB=True) == "written"
    assert P("f424", 1).path(256, 128, 256) == "written"
    assert P("f424", 2, 64).path(256, 128, 256) == "written"      # the cutoff leaves one level
    assert P("f424", 2, 200).path(256, 128, 256) == "leaf"        # ... or none
    assert P("f424", 2, fuse="off").path(256, 128, 256) == "leaf"  # fusion off: composite lists only
    assert P("laderman333", 3).path(270, 270, 270) == "written"
    assert P("strassen", 3).path(256, 256, 256) == ("fused" if precision == "f32" else "written")
    assert F.Plan("f424", 2, 1, precision="f16x3").path(256, 128, 256) == "leaf"
    # per-level and per-node rules write their leaf operands (each level or node with its own rule)
    assert P("strassen", 2).set_tree(["strassen"] + ["winograd"] * 7).path(256, 256, 256) == "written"
    assert P("strassen", 2).set_levels(["strassen", "winograd"]).path(256, 256, 256) == "written"
    assert P("f424", 2).set_levels(["f424", "strassen"]).path(256, 128, 256) == "written"


def test_fused_loads_path_selection(F):
    """With fusion "always", split precisions with 256-wide leaf blocks, at most two limbs and a
    rule with at most two nonzeros per column of U and V (Strassen's; classical) form the
    innermost level in the limb GEMM's loads; other rules, 128 tiles, three limbs, fusion off
    and the default mode (the faster limb planes) take limb planes."""
    P = lambda name, depth, prec="f16x3", fuse="always", **kw: F.Plan(name, depth, 1, precision=prec, fuse=fuse,
                                                                       **kw)
    assert P("strassen", 2, fuse="auto").path(1024, 1024, 1024) == "leaf"  # limb planes are faster
    assert P("strassen", 2).path(1024, 1024, 1024) == "fused_loads"
    assert P("strassen", 1).path(520, 1032, 600) == "fused_loads"
    assert P("classical", 0).path(600, 520, 300) == "fused_loads"
    assert P("strassen", 2, "bf16").path(1024, 1024, 1024) == "fused_loads"
    assert P("strassen", 1).path(600, 520, 300) == "leaf"            # 150-wide blocks: 128 tiles
    assert P("winograd", 1).path(1024, 1024, 1024) == "leaf"         # four nonzeros in a U column
    assert P("f424", 2).path(4096, 4096, 4096) == "leaf"
    assert P("strassen", 2, "bf16x6").path(1024, 1024, 1024) == "leaf"  # three limbs
    assert P("strassen", 2, fuse="off").path(1024, 1024, 1024) == "leaf"
    assert P("strassen", 2).set_tile(128).path(1024, 1024, 1024) == "leaf"
    # the fused path needs no limb planes: its workspace is far smaller
    assert P("strassen", 2).workspace_size(4096, 4096, 4096) < P("strassen", 2, fuse="off").workspace_size(
        4096, 4096, 4096)


def test_fused_path_matches_rules_by_coefficients(F):
    # Cyclic rotations (the rules of the backward pass) and user rules equal to a built-in
    # one take the fused path; a rule with its products reordered does not.
    for name in ("strassen", "winograd"):
        a = C.get(name)
        for t in range(3):
            r = a
            for _ in range(t):
                r = C.rotate(r)
            uid = F.fastmm_algo_register(2, 2, 2, 7, _int_rows(r.U), _int_rows(r.V), _int_rows(r.W), 0)
            assert F.Plan(uid, 1, 1, precision="f32", fuse="always").path(128, 128, 128) == "fused", (name, t)
            assert F.Plan(uid, 2, 1, precision="f64", fuse="always").path(128, 128, 128) == "fused", (name, t)
    a = C.strassen()
    perm = [1, 0, 2, 3, 4, 5, 6]
    U, V, W = (_int_rows(M)[:, perm] for M in (a.U, a.V, a.W))
    uid = F.fastmm_algo_register(2, 2, 2, 7, U, V, W, 0)
    assert F.Plan(uid, 1, 1, precision="f32").path(128, 128, 128) == "written"  # no fused kernel


def _transpose_rule(a):
    """The rule for <N0,K0,M0> that forms C^T = B^T A^T with the products of `a` transposed
    (section 3.1): written here from the index conventions (A, B single indices column-major,
    C row-major), independently of the library's own transposition."""
    M0, K0, N0, R = a.M0, a.K0, a.N0, len(a.U[0])
    U = [[0] * R for _ in range(N0 * K0)]
    V = [[0] * R for _ in range(K0 * M0)]
    W = [[0] * R for _ in range(N0 * M0)]
    for r in range(R):
        for p in range(N0):
            for q in range(K0):
                U[p + q * N0][r] = a.V[q + p * K0][r]
        for q in range(K0):
            for t in range(M0):
                V[q + t * K0][r] = a.U[t + q * M0][r]
        for p in range(N0):
            for t in range(M0):
                W[p * M0 + t][r] = a.W[t * N0 + p][r]
    return N0, K0, M0, R, U, V, W


@pytest.mark.parametrize("name", ["strassen", "winograd", "f323", "f424"])
def test_transposed_rotations_are_rules_and_form_the_transpose(F, name):
    """The backward products use the transposes of the rotations: each is a valid rule (the
    library's registration checks the Brent equations exactly), computes (A B)^T from (B^T, A^T)
    exactly on integers through its task table, and for <2,2,2;7> rules it has a compiled fused
    kernel (the backward pass stays on the fused path)."""
    a = C.get(name)
    rng = np.random.default_rng(7)
    for t in range(3):
        r = a
        for _ in range(t):
            r = C.rotate(r)
        M0, K0, N0, R, U, V, W = _transpose_rule(r)
        # coefficients in {0, +-1/2, +-1}: numerators over a common 2^1 (a denominator of 1 when integral)
        frac = any(x != int(x) for M in (U, V, W) for row in M for x in row)
        num = [np.array([[int(2 * x) if frac else int(x) for x in row] for row in M], dtype=np.int64)
               for M in (U, V, W)]
        uid = F.fastmm_algo_register(M0, K0, N0, R, *num, 1 if frac else 0)
        # (A B)^T = B^T A^T through the transposed rule's one-level task table
        m, k, n = 2 * r.M0, 3 * r.K0, 2 * r.N0
        A = rng.integers(-4, 5, (m, k)).astype(np.float64)
        B = rng.integers(-4, 5, (k, n)).astype(np.float64)
        tab = F.fastmm_task_table(F.Plan(uid, 1, 1), 1)
        got = _eval_tables(tab, np.ascontiguousarray(B.T), np.ascontiguousarray(A.T), M0, K0, N0, 1)
        assert np.array_equal(got, (A @ B).T)
        if (M0, K0, N0, R) == (2, 2, 2, 7):
            assert F.Plan(uid, 1, 1, precision="f32", fuse="always").path(128, 128, 128) == "fused", (name, t)
            assert F.Plan(uid, 2, 1, precision="f64", fuse="always").path(128, 128, 128) == "fused", (name, t)


def test_backward_workspace_and_batched_errors_on_host(F):
    p = F.Plan("strassen", 2, 64, precision="f32")
    lib = F.lib()
    size = ctypes.c_size_t()
    assert lib.fastmm_backward_workspace_size(p.handle, 300, 200, 100, ctypes.byref(size)) == 0
    need_a = ctypes.c_size_t()
    need_b = ctypes.c_size_t()
    # the two products: dA (300 x 200) = G (300 x 100) B^T, dB (200 x 100) = A^T G
    assert lib.fastmm_workspace_size(p.handle, 300, 100, 200, ctypes.byref(need_a)) == 0
    assert lib.fastmm_workspace_size(p.handle, 200, 300, 100, ctypes.byref(need_b)) == 0
    assert size.value >= min(need_a.value, need_b.value) > 0
    from paper_1507_00687_amd.fastmm import _GradProblem, _ProblemEx

    handles = (ctypes.c_void_p * 1)(p.handle.value)
    bad = (_GradProblem * 1)(_GradProblem(8, 8, 8, 4096, 8192, -1, 4, 4))
    assert lib.fastmm_backward_batched_workspace_size(handles, bad, 1, ctypes.byref(size)) == -1
    # a strided product whose ldc is below n: rejected before any launch
    base = 1 << 20
    pe = (_ProblemEx * 1)(_ProblemEx(base, 64, 0, base + 65536, 64, 1, base + 131072, 32, 64, 64, 64))
    assert lib.fastmm_batched_ex_workspace_size(handles, pe, 1, ctypes.byref(size)) == 0
    assert lib.fastmm_gemm_batched_ex(handles, pe, 1, base + (1 << 24), size.value, None) == -3
    # an output overlapping an input of the batch
    pe2 = (_ProblemEx * 1)(_ProblemEx(base, 64, 0, base + 65536, 64, 1, base + 1024, 64, 64, 64, 64))
    assert lib.fastmm_gemm_batched_ex(handles, pe2, 1, base + (1 << 24), size.value, None) == -7


# ----------------------------------------------------------------- non-uniform recursion trees
from tests.trees import dalberto_tree, f323_tree  # noqa: E402


def _eval_tables(tab, A, B, M0, K0, N0, L):
    """C from a composite task table (eq. (2) unrolled): every leaf's product of its source
    sums, then every output block the sum of its contributions (exact on small integers)."""
    m, k = A.shape
    n = B.shape[1]
    mb, kb, nb = m // M0 ** L, k // K0 ** L, n // N0 ** L
    blk = lambda X, r, c, h, w: X[r * h:(r + 1) * h, c * w:(c + 1) * w]
    Ms = []
    for a0, ac, b0, bc in tab["leaves"]:
        S = sum(tab["acoef"][i] * blk(A, *tab["asrc"][i], mb, kb) for i in range(a0, a0 + ac))
        T = sum(tab["bcoef"][i] * blk(B, *tab["bsrc"][i], kb, nb) for i in range(b0, b0 + bc))
        Ms.append(S @ T)
    Cm = np.zeros((m, n))
    NB = N0 ** L
    for b, (d0, dc) in enumerate(tab["bdest"]):
        P_, S_ = divmod(b, NB)
        acc = sum(tab["dest_coef"][i] * Ms[tab["dest_leaf"][i]] for i in range(d0, d0 + dc))
        Cm[P_ * mb:(P_ + 1) * mb, S_ * nb:(S_ + 1) * nb] = acc
    return Cm


@pytest.mark.parametrize("tree,base,dims", [("dalberto", "strassen", (2, 2, 2)), ("f323", "f323", (3, 2, 3))])
def test_tree_task_table_equals_oracle_tree(F, tree, base, dims):
    ids, rule = (dalberto_tree if tree == "dalberto" else f323_tree)(F)
    p = F.Plan(base, 2, 1).set_tree(ids)
    M0, K0, N0 = dims
    A, B = make_pair("int8", 31, M0 * M0 * 3, K0 * K0 * 2, N0 * N0 * 3)
    tab = F.fastmm_task_table(p, 2)
    got = _eval_tables(tab, A, B, M0, K0, N0, 2)
    want = O.fast_tree(A, B, rule, [dims, dims])
    assert np.array_equal(got, want)
    # and the tree really differs from the uniform rule's table
    uni = F.fastmm_task_table(F.Plan(base, 2, 1), 2)
    assert not (np.array_equal(uni["bsrc"], tab["bsrc"]) and np.array_equal(uni["dest_leaf"], tab["dest_leaf"])
                and np.array_equal(uni["bcoef"], tab["bcoef"]) and np.array_equal(uni["dest_coef"], tab["dest_coef"]))


def _tree_composites(rule, R, dims):
    """Per leaf (r1, r2), in odometer order: the sets of composite A sources, B sources and
    (output block, coefficient) destinations of a two-level tree, from eq. (2) with the rule of
    each node (A, B blocks column-major, C row-major)."""
    M0, K0, N0 = dims
    out = []
    for r1 in range(R):
        top, child = rule(()), rule((r1,))
        for r2 in range(R):
            def srcs(X1, X2, rows):
                got = set()
                for i1, row1 in enumerate(X1):
                    for i2, row2 in enumerate(X2):
                        c = row1[r1] * row2[r2]
                        if c != 0:
                            p1, q1, p2, q2 = i1 % rows, i1 // rows, i2 % rows, i2 // rows
                            cols = len(X1) // rows
                            got.add((p1 * rows + p2, q1 * cols + q2, float(c)))
                return got
            dests = set()
            for k1, row1 in enumerate(top.W):
                for k2, row2 in enumerate(child.W):
                    c = row1[r1] * row2[r2]
                    if c != 0:
                        P_ = (k1 // N0) * M0 + k2 // N0
                        S_ = (k1 % N0) * N0 + k2 % N0
                        dests.add((P_, S_, float(c)))
            out.append((srcs(top.U, child.U, M0), srcs(top.V, child.V, K0), dests))
    return out


@pytest.mark.parametrize("tree,base,dims", [("dalberto", "strassen", (2, 2, 2)), ("f323", "f323", (3, 2, 3))])
def test_tree_task_table_structure(F, tree, base, dims):
    # The right rule at the right node: every leaf's composite sources and destinations.
    ids, rule = (dalberto_tree if tree == "dalberto" else f323_tree)(F)
    R = C.get(base).R
    tab = F.fastmm_task_table(F.Plan(base, 2, 1).set_tree(ids), 2)
    want = _tree_composites(rule, R, dims)
    assert len(tab["leaves"]) == len(want)
    NB = dims[2] ** 2
    dest_of = {}
    for b, (d0, dc) in enumerate(tab["bdest"]):
        for i in range(d0, d0 + dc):
            dest_of.setdefault(int(tab["dest_leaf"][i]), set()).add((b // NB, b % NB, float(tab["dest_coef"][i])))
    for leaf, ((a0, ac, b0, bc), (wa, wb, wd)) in enumerate(zip(tab["leaves"], want)):
        ga = {(int(tab["asrc"][i][0]), int(tab["asrc"][i][1]), float(tab["acoef"][i])) for i in range(a0, a0 + ac)}
        gb = {(int(tab["bsrc"][i][0]), int(tab["bsrc"][i][1]), float(tab["bcoef"][i])) for i in range(b0, b0 + bc)}
        assert ga == wa and gb == wb and dest_of.get(leaf, set()) == wd, leaf


def test_tree_argument_errors(F):
    ids, _ = dalberto_tree(F)
    p = F.Plan("strassen", 2, 1)
    with pytest.raises(F.FastmmError):
        p.set_tree(ids[:-1])  # one node short
    with pytest.raises(F.FastmmError):
        p.set_tree([F.ALGOS["f323"]] * 8)  # another shape
    with pytest.raises(F.FastmmError):
        p.set_tree([10 ** 6] * 8)  # unknown id
    p.set_tree(ids)
    assert p.path(128, 128, 128) == "written"  # each parent node's operands formed with its own rule
    assert F.Plan("strassen", 2, 1, fuse="off").set_tree(ids).path(128, 128, 128) == "leaf"
    p.set_tree([])
    assert F.Plan("strassen", 3, 1, precision="f32").path(128, 128, 128) == "fused"


def test_stability_exponent_and_fig2_quantities(F):
    # Table 1's stability exponents (rounded to two decimals in print) and the closed forms of
    # Figure 2's axes, computed by the library from its own rules and their rotations.
    gold = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "table1_stab_exp.txt")):
        if line.strip() and not line.startswith("#"):
            key, val, _ = line.split()
            gold[key] = float(val)
    for key in ("strassen", "f323", "f332", "f424"):
        assert abs(F.fastmm_algo_stability(key)["stab_exp"] - gold[key]) <= 0.005, key
    # <4,4,2>: the printed 3.90 is log_32(89 * 89 * 92); with its rotations' E (89, 102, 92) the
    # exponent equals <4,2,4>'s.
    e442 = F.fastmm_algo_stability("f442")["stab_exp"]
    assert abs(e442 - F.fastmm_algo_stability("f424")["stab_exp"]) < 1e-12
    assert abs(np.log(89.0 * 89 * 92) / np.log(32) - gold["f442"]) <= 0.005
    for key in ("strassen", "f323", "f424", "laderman333"):
        info = F.fastmm_algo_info(key)
        for L in (1, 2, 3):
            d = F.fastmm_algo_stability(key, L)
            assert d["flops_frac"] == pytest.approx((info["R"] / (info["M0"] * info["K0"] * info["N0"])) ** L)
            assert d["rel_instability"] == pytest.approx((info["E"] / info["K0"] ** 2) ** L)
    assert F.fastmm_algo_stability("strassen", 1)["flops_frac"] == 7 / 8


# ----------------------------------------------------------- uniform non-stationary recursion
LEVELS = [(["f323", "strassen"], (37, 29, 41)), (["strassen", "f424"], (100, 60, 90)),
          (["f332", "f233", "f323"], (60, 50, 70)), (["winograd", "f424", "strassen"], (128, 64, 128))]


@pytest.mark.parametrize("levels,shape", LEVELS)
def test_levels_shape_and_tables_equal_oracle(F, levels, shape):
    from tests.trees import composites, table_composites

    rules = [C.get(ORACLE_NAME[a]) for a in levels]
    dims = [(a.M0, a.K0, a.N0) for a in rules]
    p = F.Plan(levels[0], len(levels), 1).set_levels(levels)
    L = O.effective_depth(*shape, dims, 1)
    assert p.shape(*shape) == (L, *aligned_pads(shape, dims[:L]))
    # every leaf's composite sources and destinations, from eq. (2) level by level
    NB = int(np.prod([d[2] for d in dims]))
    want = composites(lambda path: rules[len(path)], dims, len(levels))
    got = table_composites(F.fastmm_task_table(p, len(levels)), NB)
    assert got == want
    # and the cutoff keeps the first levels
    p2 = F.Plan(levels[0], len(levels), 20).set_levels(levels)
    L2 = O.effective_depth(*shape, dims, 20)
    assert p2.shape(*shape) == (L2, *aligned_pads(shape, dims[:L2]))


def test_levels_argument_errors(F):
    p = F.Plan("strassen", 2, 1)
    with pytest.raises(F.FastmmError):
        p.set_levels(["strassen"])  # depth 2 needs two rules
    with pytest.raises(F.FastmmError):
        p.set_levels(["strassen", 10 ** 6])
    p.set_levels(["f323", "strassen"])
    assert p.path(256, 256, 256) == "written"  # leaf operands written level by level, each level's rule
    assert F.Plan("strassen", 2, 1, fuse="off").set_levels(["f323", "strassen"]).path(256, 256, 256) == "leaf"
    p.set_levels([])
    assert p.shape(32, 32, 32) == (2, 32, 32, 32)


def test_every_level_scaling_plan_rules(F):
    import torch

    from tests.trees import dalberto_tree

    m = k = n = 256
    once = F.Plan("strassen", 2, 1, scaling="out_in", precision="f32")
    every = F.Plan("strassen", 2, 1, scaling="out_in", precision="f32", per_level=True)
    # from depth 2: the first level's node operands and products (7 each of 128 x 128) plus
    # the nested products' own workspace
    nested = F.Plan("strassen", 1, 1, scaling="out_in", precision="f32").workspace_size(128, 128, 128)
    assert every.workspace_size(m, k, n) >= 7 * 3 * 128 * 128 * 4 + nested
    # scaling once on the written path at depth 2: the first level's node operands of both
    # sides and the leaf products, 7 each of 128 x 128 (and the stacked leaf operands)
    assert once.workspace_size(m, k, n) >= 3 * 7 * 128 * 128 * 4
    assert every.path(m, k, n) == "every_level" and once.path(m, k, n) == "written"
    # depth <= 1 (or no scaling, or the cutoff stopping at one level): as scaling once
    for depth, mode, cutoff in ((1, "out_in", 1), (2, "none", 1), (2, "outside", 100)):
        a = F.Plan("strassen", depth, cutoff, scaling=mode, per_level=True)
        b = F.Plan("strassen", depth, cutoff, scaling=mode)
        assert a.workspace_size(m, k, n) == b.workspace_size(m, k, n)
        assert a.path(m, k, n) == b.path(m, k, n) != "every_level"
    # uniform non-stationary plans nest the remaining levels' rules
    lv = F.Plan("f323", 2, 1, scaling="outside", precision="f64", per_level=True).set_levels(["f323", "strassen"])
    assert lv.workspace_size(300, 200, 300) > 0
    # not with trees, not in a batch (from depth 2)
    ids, _ = dalberto_tree(F)
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", 2, 1, scaling="outside", per_level=True).set_tree(ids)
    F.Plan("strassen", 2, 1, scaling="none", per_level=True).set_tree(ids)  # no scaling: no conflict
    A, B = torch.zeros((m, k)), torch.zeros((k, n))
    with pytest.raises(F.FastmmError):
        F.fastmm_batched_workspace_size([every], [A], [B])
    shallow = F.Plan("strassen", 1, 1, scaling="out_in", precision="f32", per_level=True)
    assert F.fastmm_batched_workspace_size([shallow], [A], [B]) > 0
    # per_level must be 0 or 1 in the C struct
    h = ctypes.c_void_p()
    sc = F.fastmm._Scaling(1, 2, 0.0, 2)
    assert F.lib().fastmm_plan_create(ctypes.byref(h), 1, 2, 1, ctypes.byref(sc), 1) != 0


def test_plan_tile_setting(F):
    # split precisions only; 256 x 256 needs at most two limbs; 0 returns to the shape's choice
    # (through limb planes, fusion off: the planes' padding follows the tile)
    p = F.Plan("strassen", 1, 1, precision="f16x3", fuse="off")
    auto = p.workspace_size(600, 600, 600)
    assert p.set_tile(256).workspace_size(600, 600, 600) == auto  # 304-row leaf blocks take 256 tiles
    small = p.set_tile(128).workspace_size(600, 600, 600)
    assert small < auto  # planes padded to 384 rather than 512
    assert p.set_tile(0).workspace_size(600, 600, 600) == auto
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", 1, 1, precision="bf16x6").set_tile(256)
    F.Plan("strassen", 1, 1, precision="bf16x6").set_tile(128)
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", 1, 1, precision="f32").set_tile(128)
    with pytest.raises(F.FastmmError):
        F.Plan("strassen", 1, 1, precision="f16x3").set_tile(64)
