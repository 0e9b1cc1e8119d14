"""Oracle: recursive bilinear fast matrix multiplication with diagonal scaling, on the CPU.

TEST INFRASTRUCTURE ONLY. Nothing under oracle/ is part of the product path; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it. It shares no
code with the GPU library: its coefficient tables, planner rules, scaling arithmetic and
error measures are written here independently, and it never calls the product library.

What it computes, each piece following the paper:
  * classical(A, B)         -- the classical base case, sequential summation (section 4.2).
  * reference_rows(A, B)    -- error reference: classical product in long double.
  * fast(A, B, alg, L)      -- stationary recursion of eq. (2): S_r = sum_i U_ir A_i,
                               T_r = sum_j V_jr B_j, M_r = S_r * T_r recursively,
                               C_k = sum_r W_kr M_r, classical after L levels (section 3.2);
                               zero padding to multiples of M0^L, K0^L, N0^L (section 3.2).
  * fast_tree(...)          -- uniform and non-uniform non-stationary recursion
                               (sections 3.3, 3.4): one rule per level or per tree node.
  * outside/inside/repeated scaling -- Algorithms 1, 2, 3 (section 6), with the stopping
                               test of the stopping-criterion theorem (section 6.3)
                               and an exact power-of-two variant;
                               applied once (scaled_fast) or at every inner node of the
                               recursion (scaled_fast_every_level, a reading).
  * bounds                  -- Theorems 4.1 and 4.2 and the non-uniform quantities of
                               section 4.5; normwise and componentwise error measures.

All floating-point work is in the dtype of the inputs (float64 unless a float32 pair is
passed); sums run sequentially in increasing index order, multiplications by +-1 and
powers of two are exact.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import coeffs
from .coeffs import Bilinear

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "_ref.so")
        if not os.path.exists(path):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(path)
        i64, dp, fp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
        lib.orc_classical_f64.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
        lib.orc_classical_f32.argtypes = [i64, i64, i64, fp, i64, fp, i64, fp, i64]
        lib.orc_classical_ld.argtypes = [i64, ctypes.POINTER(ctypes.c_int64), i64, i64, dp, i64,
                                         dp, i64, ctypes.c_void_p, i64]
        lib.orc_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def num_threads() -> int:
    return int(_lib().orc_num_threads())


# ---------------------------------------------------------------------- classical kernels
def classical(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A B by the classical algorithm, c_ij summed sequentially over k (section 4.2)."""
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    dt = np.result_type(A.dtype, B.dtype)
    if dt == np.float32:
        A = np.ascontiguousarray(A, dtype=np.float32)
        B = np.ascontiguousarray(B, dtype=np.float32)
        C = np.empty((m, n), dtype=np.float32)
        if m and n:
            P = ctypes.POINTER(ctypes.c_float)
            _lib().orc_classical_f32(m, k, n, A.ctypes.data_as(P), k, B.ctypes.data_as(P), n,
                                     C.ctypes.data_as(P), n)
        return C
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    C = np.empty((m, n), dtype=np.float64)
    if m and n:
        P = ctypes.POINTER(ctypes.c_double)
        _lib().orc_classical_f64(m, k, n, A.ctypes.data_as(P), k, B.ctypes.data_as(P), n,
                                 C.ctypes.data_as(P), n)
    return C


def reference_rows(A: np.ndarray, B: np.ndarray, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """Rows of A B accumulated in long double (x87 extended): the error reference."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    rows = np.arange(m, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((len(rows), n), dtype=np.longdouble)
    if len(rows) and n:
        P = ctypes.POINTER(ctypes.c_double)
        _lib().orc_classical_ld(len(rows), rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k, n,
                                A.ctypes.data_as(P), k, B.ctypes.data_as(P), n,
                                out.ctypes.data_as(ctypes.c_void_p), n)
    return out


# ------------------------------------------------------------------------- planning rules
def effective_depth(m: int, k: int, n: int, dims: Sequence[Tuple[int, int, int]], cutoff: int) -> int:
    """Number of recursion levels actually used: recurse while levels remain and every child
    dimension (ceil of the unpadded dimension over the product of base sizes so far) is at
    least `cutoff`.  `dims` lists (M0, K0, N0) for the levels that may be used."""
    L = 0
    pm = pk = pn = 1
    for (M0, K0, N0) in dims:
        pm, pk, pn = pm * M0, pk * K0, pn * N0
        if -(-m // pm) < cutoff or -(-k // pk) < cutoff or -(-n // pn) < cutoff:
            break
        L += 1
    return L


def padded_dims(m, k, n, dims: Sequence[Tuple[int, int, int]]):
    pm = int(np.prod([d[0] for d in dims])) if dims else 1
    pk = int(np.prod([d[1] for d in dims])) if dims else 1
    pn = int(np.prod([d[2] for d in dims])) if dims else 1
    return (-(-m // pm) * pm, -(-k // pk) * pk, -(-n // pn) * pn)


# ------------------------------------------------------------------------------ recursion
def _coef(x) -> float:
    return float(x)


def _rec(A: np.ndarray, B: np.ndarray, alg_at: Callable[[tuple], Bilinear], depth: int,
         path: tuple, leaf: Callable) -> np.ndarray:
    """One node of the recursion tree (eq. (2)): A, B already padded to the node's size."""
    if depth == 0:
        return leaf(A, B)
    alg = alg_at(path)
    M0, K0, N0, R = alg.M0, alg.K0, alg.N0, alg.R
    m, k = A.shape
    n = B.shape[1]
    mb, kb, nb = m // M0, k // K0, n // N0
    # Blocks with single indices: A and B column-major, C row-major (section 3.1).
    Ablk = [A[(i % M0) * mb:(i % M0 + 1) * mb, (i // M0) * kb:(i // M0 + 1) * kb]
            for i in range(M0 * K0)]
    Bblk = [B[(j % K0) * kb:(j % K0 + 1) * kb, (j // K0) * nb:(j // K0 + 1) * nb]
            for j in range(K0 * N0)]
    Ms: List[Optional[np.ndarray]] = []
    for r in range(R):
        S = None
        for i in range(M0 * K0):
            u = alg.U[i][r]
            if u != 0:
                term = Ablk[i] * A.dtype.type(_coef(u))
                S = term if S is None else S + term
        T = None
        for j in range(K0 * N0):
            v = alg.V[j][r]
            if v != 0:
                term = Bblk[j] * B.dtype.type(_coef(v))
                T = term if T is None else T + term
        if S is None or T is None:  # an all-zero column: the product is zero
            Ms.append(None)
            continue
        Ms.append(_rec(S, T, alg_at, depth - 1, path + (r,), leaf))
    C = np.zeros((m, n), dtype=A.dtype)
    for kk in range(M0 * N0):
        p, s = kk // N0, kk % N0
        acc = None
        for r in range(R):
            w = alg.W[kk][r]
            if w != 0 and Ms[r] is not None:
                term = Ms[r] * A.dtype.type(_coef(w))
                acc = term if acc is None else acc + term
        if acc is not None:
            C[p * mb:(p + 1) * mb, s * nb:(s + 1) * nb] = acc
    return C


def fast_tree(A: np.ndarray, B: np.ndarray, alg_at: Callable[[tuple], Bilinear],
              dims: Sequence[Tuple[int, int, int]], leaf: Optional[Callable] = None) -> np.ndarray:
    """Recursive fast multiplication with the rule alg_at(path) at the tree node reached by
    `path` = (r_1, ..., r_{l-1}) (notation [l, r_1, ..., r_{l-1}] of section 3.4), for
    len(dims) levels, classical below.  Inputs are zero padded and the result is cropped."""
    leaf = leaf or classical
    m, k = A.shape
    n = B.shape[1]
    if len(dims) == 0:
        return leaf(A, B)
    Mp, Kp, Np = padded_dims(m, k, n, dims)
    Ap = np.zeros((Mp, Kp), dtype=A.dtype)
    Ap[:m, :k] = A
    Bp = np.zeros((Kp, Np), dtype=B.dtype)
    Bp[:k, :n] = B
    C = _rec(Ap, Bp, alg_at, len(dims), (), leaf)
    return np.ascontiguousarray(C[:m, :n])


def fast(A: np.ndarray, B: np.ndarray, alg: Bilinear, depth: int, cutoff: int = 1,
         leaf: Optional[Callable] = None) -> np.ndarray:
    """Stationary algorithm: `depth` levels of [U,V,W] (fewer if the cutoff stops it), then
    the classical algorithm (section 3.2)."""
    m, k = A.shape
    n = B.shape[1]
    L = effective_depth(m, k, n, [(alg.M0, alg.K0, alg.N0)] * depth, cutoff)
    return fast_tree(A, B, lambda path: alg, [(alg.M0, alg.K0, alg.N0)] * L, leaf)


# -------------------------------------------------------------------------------- scaling
def pow2_ceil(x: np.ndarray) -> np.ndarray:
    """Smallest power of two >= x, for finite x > 0 (exact, via the binary exponent)."""
    f, e = np.frexp(x)
    return np.ldexp(1.0, np.where(f == 0.5, e - 1, e)).astype(np.float64)


def pow2_nearest(x: np.ndarray) -> np.ndarray:
    """2^j with j the integer nearest to log2 x, for finite x > 0 (exact, via the binary
    exponent).  With x = f 2^e, f in [1/2, 1): log2 x = e + log2 f lies in [e-1, e), nearer e
    exactly when f > 2^-1/2.  No double equals the irrational 2^-1/2, so f > 2^-1/2 is
    f >= the smallest double above it, and there are no ties."""
    f, e = np.frexp(x)
    above = float.fromhex("0x1.6a09e667f3bcdp-1")  # smallest double > 2^-1/2
    return np.ldexp(1.0, np.where(f >= above, e, e - 1)).astype(np.float64)


def pow2_sqrt_ratio(b: np.ndarray, a: np.ndarray) -> np.ndarray:
    """2^j with j the nearest integer to log2(b/a)/2, ties to even; exact for finite b, a > 0.

    With b = fb 2^eb, a = fa 2^ea (fb, fa in [1/2, 1)) and d = eb - ea, log2(b/a) lies in
    (d-1, d+1).  For even d the answer is d/2.  For odd d it is (d-1)/2 or (d+1)/2 as fb < fa
    or fb > fa, and the even one of the two when fb == fa (b/a = 2^d exactly)."""
    fb, eb = np.frexp(b)
    fa, ea = np.frexp(a)
    d = (eb - ea).astype(np.int64)
    lo = (d - 1) // 2
    hi = lo + 1
    odd = (d % 2) != 0
    j = np.where(~odd, d // 2, np.where(fb < fa, lo, np.where(fb > fa, hi, np.where(lo % 2 == 0, lo, hi))))
    return np.ldexp(1.0, j).astype(np.float64)


def _safe_positive(x: np.ndarray) -> np.ndarray:
    return np.isfinite(x) & (x > 0)


@dataclass
class ScalingResult:
    A: np.ndarray  # A' after the steps
    B: np.ndarray  # B' after the steps
    r: np.ndarray  # diagonal of D_A (cumulative)
    s: np.ndarray  # diagonal of D_B (cumulative)
    p: Optional[np.ndarray] = None  # product of the applied inside factors (A' = .. A diag(p))
    steps: List[str] = field(default_factory=list)  # 'O' / 'I' per step taken
    factors: List[tuple] = field(default_factory=list)  # unrounded (r', s') or (p',) per step
    stopped_early: bool = False


def o_step(A1, B1, pow2: bool, o_round: str = "up"):
    """Outside step (Algorithm 1; Algorithm 3 'O step'): divide rows of A' by their max-abs and
    columns of B' by theirs.  Returns new A', B', the applied factors and the unrounded ones.
    All-zero rows/columns (and non-finite maxima) get factor 1.  With pow2 each factor is
    rounded to a power of two (section 6): the smallest one >= the max (o_round 'up') or the
    one nearest to it in log scale ('nearest')."""
    rnd = {"up": pow2_ceil, "nearest": pow2_nearest}[o_round]
    ra = np.max(np.abs(A1), axis=1) if A1.shape[1] else np.zeros(A1.shape[0])
    sb = np.max(np.abs(B1), axis=0) if B1.shape[0] else np.zeros(B1.shape[1])
    ra_ok, sb_ok = _safe_positive(ra), _safe_positive(sb)
    ra_u = np.where(ra_ok, ra, 1.0)
    sb_u = np.where(sb_ok, sb, 1.0)
    if pow2:
        rp = np.where(ra_ok, rnd(ra_u), 1.0)
        sp = np.where(sb_ok, rnd(sb_u), 1.0)
    else:
        rp, sp = ra_u, sb_u
    A2 = A1 / rp.astype(A1.dtype)[:, None]
    B2 = B1 / sp.astype(B1.dtype)[None, :]
    return A2, B2, rp, sp, ra_u, sb_u


def i_step(A1, B1, pow2: bool):
    """Inside step (Algorithm 2; Algorithm 3 'I step'): D = diag(sqrt(max_j|B'_kj| /
    max_i|A'_ik|)), A' <- A' D, B' <- D^{-1} B'.  Factor 1 where either maximum is zero."""
    amax = np.max(np.abs(A1), axis=0) if A1.shape[0] else np.zeros(A1.shape[1])
    bmax = np.max(np.abs(B1), axis=1) if B1.shape[1] else np.zeros(B1.shape[0])
    ok = _safe_positive(amax) & _safe_positive(bmax)
    a_ = np.where(ok, amax, 1.0).astype(np.float64)
    b_ = np.where(ok, bmax, 1.0).astype(np.float64)
    p_exact = np.where(ok, np.sqrt(b_ / a_), 1.0)
    p = np.where(ok, pow2_sqrt_ratio(b_, a_), 1.0) if pow2 else p_exact
    A2 = A1 * p.astype(A1.dtype)[None, :]
    B2 = B1 / p.astype(B1.dtype)[:, None]
    return A2, B2, p, p_exact


def scale(A: np.ndarray, B: np.ndarray, schedule: str, tau: Optional[float] = None,
          pow2: bool = True, o_round: str = "up") -> ScalingResult:
    """Run a sequence of O and I steps (e.g. 'O' = Algorithm 1, 'I' = Algorithm 2, 'OI',
    'IO', 'OIOI' = Algorithm 3 with 4 steps).  With tau, the stopping test of the
    stopping-criterion theorem (section 6.3) is
    applied to every step after the first O step, on the unrounded factors.  o_round: the
    power of two an O step rounds to (o_step)."""
    A1 = np.array(A, copy=True)
    B1 = np.array(B, copy=True)
    r = np.ones(A.shape[0])
    s = np.ones(B.shape[1])
    pc = np.ones(A.shape[1])
    res = ScalingResult(A1, B1, r, s)
    seen_o = False
    for kind in schedule:
        if kind == "O":
            A1, B1, rp, sp, ru, su = o_step(A1, B1, pow2, o_round)
            r = r * rp  # D_A <- D_A D_A'
            s = sp * s  # D_B <- D_B' D_B
            res.steps.append("O")
            res.factors.append((ru, su))
            test = seen_o and tau is not None
            seen_o = True
            if test:
                thr = (1.0 + tau) ** -0.5
                if np.min(ru, initial=1.0) >= thr and np.min(su, initial=1.0) >= thr:
                    res.stopped_early = True
                    break
        elif kind == "I":
            A1, B1, p, pe = i_step(A1, B1, pow2)
            pc = pc * p
            res.steps.append("I")
            res.factors.append((pe,))
            if seen_o and tau is not None:
                lo, hi = (1.0 + tau) ** -0.25, (1.0 + tau) ** 0.25
                if np.min(pe, initial=1.0) >= lo and np.max(pe, initial=1.0) <= hi:
                    res.stopped_early = True
                    break
        else:
            raise ValueError(kind)
    res.A, res.B, res.r, res.s, res.p = A1, B1, r, s, pc
    return res


SCHEDULES = {
    "none": "",
    "outside": "O",
    "inside": "I",
    "out_in": "OI",
    "in_out": "IO",
}


def schedule_for(mode: str, steps: int = 2) -> str:
    """Step sequence for a scaling mode; 'repeated' alternates starting with an O step."""
    if mode == "repeated":
        return "".join("O" if t % 2 == 0 else "I" for t in range(steps))
    return SCHEDULES[mode]


def scaled_fast(A, B, alg: Bilinear, depth: int, cutoff: int = 1, mode: str = "none",
                steps: int = 2, tau: Optional[float] = None, pow2: bool = True,
                leaf: Optional[Callable] = None, o_round: str = "up") -> np.ndarray:
    """C = D_A fast(A', B') D_B after the chosen scaling steps (Algorithms 1-3)."""
    sc = scale(A, B, schedule_for(mode, steps), tau, pow2, o_round)
    Cp = fast(sc.A, sc.B, alg, depth, cutoff, leaf)
    return (sc.r.astype(Cp.dtype)[:, None] * Cp) * sc.s.astype(Cp.dtype)[None, :]


def scaled_fast_every_level(A, B, rules: Sequence[Bilinear], cutoff: int = 1, mode: str = "none",
                            steps: int = 2, tau: Optional[float] = None, pow2: bool = True,
                            leaf: Optional[Callable] = None, trace: Optional[list] = None,
                            o_round: str = "up") -> np.ndarray:
    """Diagonal scaling applied at every level (a reading: the paper scales once, before the
    multiplication).  `rules` holds one rule per level (the same rule repeated for a
    stationary algorithm); the cutoff may stop the recursion earlier.  Every node of the
    recursion with at least one level below it runs the scaling steps (Algorithms 1-3) on its
    own operands, splits the scaled operands by one level of eq. (2) -- its children are
    handled the same way -- and multiplies its W-combined product by D_A on the left and D_B
    on the right.  Leaves are not scaled: power-of-two factors commute exactly with the
    classical product.  `trace`, when given, receives (level, ScalingResult) for every
    scaled node, in the order the recursion visits them."""
    leaf = leaf or classical
    m, k = A.shape
    n = B.shape[1]
    dims = [(a.M0, a.K0, a.N0) for a in rules]
    L = effective_depth(m, k, n, dims, cutoff)
    schedule = schedule_for(mode, steps)

    def node(X, Y, level):
        if level == L:
            return leaf(X, Y)
        sc = scale(X, Y, schedule, tau, pow2, o_round)
        if trace is not None:
            trace.append((level, sc))
        alg = rules[level]
        Cp = _rec(sc.A, sc.B, lambda path: alg, 1, (), lambda S, T: node(S, T, level + 1))
        return (sc.r.astype(Cp.dtype)[:, None] * Cp) * sc.s.astype(Cp.dtype)[None, :]

    if L == 0:  # the root is the only node: one scaling around the classical product
        sc = scale(A, B, schedule, tau, pow2, o_round)
        Cp = leaf(sc.A, sc.B)
        return (sc.r.astype(Cp.dtype)[:, None] * Cp) * sc.s.astype(Cp.dtype)[None, :]
    Mp, Kp, Np = padded_dims(m, k, n, dims[:L])
    Ap = np.zeros((Mp, Kp), dtype=A.dtype)
    Ap[:m, :k] = A
    Bp = np.zeros((Kp, Np), dtype=B.dtype)
    Bp[:k, :n] = B
    return np.ascontiguousarray(node(Ap, Bp, 0)[:m, :n])


# --------------------------------------------------------------------------------- bounds
def thm41_bound(K: int, K0: int, L: int, Q, E, u: float) -> float:
    """Theorem 4.1: (K/K0^L + Q L) (K/K0^L) E^L u, the bound on ||C^ - C|| / (||A|| ||B||)
    (max-norms) for L stationary levels over an inner dimension K (padded)."""
    kl = K / (K0 ** L)
    return (kl + float(Q) * L) * kl * float(E) ** L * u


def thm42_bound(K: int, levels: Sequence[Bilinear], u: float) -> float:
    """Theorem 4.2 (uniform non-stationary): (K/prod K0 + sum Q) (K/prod K0) prod E * u."""
    kl = K / float(np.prod([a.K0 for a in levels])) if levels else float(K)
    qs = sum(float(coeffs.quantities(a).Q) for a in levels)
    es = float(np.prod([float(coeffs.quantities(a).E) for a in levels])) if levels else 1.0
    return (kl + qs) * kl * es * u


def nonuniform_two_level_xi(top: Bilinear, child: Callable[[int], Bilinear]) -> List[Fraction]:
    """xi_k of section 4.5 for a two-level non-uniform tree: rule `top` at node [1] and rule
    child(r1) at node [2, r1].  Index k = (k1, k2) returned as k1 * (M0 N0) + k2."""
    qt = coeffs.quantities(top)
    out = []
    for k1 in range(len(top.W)):
        for k2 in range(len(top.W)):
            tot = Fraction(0)
            for r1 in range(top.R):
                w1 = abs(top.W[k1][r1])
                if w1 == 0:
                    continue
                c = child(r1)
                qc = coeffs.quantities(c)
                inner = sum((abs(c.W[k2][r2]) * qc.a[r2] * qc.b[r2] for r2 in range(c.R)), Fraction(0))
                tot += w1 * qt.a[r1] * qt.b[r1] * inner
            out.append(tot)
    return out


def stationary_stability_vector(alg: Bilinear, L: int) -> List[Fraction]:
    """Entries xi_k for L stationary levels: the L-fold Kronecker product of e (proof of
    Theorem 4.1)."""
    e = coeffs.quantities(alg).e
    out = [Fraction(1)]
    for _ in range(L):
        out = [x * y for x in out for y in e]
    return out


# ---------------------------------------------------------------------------- error measures
def maxabs(X: np.ndarray) -> float:
    return float(np.max(np.abs(X))) if X.size else 0.0


def normwise_error(Chat: np.ndarray, Cref: np.ndarray, A: np.ndarray, B: np.ndarray,
                   rows: Optional[Sequence[int]] = None) -> float:
    """max |C^ - C| / (max|A| max|B|) (max-norm, as in Theorem 4.1), over the given rows of
    C^ (Cref holds exactly those rows, in long double)."""
    sub = Chat if rows is None else Chat[np.asarray(rows)]
    diff = np.max(np.abs(sub.astype(np.longdouble) - Cref)) if sub.size else 0.0
    den = maxabs(A) * maxabs(B)
    return float(diff) / den if den > 0 else float(diff)


def componentwise_error(Chat: np.ndarray, Cref: np.ndarray, rows: Optional[Sequence[int]] = None) -> float:
    """max_ij |c^_ij - c_ij| / |c_ij| over entries with c_ij != 0 (section 6.5)."""
    sub = Chat if rows is None else Chat[np.asarray(rows)]
    nz = Cref != 0
    if not np.any(nz):
        return 0.0
    return float(np.max(np.abs(sub.astype(np.longdouble)[nz] - Cref[nz]) / np.abs(Cref[nz])))


def gradients(A: np.ndarray, B: np.ndarray, G: np.ndarray):
    """For the loss <G, A B>: dA = G B^T and dB = A^T G, by the classical algorithm."""
    return classical(G, np.ascontiguousarray(B.T)), classical(np.ascontiguousarray(A.T), G)
