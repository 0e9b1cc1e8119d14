"""Thin Python binding of the fastmm C ABI (include/fastmm.h).

Argument marshalling only: every step of the multiplication runs in the HIP kernels of
libfastmm.so.  PyTorch provides device memory (tensors, the caching allocator for the
workspace) and the current stream.  If the shared library is missing the import of this
module still works, but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastmm.so")

FASTMM_OK = 0

ALGOS = {
    "classical": 0,
    "strassen": 1,
    "winograd": 2,
    "f323": 3,
    "f332": 4,
    "f233": 5,
    "f442": 6,
    "f424": 7,
    "f244": 8,
    "laderman333": 9,
}
FUSION = {"off": 0, "auto": 1, "always": 2, "written": 3}
SCALE_MODES = {"none": 0, "outside": 1, "inside": 2, "out_in": 3, "in_out": 4, "repeated": 5}
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16x3": 4, "f16x3": 5, "bf16x6": 6}


class FastmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fastmm error {status}: {msg}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("k", ctypes.c_int64), ("n", ctypes.c_int64)]


class _ProblemEx(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("transA", ctypes.c_int), ("B", ctypes.c_void_p),
                ("ldb", ctypes.c_int64), ("transB", ctypes.c_int), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64)]


class _GradProblem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("G", ctypes.c_void_p), ("dA", ctypes.c_void_p),
                ("dB", ctypes.c_void_p), ("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64)]


class _Scaling(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("steps", ctypes.c_int), ("tau", ctypes.c_double),
                ("per_level", ctypes.c_int), ("o_round", ctypes.c_int)]


O_ROUNDS = {"up": 0, "nearest": 1}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libfastmm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: its HIP runtime (libamdhip64.so, SONAME libamdhip64.so.7) must be the
        # one in the process before libfastmm.so is loaded, so that the library's dependency on
        # libamdhip64.so.7 binds to it.  Loading libfastmm.so first would pull in a second
        # HIP/HSA runtime from /opt/rocm next to torch's, and the two contend for the device.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1507_00687_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, vp, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
        pi32, pi64, pd = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        L.fastmm_algo_register.argtypes = [i32, i32, i32, i32, pi64, pi64, pi64, i32, pi32]
        L.fastmm_algo_info.argtypes = [i32, pi32, pi32, pi32, pi32, pi32, pd, pd]
        L.fastmm_algo_coeffs.argtypes = [i32, pd, pd, pd]
        L.fastmm_algo_stability.argtypes = [i32, i32, pd, pd, pd]
        L.fastmm_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, ctypes.POINTER(_Scaling), i32]
        L.fastmm_plan_destroy.argtypes = [vp]
        L.fastmm_plan_shape.argtypes = [vp, i64, i64, i64, pi32, pi64, pi64, pi64]
        L.fastmm_workspace_size.argtypes = [vp, i64, i64, i64, ctypes.POINTER(sz)]
        L.fastmm_plan_set_fusion.argtypes = [vp, i32]
        L.fastmm_plan_set_tree.argtypes = [vp, pi32, i64]
        L.fastmm_plan_set_levels.argtypes = [vp, pi32, i32]
        L.fastmm_plan_set_tile.argtypes = [vp, i32]
        L.fastmm_plan_path.argtypes = [vp, i64, i64, i64, i32, i32, pi32]
        L.fastmm_gemm.argtypes = [vp, vp, vp, vp, i64, i64, i64, vp, sz, vp]
        L.fastmm_gemm_ex.argtypes = [vp, vp, i64, i32, vp, i64, i32, vp, i64, i64, i64, i64, vp, sz, vp]
        L.fastmm_gemm_noalloc.argtypes = [vp, vp, vp, vp, i64, i64, i64, vp]
        L.fastmm_scaling_exponents.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, vp, vp, sz, vp]
        L.fastmm_task_table.argtypes = [vp, i32, pi64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fastmm_batched_workspace_size.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Problem), i32,
                                                     ctypes.POINTER(sz)]
        L.fastmm_gemm_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Problem), i32, vp, sz, vp]
        L.fastmm_batched_ex_workspace_size.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_ProblemEx), i32,
                                                        ctypes.POINTER(sz)]
        L.fastmm_gemm_batched_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_ProblemEx), i32, vp, sz, vp]
        L.fastmm_backward_batched_workspace_size.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_GradProblem), i32,
                                                              ctypes.POINTER(sz)]
        L.fastmm_gemm_backward_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_GradProblem), i32, vp, sz, vp]
        L.fastmm_backward_workspace_size.argtypes = [vp, i64, i64, i64, ctypes.POINTER(sz)]
        L.fastmm_gemm_backward.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, i64, vp, sz, vp]
        L.fastmm_profile_enable.argtypes = [i32]
        L.fastmm_profile_read.argtypes = [pd, pd, pd, pd, pi32]
        L.fastmm_strerror.argtypes = [i32]
        L.fastmm_strerror.restype = ctypes.c_char_p
        L.fastmm_last_error.restype = ctypes.c_char_p
        for name in ("fastmm_algo_register", "fastmm_algo_info", "fastmm_algo_coeffs", "fastmm_plan_create",
                     "fastmm_plan_destroy", "fastmm_plan_shape", "fastmm_workspace_size", "fastmm_gemm",
                     "fastmm_gemm_ex", "fastmm_scaling_exponents", "fastmm_profile_enable", "fastmm_profile_read", "fastmm_task_table",
                     "fastmm_backward_workspace_size", "fastmm_gemm_backward", "fastmm_batched_workspace_size",
                     "fastmm_gemm_batched", "fastmm_plan_set_fusion", "fastmm_plan_path", "fastmm_plan_set_tree",
                     "fastmm_algo_stability", "fastmm_plan_set_levels", "fastmm_plan_set_tile",
                     "fastmm_gemm_noalloc", "fastmm_batched_ex_workspace_size", "fastmm_gemm_batched_ex",
                     "fastmm_backward_batched_workspace_size", "fastmm_gemm_backward_batched"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != FASTMM_OK:
        L = lib()
        msg = L.fastmm_last_error().decode() or L.fastmm_strerror(status).decode()
        raise FastmmError(status, msg)


def _id(table: dict, key) -> int:
    return table[key] if isinstance(key, str) else int(key)


# --------------------------------------------------------------------------- algorithms
def fastmm_algo_info(algo) -> dict:
    vals = [ctypes.c_int() for _ in range(5)]
    Q, E = ctypes.c_double(), ctypes.c_double()
    _check(lib().fastmm_algo_info(_id(ALGOS, algo), *[ctypes.byref(v) for v in vals], ctypes.byref(Q),
                                  ctypes.byref(E)))
    M0, K0, N0, R, nnz = (v.value for v in vals)
    return {"M0": M0, "K0": K0, "N0": N0, "R": R, "nnz": nnz, "Q": Q.value, "E": E.value}


def fastmm_algo_stability(algo, levels: int = 1) -> dict:
    """Stability exponent, fraction of classical multiplications and relative instability of a
    rule at `levels` levels (the library computes them)."""
    st, fr, ri = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().fastmm_algo_stability(_id(ALGOS, algo), levels, ctypes.byref(st), ctypes.byref(fr),
                                       ctypes.byref(ri)))
    return {"stab_exp": st.value, "flops_frac": fr.value, "rel_instability": ri.value}


def fastmm_algo_coeffs(algo):
    import numpy as np

    info = fastmm_algo_info(algo)
    M0, K0, N0, R = info["M0"], info["K0"], info["N0"], info["R"]
    U = np.zeros((M0 * K0, R))
    V = np.zeros((K0 * N0, R))
    W = np.zeros((M0 * N0, R))
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib().fastmm_algo_coeffs(_id(ALGOS, algo), U.ctypes.data_as(P), V.ctypes.data_as(P),
                                    W.ctypes.data_as(P)))
    return U, V, W


def fastmm_algo_register(M0, K0, N0, R, num_U, num_V, num_W, log2_den=0) -> int:
    import numpy as np

    arrs = [np.ascontiguousarray(x, dtype=np.int64) for x in (num_U, num_V, num_W)]
    out = ctypes.c_int()
    P = ctypes.POINTER(ctypes.c_int64)
    _check(lib().fastmm_algo_register(M0, K0, N0, R, *[a.ctypes.data_as(P) for a in arrs], log2_den,
                                      ctypes.byref(out)))
    return out.value


# --------------------------------------------------------------------------------- plans
class Plan:
    """A fastmm plan: algorithm, recursion depth, cutoff, scaling procedure, precision.

    per_level=True runs the scaling steps also on the operands of every inner node of the
    recursion (scaling at every level), not only on A and B."""

    def __init__(self, algo="strassen", depth: int = 1, cutoff: int = 1, scaling: str = "none",
                 steps: int = 2, tau: float = 0.0, precision: str = "f64", fuse="auto",
                 per_level: bool = False, o_round: str = "up"):
        self.algo, self.depth, self.cutoff = algo, depth, cutoff
        self.scaling, self.steps, self.tau, self.precision = scaling, steps, tau, precision
        self.fuse, self.per_level, self.o_round = fuse, per_level, o_round
        self._h = ctypes.c_void_p()
        sc = _Scaling(_id(SCALE_MODES, scaling), steps, tau, int(bool(per_level)), _id(O_ROUNDS, o_round))
        _check(lib().fastmm_plan_create(ctypes.byref(self._h), _id(ALGOS, algo), depth, cutoff, ctypes.byref(sc),
                                        _id(PRECISIONS, precision)))
        mode = FUSION[fuse] if isinstance(fuse, str) else (FUSION["auto"] if fuse else FUSION["off"])
        if mode != FUSION["auto"]:
            _check(lib().fastmm_plan_set_fusion(self._h, mode))

    def set_tile(self, tile: int) -> "Plan":
        """Split precisions: the limb GEMM's output tile, 0 (by the leaf-block shape), 128 or 256."""
        _check(lib().fastmm_plan_set_tile(self._h, int(tile)))
        self.tile = int(tile)
        return self

    def set_tree(self, node_algos) -> "Plan":
        """Non-uniform recursion: one rule (name or id) per internal node, breadth first
        (node [l, r_1 .. r_{l-1}] at (R^(l-1) - 1)/(R - 1) + (r_1 .. r_{l-1} in base R)); an
        empty list restores the plan's rule everywhere."""
        ids = [_id(ALGOS, a) for a in node_algos]
        arr = (ctypes.c_int32 * max(len(ids), 1))(*ids)
        _check(lib().fastmm_plan_set_tree(self._h, arr, len(ids)))
        self.tree = list(node_algos)
        return self

    def set_levels(self, level_algos) -> "Plan":
        """Uniform non-stationary recursion: one rule (name or id) per level, outermost first
        (as many as the plan's depth); an empty list restores the plan's rule at every level."""
        ids = [_id(ALGOS, a) for a in level_algos]
        arr = (ctypes.c_int32 * max(len(ids), 1))(*ids)
        _check(lib().fastmm_plan_set_levels(self._h, arr, len(ids)))
        self.levels = list(level_algos)
        return self

    def path(self, m: int, k: int, n: int, transA: bool = False, transB: bool = False) -> str:
        """'leaf', 'fused', 'every_level', 'written' or 'fused_loads': the execution path of an
        m x k by k x n product."""
        v = ctypes.c_int()
        _check(lib().fastmm_plan_path(self._h, m, k, n, int(transA), int(transB), ctypes.byref(v)))
        return {0: "leaf", 1: "fused", 2: "every_level", 3: "written", 4: "fused_loads"}[v.value]

    @property
    def handle(self):
        return self._h

    def shape(self, m: int, k: int, n: int) -> Tuple[int, int, int, int]:
        L = ctypes.c_int()
        Mp, Kp, Np = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fastmm_plan_shape(self._h, m, k, n, ctypes.byref(L), ctypes.byref(Mp), ctypes.byref(Kp),
                                       ctypes.byref(Np)))
        return L.value, Mp.value, Kp.value, Np.value

    def workspace_size(self, m: int, k: int, n: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().fastmm_workspace_size(self._h, m, k, n, ctypes.byref(b)))
        return b.value

    @property
    def dtype(self):
        import torch

        return torch.float64 if self.precision == "f64" else torch.float32

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.fastmm_plan_destroy(h)
            self._h = ctypes.c_void_p()


# ------------------------------------------------------------------------ multiplication
def _stream_ptr(stream) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _workspace(plan: Plan, m, k, n, device, workspace):
    import torch

    need = plan.workspace_size(m, k, n)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    return workspace, need


def fastmm_gemm(plan: Plan, A, B, C=None, workspace=None, stream=None):
    """C = A @ B on the GPU (A: m x k, B: k x n, contiguous row-major CUDA tensors)."""
    import torch

    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if A.dtype != plan.dtype or B.dtype != plan.dtype:
        raise TypeError(f"plan precision {plan.precision} takes {plan.dtype} operands")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("operands must be on the GPU")
    A = A.contiguous()
    B = B.contiguous()
    if C is None:
        C = torch.empty((m, n), dtype=plan.dtype, device=A.device)
    ws, need = _workspace(plan, m, k, n, A.device, workspace)
    _check(lib().fastmm_gemm(plan.handle, A.data_ptr(), B.data_ptr(), C.data_ptr(), m, k, n, ws.data_ptr(),
                             ws.numel(), _stream_ptr(stream)))
    return C


def fastmm_gemm_noalloc(plan: Plan, A, B, C, stream=None):
    """C = A @ B with the library's fixed scratch array as workspace (no device allocation in
    the call; C must be given).  The plan needs one earlier fastmm_gemm call at this shape on
    the device (which uploads its task tables)."""
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if A.dtype != plan.dtype or B.dtype != plan.dtype or C.dtype != plan.dtype:
        raise TypeError(f"plan precision {plan.precision} takes {plan.dtype} operands")
    if not (A.is_cuda and B.is_cuda and C.is_cuda):
        raise ValueError("operands must be on the GPU")
    if not (A.is_contiguous() and B.is_contiguous() and C.is_contiguous()) or tuple(C.shape) != (m, n):
        raise ValueError("contiguous operands and an m x n C are required")
    _check(lib().fastmm_gemm_noalloc(plan.handle, A.data_ptr(), B.data_ptr(), C.data_ptr(), m, k, n,
                                     _stream_ptr(stream)))
    return C


def fastmm_gemm_ex(plan: Plan, A, transA: bool, B, transB: bool, C=None, workspace=None, stream=None):
    """C = op(A) @ op(B) with op(X) = X.T when the flag is set (X stored row-major)."""
    import torch

    m, k = (A.shape[1], A.shape[0]) if transA else (A.shape[0], A.shape[1])
    kb, n = (B.shape[1], B.shape[0]) if transB else (B.shape[0], B.shape[1])
    if k != kb:
        raise ValueError("inner dimensions differ")
    if A.stride(1) != 1 or B.stride(1) != 1:
        raise ValueError("operands need contiguous rows")
    if C is None:
        C = torch.empty((m, n), dtype=plan.dtype, device=A.device)
    ws, need = _workspace(plan, m, k, n, A.device, workspace)
    _check(lib().fastmm_gemm_ex(plan.handle, A.data_ptr(), A.stride(0), int(bool(transA)), B.data_ptr(),
                                B.stride(0), int(bool(transB)), C.data_ptr(), C.stride(0), m, k, n, ws.data_ptr(),
                                ws.numel(), _stream_ptr(stream)))
    return C


def _batch_problems(plans, As, Bs, Cs):
    count = len(As)
    probs = (_Problem * max(count, 1))()
    for i, (a, b, c) in enumerate(zip(As, Bs, Cs)):
        if a.shape[1] != b.shape[0]:
            raise ValueError(f"problem {i}: inner dimensions differ")
        if a.dtype != plans[i].dtype or b.dtype != plans[i].dtype:
            raise TypeError(f"problem {i}: operands must be {plans[i].dtype}")
        probs[i] = _Problem(a.data_ptr(), b.data_ptr(), c.data_ptr() if c is not None else 0, a.shape[0], a.shape[1],
                            b.shape[1])
    handles = (ctypes.c_void_p * max(count, 1))(*[p.handle.value for p in plans])
    return probs, handles


def fastmm_batched_workspace_size(plans, As, Bs) -> int:
    """Workspace bytes fastmm_gemm_batched needs for these problems."""
    if not (len(As) == len(Bs) == len(plans)):
        raise ValueError("plans, As and Bs must have the same length")
    probs, handles = _batch_problems(plans, As, Bs, [None] * len(As))
    need = ctypes.c_size_t()
    _check(lib().fastmm_batched_workspace_size(handles, probs, len(As), ctypes.byref(need)))
    return need.value


def fastmm_gemm_batched(plans, As, Bs, Cs=None, workspace=None, stream=None):
    """C_i = A_i @ B_i for all i with plans[i]; one persistent leaf launch for the batch."""
    import torch

    count = len(As)
    if not (len(Bs) == count and len(plans) == count):
        raise ValueError("plans, As and Bs must have the same length")
    As = [a.contiguous() for a in As]
    Bs = [b.contiguous() for b in Bs]
    if Cs is None:
        Cs = [torch.empty((a.shape[0], b.shape[1]), dtype=a.dtype, device=a.device) for a, b in zip(As, Bs)]
    probs, handles = _batch_problems(plans, As, Bs, Cs)
    need = ctypes.c_size_t()
    _check(lib().fastmm_batched_workspace_size(handles, probs, count, ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=As[0].device if count else "cuda")
    _check(lib().fastmm_gemm_batched(handles, probs, count, workspace.data_ptr(), workspace.numel(),
                                     _stream_ptr(stream)))
    return Cs


def fastmm_gemm_batched_ex(plans, As, Bs, transA=None, transB=None, Cs=None, workspace=None, stream=None):
    """C_i = op(A_i) @ op(B_i) for all i with plans[i], op(X) = X.T where trans*[i] is set; the
    stored operands may be row-strided 2-D views (unit column stride).  One launch of the
    products for the batch."""
    import torch

    count = len(As)
    if not (len(Bs) == count and len(plans) == count):
        raise ValueError("plans, As and Bs must have the same length")
    transA = list(transA) if transA is not None else [False] * count
    transB = list(transB) if transB is not None else [False] * count
    probs = (_ProblemEx * max(count, 1))()
    outs = []
    for i in range(count):
        a, b = As[i], Bs[i]
        for x in (a, b):
            if x.dim() != 2 or x.stride(1) != 1:
                raise ValueError(f"problem {i}: operands must be 2-D with unit column stride")
            if x.dtype != plans[i].dtype:
                raise TypeError(f"problem {i}: operands must be {plans[i].dtype}")
        m, k = (a.shape[1], a.shape[0]) if transA[i] else (a.shape[0], a.shape[1])
        kb, n = (b.shape[1], b.shape[0]) if transB[i] else (b.shape[0], b.shape[1])
        if k != kb:
            raise ValueError(f"problem {i}: inner dimensions differ")
        c = Cs[i] if Cs is not None else torch.empty((m, n), dtype=a.dtype, device=a.device)
        if c.dim() != 2 or c.stride(1) != 1 or tuple(c.shape) != (m, n):
            raise ValueError(f"problem {i}: C must be an {m} x {n} view with unit column stride")
        outs.append(c)
        probs[i] = _ProblemEx(a.data_ptr(), max(a.stride(0), 1), int(bool(transA[i])), b.data_ptr(),
                              max(b.stride(0), 1), int(bool(transB[i])), c.data_ptr(), max(c.stride(0), 1), m, k, n)
    handles = (ctypes.c_void_p * max(count, 1))(*[p.handle.value for p in plans])
    need = ctypes.c_size_t()
    _check(lib().fastmm_batched_ex_workspace_size(handles, probs, count, ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=As[0].device if count else "cuda")
    _check(lib().fastmm_gemm_batched_ex(handles, probs, count, workspace.data_ptr(), workspace.numel(),
                                        _stream_ptr(stream)))
    return outs


def fastmm_gemm_backward_batched(plans, As, Bs, Gs, need_dA: bool = True, need_dB: bool = True, workspace=None,
                                 stream=None):
    """[(dA_i, dB_i)] = [(G_i B_i^T, A_i^T G_i)] for all i with plans[i]: the gradient products of
    the whole batch in one launch (None where not needed)."""
    import torch

    count = len(As)
    if not (len(Bs) == count and len(Gs) == count and len(plans) == count):
        raise ValueError("plans, As, Bs and Gs must have the same length")
    As = [a.contiguous() for a in As]
    Bs = [b.contiguous() for b in Bs]
    Gs = [g.contiguous() for g in Gs]
    probs = (_GradProblem * max(count, 1))()
    outs = []
    for i in range(count):
        a, b, g = As[i], Bs[i], Gs[i]
        m, k = a.shape
        n = b.shape[1]
        if b.shape[0] != k or tuple(g.shape) != (m, n):
            raise ValueError(f"problem {i}: shapes do not match")
        for x in (a, b, g):
            if x.dtype != plans[i].dtype:
                raise TypeError(f"problem {i}: operands must be {plans[i].dtype}")
        dA = torch.empty((m, k), dtype=a.dtype, device=a.device) if need_dA else None
        dB = torch.empty((k, n), dtype=a.dtype, device=a.device) if need_dB else None
        outs.append((dA, dB))
        probs[i] = _GradProblem(a.data_ptr(), b.data_ptr(), g.data_ptr(), dA.data_ptr() if dA is not None else None,
                                dB.data_ptr() if dB is not None else None, m, k, n)
    handles = (ctypes.c_void_p * max(count, 1))(*[p.handle.value for p in plans])
    need = ctypes.c_size_t()
    _check(lib().fastmm_backward_batched_workspace_size(handles, probs, count, ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=As[0].device if count else "cuda")
    _check(lib().fastmm_gemm_backward_batched(handles, probs, count, workspace.data_ptr(), workspace.numel(),
                                              _stream_ptr(stream)))
    return outs


def fastmm_gemm_backward(plan: Plan, A, B, G, need_dA: bool = True, need_dB: bool = True, workspace=None,
                         stream=None):
    """(dA, dB) = (G B^T, A^T G) through the transposed rotations of the plan's rule (None where not
    needed)."""
    import torch

    m, k = A.shape
    n = B.shape[1]
    A, B, G = A.contiguous(), B.contiguous(), G.contiguous()
    dA = torch.empty((m, k), dtype=plan.dtype, device=A.device) if need_dA else None
    dB = torch.empty((k, n), dtype=plan.dtype, device=A.device) if need_dB else None
    b = ctypes.c_size_t()
    _check(lib().fastmm_backward_workspace_size(plan.handle, m, k, n, ctypes.byref(b)))
    if workspace is None:
        workspace = torch.empty(max(b.value, 1), dtype=torch.uint8, device=A.device)
    _check(lib().fastmm_gemm_backward(plan.handle, A.data_ptr(), B.data_ptr(), G.data_ptr(),
                                      dA.data_ptr() if dA is not None else None,
                                      dB.data_ptr() if dB is not None else None, m, k, n, workspace.data_ptr(),
                                      workspace.numel(), _stream_ptr(stream)))
    return dA, dB


def fastmm_scaling_exponents(plan: Plan, A, B, workspace=None, stream=None):
    """Power-of-two exponents (ea, eb, ep) of the plan's scaling of (A, B), int32 tensors."""
    import torch

    m, k = A.shape
    n = B.shape[1]
    ea = torch.empty(m, dtype=torch.int32, device=A.device)
    eb = torch.empty(n, dtype=torch.int32, device=A.device)
    ep = torch.empty(k, dtype=torch.int32, device=A.device)
    ws, need = _workspace(plan, m, k, n, A.device, workspace)
    _check(lib().fastmm_scaling_exponents(plan.handle, A.contiguous().data_ptr(), B.contiguous().data_ptr(), m, k,
                                          n, ea.data_ptr(), eb.data_ptr(), ep.data_ptr(), ws.data_ptr(),
                                          ws.numel(), _stream_ptr(stream)))
    return ea, eb, ep


def fastmm_task_table(plan: "Plan", levels: int) -> dict:
    """The composite leaf task table of `plan` at `levels` levels, as numpy arrays."""
    import numpy as np

    counts = (ctypes.c_int64 * 5)()
    _check(lib().fastmm_task_table(plan.handle, levels, counts, *([None] * 8)))
    nl, na, nb, nblk, nd = list(counts)
    out = {
        "leaves": np.zeros((nl, 4), np.int32), "asrc": np.zeros((na, 2), np.int32), "acoef": np.zeros(na),
        "bsrc": np.zeros((nb, 2), np.int32), "bcoef": np.zeros(nb), "bdest": np.zeros((nblk, 2), np.int32),
        "dest_leaf": np.zeros(nd, np.int32), "dest_coef": np.zeros(nd),
    }
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().fastmm_task_table(plan.handle, levels, counts, ptr(out["leaves"]), ptr(out["asrc"]),
                                   ptr(out["acoef"]), ptr(out["bsrc"]), ptr(out["bcoef"]), ptr(out["bdest"]),
                                   ptr(out["dest_leaf"]), ptr(out["dest_coef"])))
    return out


def fastmm_profile_enable(enable: bool = True) -> None:
    _check(lib().fastmm_profile_enable(int(bool(enable))))


def fastmm_profile_read() -> dict:
    """Summed milliseconds per phase of the profiled calls since the last read."""
    a, f, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_int()
    _check(lib().fastmm_profile_read(ctypes.byref(a), ctypes.byref(f), ctypes.byref(b), ctypes.byref(c),
                                     ctypes.byref(n)))
    return {"scaling_ms": a.value, "form_ms": f.value, "leaf_ms": b.value, "combine_ms": c.value, "calls": n.value}


def matmul(A, B, plan: Optional[Plan] = None, **plan_kwargs):
    """Convenience: C = A @ B through a (new or given) plan."""
    plan = plan or Plan(**plan_kwargs)
    return fastmm_gemm(plan, A, B)
