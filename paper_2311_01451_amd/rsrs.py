"""Thin Python binding of ``include/rsrs.h`` (ctypes).

Argument marshalling only: every step of the method runs in ``librsrs.so``.
PyTorch supplies device memory (``torch.float64`` CUDA/HIP tensors, or
``torch.float32`` for FP32 sketches, row-major N x w with ``stride(0)`` as
leading dimension) and the current HIP stream.
The functions carry the names of the C entry points; small handle classes own
the C handles and free them on garbage collection.

If ``librsrs.so`` is missing this module raises on first use: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsrs.so")
_lib = None

RSRS_OP_LOG2D = 1
RSRS_OP_INVR3D = 2
RSRS_OP_LOG2D_SKEW = 3
RSRS_OP_LOG2D_FIRST = 4
RSRS_PREC_F64 = 0
RSRS_ID_SUM, RSRS_ID_CONCAT = 0, 1
RSRS_PREC_F32_MIXED = 1
RSRS_F64 = 0
RSRS_F32 = 1
RSRS_BF16 = 2

STATUS = {0: "RSRS_OK", 1: "RSRS_E_INVALID", 2: "RSRS_E_SAMPLES", 3: "RSRS_E_SINGULAR",
          4: "RSRS_E_CALLBACK", 5: "RSRS_E_NUMERIC", 6: "RSRS_E_NOMEM", 7: "RSRS_E_HIP",
          8: "RSRS_E_UNSUPPORTED", 9: "RSRS_E_TIMEOUT"}


class RSRSError(RuntimeError):
    def __init__(self, status: int, message: str, required_s: int = -1):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.required_s = required_s


class TreeOpts(C.Structure):
    _fields_ = [("dim", C.c_int), ("leaf_size", C.c_int), ("qbits", C.c_int),
                ("root_lo", C.c_double * 3), ("root_side", C.c_double)]


class TreeInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("nlevels", C.c_int), ("qbits", C.c_int),
                ("n", C.c_int64), ("nbox", C.c_int64),
                ("level", C.POINTER(C.c_int32)), ("coords", C.POINTER(C.c_int32)),
                ("parent", C.POINTER(C.c_int64)), ("is_leaf", C.POINTER(C.c_uint8)),
                ("pt_begin", C.POINTER(C.c_int64)), ("pt_end", C.POINTER(C.c_int64)),
                ("perm", C.POINTER(C.c_int64))]


class FactorOpts(C.Structure):
    _fields_ = [("k", C.c_int), ("p", C.c_int), ("precision", C.c_int), ("reproject", C.c_int),
                ("symmetric", C.c_int), ("id_mode", C.c_int), ("rank_tol", C.c_double),
                ("col_subset", C.c_int)]


class FactorInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("s", C.c_int64), ("k", C.c_int64), ("nboxes", C.c_int64),
                ("root_size", C.c_int64), ("stored_values", C.c_int64), ("stored_bytes", C.c_int64),
                ("precision", C.c_int), ("flops", C.c_double), ("factor_ms", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_batch_cols", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("solves_done", C.c_int64), ("factors_done", C.c_int64), ("batches", C.c_int64),
                ("cols_done", C.c_int64), ("hbm_in_use", C.c_int64), ("hbm_peak", C.c_int64),
                ("resident_factors", C.c_int64), ("queued_solves", C.c_int64),
                ("queued_factors", C.c_int64), ("solve_p50_ms", C.c_double),
                ("solve_p99_ms", C.c_double), ("factor_p50_ms", C.c_double),
                ("factor_p99_ms", C.c_double), ("refined_batches", C.c_int64),
                ("refine_steps", C.c_int64), ("max_relres", C.c_double)]


class ProfileEntry(C.Structure):
    _fields_ = [("tag", C.c_char * 48), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


MATVEC_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int64,
                        C.c_void_p, C.c_int64, C.c_void_p)

EXPORTS = [
    "rsrs_status_string", "rsrs_last_error", "rsrs_last_required_s", "rsrs_build_tree",
    "rsrs_tree_destroy", "rsrs_tree_get_info", "rsrs_tree_neighbours", "rsrs_tree_schedule",
    "rsrs_samples_required", "rsrs_work_model", "rsrs_gemm_autotune", "rsrs_gemm_autotune_workload",
    "rsrs_gemm_tile_override", "rsrs_op_library_gemm", "rsrs_op_create_kernel", "rsrs_op_create_dense",
    "rsrs_op_create_poisson7", "rsrs_op_matvec", "rsrs_op_destroy", "rsrs_samples_wrap",
    "rsrs_sample", "rsrs_sample_symmetric", "rsrs_samples_wrap_symmetric", "rsrs_samples_destroy", "rsrs_gaussian", "rsrs_factor", "rsrs_factor_redraw", "rsrs_factor_batched",
    "rsrs_factor_destroy", "rsrs_release_cached",
    "rsrs_factor_get_info", "rsrs_factor_box_sizes", "rsrs_factor_box_copy",
    "rsrs_factor_root_copy", "rsrs_solve", "rsrs_solve_noalloc", "rsrs_apply", "rsrs_solve_refine", "rsrs_solve_gmres",
    "rsrs_profile_enable", "rsrs_profile_filter", "rsrs_profile_reset", "rsrs_profile_read", "rsrs_solve_graphs",
    "rsrs_server_create", "rsrs_server_destroy", "rsrs_server_add_factor",
    "rsrs_server_release_factor", "rsrs_server_set_refine", "rsrs_server_submit_solve", "rsrs_server_submit_factor",
    "rsrs_server_wait", "rsrs_server_get_stats",
]


def lib():
    """Load librsrs.so (once); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2311_01451_amd.build` "
                           "(there is no non-HIP fallback)")
    # PyTorch's wheel carries its own HIP runtime beside the one this library
    # links; the device tensors passed in are torch's, and torch's runtime
    # finds no device once the other one has opened it, so it goes first.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    P = C.POINTER
    sig = {
        "rsrs_status_string": (C.c_char_p, [C.c_int]),
        "rsrs_last_error": (C.c_char_p, []),
        "rsrs_last_required_s": (i64, []),
        "rsrs_build_tree": (i32, [P(C.c_double), i64, P(TreeOpts), P(vp)]),
        "rsrs_tree_destroy": (None, [vp]),
        "rsrs_tree_get_info": (i32, [vp, P(TreeInfo)]),
        "rsrs_tree_neighbours": (i32, [vp, i32, P(i64), P(P(i64)), P(P(i64)), P(P(i64))]),
        "rsrs_tree_schedule": (i32, [vp, i32, P(C.c_int32), P(i64), P(i64), P(i64)]),
        "rsrs_samples_required": (i64, [vp, i32, i32]),
        "rsrs_work_model": (i32, [vp, P(FactorOpts), i64, i32, P(dbl), P(dbl), P(i64)]),
        "rsrs_gemm_autotune": (i32, [C.c_char_p, P(i64), P(i64)]),
        "rsrs_gemm_tile_override": (i32, [i32]),
        "rsrs_op_library_gemm": (i32, [i32]),
        "rsrs_gemm_autotune_workload": (i32, [vp, P(FactorOpts), i64, P(i64), P(i64)]),
        "rsrs_op_create_kernel": (i32, [i32, P(C.c_double), i64, i32, dbl, dbl, P(vp)]),
        "rsrs_op_create_dense": (i32, [vp, i64, i64, P(vp)]),
        "rsrs_op_create_poisson7": (i32, [i32, P(C.c_double), P(vp)]),
        "rsrs_op_matvec": (i32, [vp, i32, i32, i64, vp, i64, vp, i64, vp]),
        "rsrs_op_destroy": (None, [vp]),
        "rsrs_samples_wrap": (i32, [vp, i32, vp, vp, vp, vp, i64, i64, vp, P(vp)]),
        "rsrs_sample": (i32, [vp, vp, vp, i64, C.c_uint64, i32, vp, P(vp)]),
        "rsrs_sample_symmetric": (i32, [vp, vp, vp, i64, C.c_uint64, i32, vp, P(vp)]),
        "rsrs_samples_wrap_symmetric": (i32, [vp, i32, vp, vp, i64, i64, vp, P(vp)]),
        "rsrs_samples_destroy": (None, [vp]),
        "rsrs_gaussian": (i32, [vp, i64, i64, i64, C.c_uint64, C.c_uint32, vp]),
        "rsrs_factor": (i32, [vp, vp, P(FactorOpts), vp, P(vp)]),
        "rsrs_factor_redraw": (i32, [vp, vp, vp, i64, C.c_uint64, i32, P(FactorOpts), vp, P(vp)]),
        "rsrs_factor_batched": (i32, [i64, P(vp), P(vp), P(FactorOpts), vp, P(vp)]),
        "rsrs_factor_destroy": (None, [vp]),
        "rsrs_factor_get_info": (i32, [vp, P(FactorInfo)]),
        "rsrs_factor_box_sizes": (i32, [vp, i64, P(i64), P(C.c_int32), P(C.c_int32), P(i64),
                                        P(i64), P(i64), P(i64)]),
        "rsrs_factor_box_copy": (i32, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]),
        "rsrs_factor_root_copy": (i32, [vp, P(i64), vp, vp]),
        "rsrs_solve": (i32, [vp, i32, i64, vp, i64, vp, i64, vp]),
        "rsrs_apply": (i32, [vp, i32, i64, vp, i64, vp, i64, vp]),
        "rsrs_solve_noalloc": (i32, [vp, i32, i64, vp, i64, vp, i64, vp]),
        "rsrs_solve_refine": (i32, [vp, vp, vp, i64, vp, i64, vp, i64, dbl, i32, P(dbl),
                                    P(i32), vp]),
        "rsrs_solve_gmres": (i32, [vp, vp, vp, i64, vp, i64, vp, i64, dbl, i32, i32, P(dbl), P(i32), vp]),
        "rsrs_server_create": (i32, [P(ServerOpts), P(vp)]),
        "rsrs_server_destroy": (None, [vp]),
        "rsrs_server_add_factor": (i32, [vp, vp, P(i64)]),
        "rsrs_server_release_factor": (i32, [vp, i64]),
        "rsrs_server_set_refine": (i32, [vp, i64, vp, vp, dbl, i32]),
        "rsrs_server_set_refine": (i32, [vp, i64, vp, vp, dbl, i32]),
        "rsrs_server_submit_solve": (i32, [vp, i64, i64, vp, i64, vp, i64, P(i64)]),
        "rsrs_server_submit_factor": (i32, [vp, vp, vp, vp, i64, C.c_uint64, i32, P(FactorOpts),
                                            P(i64)]),
        "rsrs_server_wait": (i32, [vp, i64, dbl, P(i64), P(dbl)]),
        "rsrs_server_get_stats": (i32, [vp, i32, P(ServerStats)]),
        "rsrs_profile_enable": (None, [i32]),
        "rsrs_release_cached": (None, []),
        "rsrs_solve_graphs": (None, [i32]),
        "rsrs_profile_reset": (None, []),
        "rsrs_profile_filter": (None, [C.c_char_p]),
        "rsrs_profile_read": (i32, [P(ProfileEntry), i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        L = lib()
        msg = L.rsrs_last_error().decode()
        raise RSRSError(st, msg, int(L.rsrs_last_required_s()) if st == 2 else -1)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(int(s.cuda_stream))


def _dev(t, name="tensor", dtypes=("float64",)):
    import torch
    ok = isinstance(t, torch.Tensor) and t.is_cuda and str(t.dtype).replace("torch.", "") in dtypes
    if not ok:
        raise TypeError(f"{name} must be a {' or '.join(dtypes)} device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise TypeError(f"{name} must be 2-D row-major (stride(1) == 1)")
    return C.c_void_p(t.data_ptr()), t.stride(0)


def _dtype_code(t) -> int:
    import torch
    return RSRS_F32 if t.dtype == torch.float32 else RSRS_F64


# --------------------------------------------------------------------------- tree
class Tree:
    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.rsrs_tree_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        ti = TreeInfo()
        _check(lib().rsrs_tree_get_info(self._h, C.byref(ti)))
        nb, d, n = ti.nbox, ti.dim, ti.n
        arr = lambda p, cnt, dt: np.ctypeslib.as_array(p, shape=(cnt,)).astype(dt, copy=True)
        return dict(dim=d, nlevels=ti.nlevels, qbits=ti.qbits, n=n, nbox=nb,
                    level=arr(ti.level, nb, np.int64), coords=arr(ti.coords, nb * d, np.int64).reshape(nb, d),
                    parent=arr(ti.parent, nb, np.int64), is_leaf=arr(ti.is_leaf, nb, bool),
                    pt_begin=arr(ti.pt_begin, nb, np.int64), pt_end=arr(ti.pt_end, nb, np.int64),
                    perm=arr(ti.perm, n, np.int64))

    def neighbours(self, level: int) -> dict:
        nb = C.c_int64()
        bx, off, ids = C.POINTER(C.c_int64)(), C.POINTER(C.c_int64)(), C.POINTER(C.c_int64)()
        _check(lib().rsrs_tree_neighbours(self._h, level, C.byref(nb), C.byref(bx), C.byref(off),
                                          C.byref(ids)))
        n = nb.value
        boxes = np.ctypeslib.as_array(bx, shape=(n,)).copy()
        offs = np.ctypeslib.as_array(off, shape=(n + 1,)).copy()
        allid = np.ctypeslib.as_array(ids, shape=(int(offs[-1]),)).copy() if offs[-1] else np.zeros(0, np.int64)
        return {int(b): allid[offs[i]:offs[i + 1]] for i, b in enumerate(boxes)}

    def schedule(self, k: int):
        nb = self.info()["nbox"]
        col = np.zeros(nb, np.int32)
        bc = np.zeros(nb, np.int64)
        lc = np.zeros(nb, np.int64)
        rc = C.c_int64()
        _check(lib().rsrs_tree_schedule(self._h, k, col.ctypes.data_as(C.POINTER(C.c_int32)),
                                        bc.ctypes.data_as(C.POINTER(C.c_int64)),
                                        lc.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(rc)))
        return col, bc, lc, rc.value

    def samples_required(self, k: int, p: int | None = None) -> int:
        return rsrs_samples_required(self, k, k if p is None else p)


def rsrs_build_tree(points, leaf_size: int, root_lo=None, root_side: float = 1.0,
                    qbits: int = 0) -> Tree:
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    o = TreeOpts()
    o.dim, o.leaf_size, o.qbits = d, leaf_size, qbits
    lo = [0.0, 0.0, 0.0] if root_lo is None else list(root_lo) + [0.0] * (3 - len(root_lo))
    for a in range(3):
        o.root_lo[a] = lo[a]
    o.root_side = root_side
    h = C.c_void_p()
    _check(lib().rsrs_build_tree(pts.ctypes.data_as(C.POINTER(C.c_double)), n, C.byref(o),
                                 C.byref(h)))
    return Tree(h, n)


def rsrs_samples_required(tree: Tree, k: int, p: int) -> int:
    v = lib().rsrs_samples_required(tree.handle, k, p)
    if v < 0:
        raise RSRSError(1, "invalid arguments to rsrs_samples_required")
    return int(v)


def rsrs_work_model(tree: Tree, k: int, s: int, symmetric: bool = False, esize: int = 8,
                    col_subset: bool = False, p: int = -1) -> dict:
    """Algorithmic flops, bytes and stored entries of a fixed-rank factorization."""
    f, b, st = C.c_double(), C.c_double(), C.c_int64()
    o = FactorOpts(int(k), int(p), 0, 1, int(symmetric), 0, 0.0, int(col_subset))
    _check(lib().rsrs_work_model(tree.handle, C.byref(o), int(s), esize, C.byref(f), C.byref(b),
                                 C.byref(st)))
    return {"flops": f.value, "bytes": b.value, "stored_entries": st.value}


def rsrs_gemm_autotune(cache_path: str | None = None) -> dict:
    """Measures (or loads from cache_path) the GEMM tile table; returns the
    number of launch classes and how many differ from the built-in rule."""
    e, c = C.c_int64(), C.c_int64()
    _check(lib().rsrs_gemm_autotune(cache_path.encode() if cache_path else None, C.byref(e), C.byref(c)))
    return {"classes": e.value, "changed": c.value}


def rsrs_gemm_autotune_workload(tree: Tree, k: int, s: int, precision: int = RSRS_PREC_F64,
                                symmetric: bool = False, p: int = -1, reproject: int = 1, id_mode: int = 0,
                                col_subset: bool = False) -> dict:
    """Times the factorization of this workload under each tile shape and
    keeps, per GEMM shape signature, the fastest; returns the number of
    signatures and how many moved from the current choice."""
    o = FactorOpts(int(k), int(p), precision, reproject, int(symmetric), int(id_mode), 0.0, int(col_subset))
    n, c = C.c_int64(), C.c_int64()
    _check(lib().rsrs_gemm_autotune_workload(tree.handle, C.byref(o), int(s), C.byref(n), C.byref(c)))
    return {"signatures": n.value, "changed": c.value}


def rsrs_gemm_tile_override(shape: int) -> None:
    """Forces a tile shape (0, 1, 2); -1 back to the table, -2 forgets it."""
    _check(lib().rsrs_gemm_tile_override(int(shape)))


def rsrs_op_library_gemm(enable: bool) -> None:
    """Wide products of the built-in dense operators through rocBLAS /
    hipBLASLt (True, the default) or the library's own MFMA GEMMs (False)."""
    _check(lib().rsrs_op_library_gemm(int(bool(enable))))


# --------------------------------------------------------------------------- operators
class Operator:
    """A built-in black-box operator; ``matvec_fn``/``handle`` satisfy rsrs_matvec_fn."""

    def __init__(self, handle, n, keep=None):
        self._h = handle
        self.n = n
        self._keep = keep

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.rsrs_op_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    @staticmethod
    def fn_ptr():
        return C.cast(lib().rsrs_op_matvec, C.c_void_p)

    def matvec(self, X, transpose: bool = False, out=None, stream=None, bf16: bool = False):
        """A X or A^T X for an FP64 or FP32 device block X (same type out);
        bf16=True asks for the BF16 product of an FP32 block of BF16 values."""
        import torch
        px, ldx = _dev(X, "X", ("float64", "float32"))
        if out is None:
            out = torch.empty_like(X)
        if out.dtype != X.dtype:
            raise TypeError("out must have the dtype of X")
        py, ldy = _dev(out, "out", ("float64", "float32"))
        code = RSRS_BF16 if bf16 else _dtype_code(X)
        st = lib().rsrs_op_matvec(self._h, int(transpose), code, X.shape[1], px, ldx, py,
                                  ldy, _stream(stream))
        if st != 0:
            raise RSRSError(4, "rsrs_op_matvec failed: " + lib().rsrs_last_error().decode())
        return out


def rsrs_op_create_kernel(kind: int, points, param: float = 0.0, param2: float = 0.0) -> Operator:
    pts = np.ascontiguousarray(points, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().rsrs_op_create_kernel(kind, pts.ctypes.data_as(C.POINTER(C.c_double)), pts.shape[0],
                                       pts.shape[1], param, param2, C.byref(h)))
    return Operator(h, pts.shape[0])


def rsrs_op_create_dense(A) -> Operator:
    pa, lda = _dev(A, "A")
    h = C.c_void_p()
    _check(lib().rsrs_op_create_dense(pa, A.shape[0], lda, C.byref(h)))
    return Operator(h, A.shape[0], keep=A)


def rsrs_op_create_poisson7(n: int, coef_nodes) -> Operator:
    c = np.ascontiguousarray(coef_nodes, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().rsrs_op_create_poisson7(n, c.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
    return Operator(h, n ** 3)


# --------------------------------------------------------------------------- samples
class Samples:
    def __init__(self, handle, s):
        self._h = handle
        self.s = s

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.rsrs_samples_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h


def rsrs_samples_wrap(tree: Tree, Y, Z, Om, Psi, stream=None) -> Samples:
    """Sketches as FP64 or FP32 device tensors (all four of one dtype); with
    Z and Psi None, symmetric samples (rsrs_samples_wrap_symmetric)."""
    if Z is None and Psi is None:
        py_, ld = _dev(Y, "Y", ("float64", "float32"))
        po, ldo = _dev(Om, "Omega", ("float64", "float32"))
        if ldo != ld or Om.shape != Y.shape or Om.dtype != Y.dtype:
            raise TypeError("sketches must share shape, dtype and leading dimension")
        h = C.c_void_p()
        _check(lib().rsrs_samples_wrap_symmetric(tree.handle, _dtype_code(Y), py_, po, ld, Y.shape[1],
                                                 _stream(stream), C.byref(h)))
        return Samples(h, Y.shape[1])
    ptrs = []
    ld = None
    for name, t in (("Y", Y), ("Z", Z), ("Omega", Om), ("Psi", Psi)):
        p, l = _dev(t, name, ("float64", "float32"))
        if ld is None:
            ld = l
        if l != ld or t.shape != Y.shape or t.dtype != Y.dtype:
            raise TypeError("sketches must share shape, dtype and leading dimension")
        ptrs.append(p)
    h = C.c_void_p()
    _check(lib().rsrs_samples_wrap(tree.handle, _dtype_code(Y), *ptrs, ld, Y.shape[1],
                                   _stream(stream), C.byref(h)))
    return Samples(h, Y.shape[1])


def rsrs_sample(tree: Tree, op: Operator, s: int, seed: int, dtype: int = RSRS_F64,
                stream=None, symmetric: bool = False) -> Samples:
    h = C.c_void_p()
    fn = lib().rsrs_sample_symmetric if symmetric else lib().rsrs_sample
    _check(fn(tree.handle, Operator.fn_ptr(), op.handle, s, seed, dtype, _stream(stream), C.byref(h)))
    return Samples(h, s)


def rsrs_gaussian(nrows: int, ncols: int, seed: int, word: int = 0, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((nrows, ncols), dtype=torch.float64, device="cuda")
    p, ld = _dev(out, "out")
    _check(lib().rsrs_gaussian(p, nrows, ncols, ld, seed, word, _stream(stream)))
    return out


# --------------------------------------------------------------------------- factor
class Factor:
    def __init__(self, handle, keep=None):
        self._h = handle
        self._keep = keep

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.rsrs_factor_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        fi = FactorInfo()
        _check(lib().rsrs_factor_get_info(self._h, C.byref(fi)))
        return {f: getattr(fi, f) for f, _ in FactorInfo._fields_}

    def box(self, i: int) -> dict:
        L = lib()
        box, lev, col = C.c_int64(), C.c_int32(), C.c_int32()
        b, n, r, k = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(L.rsrs_factor_box_sizes(self._h, i, C.byref(box), C.byref(lev), C.byref(col), C.byref(b),
                                       C.byref(n), C.byref(r), C.byref(k)))
        b, n, r, k = b.value, n.value, r.value, k.value
        out = dict(box=box.value, level=lev.value, colour=col.value,
                   Ba=np.zeros(b, np.int64), Na=np.zeros(n, np.int64), S=np.zeros(k, np.int64),
                   R=np.zeros(r, np.int64), T=np.zeros((r, k)), XRR=np.zeros((r, r)),
                   KU=np.zeros((r, k + n)), KL=np.zeros((k + n, r)))
        ptr = lambda a: C.c_void_p(a.ctypes.data) if a.size else None
        _check(L.rsrs_factor_box_copy(self._h, i, ptr(out["Ba"]), ptr(out["Na"]), ptr(out["S"]),
                                      ptr(out["R"]), ptr(out["T"]), ptr(out["XRR"]), ptr(out["KU"]),
                                      ptr(out["KL"])))
        return out

    def root(self):
        nt = C.c_int64()
        _check(lib().rsrs_factor_root_copy(self._h, C.byref(nt), None, None))
        Bt = np.zeros(nt.value, np.int64)
        At = np.zeros((nt.value, nt.value))
        _check(lib().rsrs_factor_root_copy(self._h, C.byref(nt), C.c_void_p(Bt.ctypes.data),
                                           C.c_void_p(At.ctypes.data)))
        return Bt, At

    def solve(self, F, transpose=False, out=None, stream=None):
        return rsrs_solve(self, F, transpose, out, stream)

    def apply(self, X, transpose=False, out=None, stream=None):
        return rsrs_apply(self, X, transpose, out, stream)


def rsrs_factor(tree: Tree, samples: Samples, k: int, p: int = -1, reproject: int = 1,
                precision: int = RSRS_PREC_F64, stream=None, symmetric: bool = False,
                id_mode: int = 0, rank_tol: float = 0.0, col_subset: bool = False) -> Factor:
    o = FactorOpts(k, p, precision, reproject, int(symmetric), int(id_mode), float(rank_tol), int(col_subset))
    h = C.c_void_p()
    _check(lib().rsrs_factor(tree.handle, samples.handle, C.byref(o), _stream(stream), C.byref(h)))
    return Factor(h, keep=tree)


def rsrs_factor_redraw(tree: Tree, op: "Operator", s: int, seed: int, k: int, p: int = -1, reproject: int = 1,
                       precision: int = RSRS_PREC_F64, dtype: int | None = None, stream=None,
                       symmetric: bool = False, id_mode: int = 0, rank_tol: float = 0.0,
                       col_subset: bool = False) -> Factor:
    """Sample and factor with fresh samples at every processed level after the
    first (rsrs_factor_redraw)."""
    if dtype is None:
        dtype = RSRS_F64 if precision == RSRS_PREC_F64 else RSRS_F32
    o = FactorOpts(k, p, precision, reproject, int(symmetric), int(id_mode), float(rank_tol), int(col_subset))
    h = C.c_void_p()
    _check(lib().rsrs_factor_redraw(tree.handle, Operator.fn_ptr(), op.handle, int(s), int(seed), int(dtype),
                                    C.byref(o), _stream(stream), C.byref(h)))
    return Factor(h, keep=tree)


def rsrs_factor_batched(trees, samples, ks, p: int = -1, reproject: int = 1,
                        precision: int = RSRS_PREC_F64, stream=None, symmetric: bool = False,
                        id_mode: int = 0, rank_tol: float = 0.0, col_subset: bool = False) -> list:
    """Factor independent problems together; ks gives each problem's rank."""
    n = len(trees)
    if len(samples) != n or len(ks) != n:
        raise ValueError("trees, samples and ks must have the same length")
    th = (C.c_void_p * n)(*[t.handle for t in trees])
    sh = (C.c_void_p * n)(*[x.handle for x in samples])
    opts = (FactorOpts * n)(*[FactorOpts(int(k), p, precision, reproject, int(symmetric), int(id_mode),
                                         float(rank_tol), int(col_subset)) for k in ks])
    outs = (C.c_void_p * n)()
    _check(lib().rsrs_factor_batched(n, th, sh, opts, _stream(stream), outs))
    return [Factor(C.c_void_p(outs[i]), keep=trees[i]) for i in range(n)]


def rsrs_solve(f: Factor, F, transpose=False, out=None, stream=None):
    import torch
    pf, ldf = _dev(F, "F")
    if out is None:
        out = torch.empty_like(F)
    pu, ldu = _dev(out, "out")
    _check(lib().rsrs_solve(f.handle, int(transpose), F.shape[1], pf, ldf, pu, ldu, _stream(stream)))
    return out


def rsrs_solve_noalloc(f: Factor, F, out, transpose=False, stream=None):
    """rsrs_solve without any device allocation (the caller provides ``out``)."""
    pf, ldf = _dev(F, "F")
    pu, ldu = _dev(out, "out")
    _check(lib().rsrs_solve_noalloc(f.handle, int(transpose), F.shape[1], pf, ldf, pu, ldu, _stream(stream)))
    return out


def rsrs_solve_graphs(on: bool = True):
    """Replay HIP graphs for solves of up to 1024 columns (default on)."""
    lib().rsrs_solve_graphs(int(on))


def rsrs_apply(f: Factor, X, transpose=False, out=None, stream=None):
    import torch
    px, ldx = _dev(X, "X")
    if out is None:
        out = torch.empty_like(X)
    py, ldy = _dev(out, "out")
    _check(lib().rsrs_apply(f.handle, int(transpose), X.shape[1], px, ldx, py, ldy, _stream(stream)))
    return out


def rsrs_solve_refine(f: Factor, op: Operator, F, tol: float = 1e-10, maxit: int = 10, out=None,
                      stream=None):
    import torch
    pf, ldf = _dev(F, "F")
    if out is None:
        out = torch.empty_like(F)
    pu, ldu = _dev(out, "out")
    rel = C.c_double()
    it = C.c_int()
    _check(lib().rsrs_solve_refine(f.handle, Operator.fn_ptr(), op.handle, F.shape[1], pf, ldf, pu, ldu,
                                   tol, maxit, C.byref(rel), C.byref(it), _stream(stream)))
    return out, rel.value, it.value


def rsrs_solve_gmres(f: Factor, op: Operator, F, tol: float = 1e-10, restart: int = 30, maxit: int = 200,
                     out=None, stream=None):
    """GMRES preconditioned by the factorization; returns (u, relres, iterations)."""
    import torch
    pf, ldf = _dev(F, "F")
    if out is None:
        out = torch.empty_like(F)
    pu, ldu = _dev(out, "out")
    rel = C.c_double()
    it = C.c_int()
    _check(lib().rsrs_solve_gmres(f.handle, Operator.fn_ptr(), op.handle, F.shape[1], pf, ldf, pu, ldu,
                                  float(tol), int(restart), int(maxit), C.byref(rel), C.byref(it),
                                  _stream(stream)))
    return out, rel.value, it.value


# --------------------------------------------------------------------------- serving
class Server:
    """Continuous-batching server (rsrs_server_*): resident factors, batched
    solves, budget-admitted factorizations.  Device tensors handed to a request
    are kept alive here until the request has been waited for."""

    def __init__(self, hbm_budget: int = 0, max_batch_cols: int = 1024):
        o = ServerOpts(int(hbm_budget), int(max_batch_cols))
        h = C.c_void_p()
        _check(lib().rsrs_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rsrs_server_destroy(h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_factor(self, f: Factor) -> int:
        fid = C.c_int64()
        _check(lib().rsrs_server_add_factor(self._h, f.handle, C.byref(fid)))
        f._h = None   # owned by the server now
        return fid.value

    def set_refine(self, fid: int, op: "Operator | None", tol: float = 1e-6, maxit: int = 10):
        """Refine served solves of factor fid through op to tol (None: one-shot)."""
        if op is None:
            _check(lib().rsrs_server_set_refine(self._h, int(fid), None, None, 0.0, 0))
        else:
            self._keep[("refine", fid)] = op
            _check(lib().rsrs_server_set_refine(self._h, int(fid), Operator.fn_ptr(), op.handle,
                                                float(tol), int(maxit)))

    def release(self, fid: int):
        _check(lib().rsrs_server_release_factor(self._h, int(fid)))

    def submit_solve(self, fid: int, F, out=None) -> tuple:
        import torch
        pf, ldf = _dev(F, "F")
        if out is None:
            out = torch.empty_like(F)
        pu, ldu = _dev(out, "out")
        t = C.c_int64()
        _check(lib().rsrs_server_submit_solve(self._h, int(fid), F.shape[1], pf, ldf, pu, ldu,
                                              C.byref(t)))
        self._keep[t.value] = (F, out)
        return t.value, out

    def submit_factor(self, tree: Tree, op: Operator, s: int, seed: int, k: int,
                      precision: int = RSRS_PREC_F64, p: int = -1, reproject: int = 1,
                      dtype: int | None = None, symmetric: bool = False, id_mode: int = 0,
                      rank_tol: float = 0.0, col_subset: bool = False) -> int:
        if dtype is None:
            dtype = RSRS_F64 if precision == RSRS_PREC_F64 else RSRS_F32
        o = FactorOpts(int(k), p, precision, reproject, int(symmetric), int(id_mode), float(rank_tol),
                       int(col_subset))
        t = C.c_int64()
        _check(lib().rsrs_server_submit_factor(self._h, tree.handle, Operator.fn_ptr(), op.handle,
                                               int(s), int(seed), dtype, C.byref(o), C.byref(t)))
        self._keep[t.value] = (tree, op)
        return t.value

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        """(result id or -1, latency in ms); raises RSRSError on a failed request."""
        res = C.c_int64()
        lat = C.c_double()
        st = lib().rsrs_server_wait(self._h, int(ticket), float(timeout_ms), C.byref(res),
                                    C.byref(lat))
        if st != 9:
            self._keep.pop(int(ticket), None)
        _check(st)
        return res.value, lat.value

    def stats(self, reset: bool = False) -> dict:
        s = ServerStats()
        _check(lib().rsrs_server_get_stats(self._h, int(reset), C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}


def rsrs_release_cached():
    """Free the factorization scratch kept for reuse by later factorizations."""
    lib().rsrs_release_cached()


# --------------------------------------------------------------------------- measurement
def rsrs_profile_enable(on: bool = True):
    lib().rsrs_profile_enable(int(on))


def rsrs_profile_filter(prefix: str | None = None):
    """Record only launches whose tag begins with `prefix` (None: all)."""
    lib().rsrs_profile_filter(prefix.encode() if prefix else None)


def rsrs_profile_reset():
    lib().rsrs_profile_reset()


def rsrs_profile_read() -> dict:
    """{tag: dict(launches, ms, flops, bytes)} for launches since the last reset."""
    L = lib()
    n = L.rsrs_profile_read(None, 0)
    if n < 0:
        raise RSRSError(7, "rsrs_profile_read failed")
    arr = (ProfileEntry * max(n, 1))()
    n = L.rsrs_profile_read(arr, n)
    return {arr[i].tag.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                                      bytes=arr[i].bytes) for i in range(n)}
