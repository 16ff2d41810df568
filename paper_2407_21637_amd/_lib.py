"""ctypes binding of ``libhodlr.so`` (argument marshalling only).

Every step of the product runs in the HIP library; this module converts
numpy arrays and torch tensors into pointers and sizes, calls the C ABI
declared in ``include/hodlr.h`` and turns error codes into exceptions.  It
has no fallback: if the library is not built, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhodlr.so")

DTYPES = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "e4m3": 4, "e5m2": 5}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}
CODE_NP = {0: np.uint64, 1: np.uint32, 2: np.uint16, 3: np.uint16, 4: np.uint8, 5: np.uint8}

NO_COLUMN_SCALE = 0x1
ACC_FP32 = 0x2
ACC_FP64 = 0x4
PER_BLOCK = 0x8

STATUS = {0: "HODLR_OK", 1: "HODLR_E_ARG", 2: "HODLR_E_STATE", 3: "HODLR_E_NOMEM",
          4: "HODLR_E_DEVICE", 5: "HODLR_E_RANGE", 6: "HODLR_E_UNSUPPORTED"}

# every symbol include/hodlr.h declares
EXPORTS = ("hodlr_depth_for_leaf", "hodlr_tree_bounds", "hodlr_tree_blocks", "hodlr_create",
           "hodlr_assign_precision", "hodlr_set_level_precisions", "hodlr_get_level",
           "hodlr_get_info", "hodlr_get_block", "hodlr_query", "hodlr_export_block", "hodlr_matvec",
           "hodlr_matvec_noalloc", "hodlr_matvec_batched", "hodlr_profile", "hodlr_profile_read",
           "hodlr_destroy", "hodlr_status_string", "hodlr_last_error_message", "hodlr_last_error",
           "hodlr_build_kernel", "hodlr_get_norms", "hodlr_lu", "hodlr_solve", "hodlr_lu_dense")
# kernel matrices the library evaluates itself (hodlr_build_kernel)
KERNELS = {"gaussian": 0, "inv_dist": 1, "log": 2, "exp": 3, "signed_inv": 4}
# entry points that return something other than hodlr_status
_NON_STATUS = ("hodlr_depth_for_leaf", "hodlr_status_string", "hodlr_last_error_message", "hodlr_last_error")
MAX_LEVELS = 24

PHASES = ("pad_x", "contract", "expand", "reduce")


class HodlrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class LowRank(C.Structure):
    _fields_ = [("rank", C.c_int32), ("U", C.c_void_p), ("ldu", C.c_int64),
                ("V", C.c_void_p), ("ldv", C.c_int64)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("depth", C.c_int32), ("nblocks", C.c_int32),
                ("acc_dtype", C.c_int32), ("max_rank", C.c_int32), ("on_device", C.c_int32),
                ("device", C.c_int32), ("eps", C.c_double), ("leaf_bytes", C.c_int64),
                ("factor_bytes", C.c_int64), ("scale_bytes", C.c_int64),
                ("device_bytes", C.c_int64)]


class Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("a", C.c_double), ("diag_shift", C.c_double),
                ("diag_value", C.c_double), ("diag_given", C.c_int32), ("reserved_", C.c_int32)]


class BuildReport(C.Structure):
    _fields_ = [("ms_norms", C.c_double), ("ms_factors", C.c_double), ("ms_total", C.c_double),
                ("max_rank", C.c_int32), ("max_sketch", C.c_int32), ("sketch_rounds", C.c_int32),
                ("exact_residual", C.c_int32)]


class LuReport(C.Structure):
    _fields_ = [("ms_factor", C.c_double), ("norm_l", C.c_double), ("norm_u", C.c_double),
                ("max_rank", C.c_int32), ("reserved_", C.c_int32)]


class QueryInfo(C.Structure):
    _fields_ = [("info", Info), ("level_dtype", C.c_int32 * MAX_LEVELS), ("insufficient", C.c_int32 * MAX_LEVELS),
                ("xi", C.c_double * MAX_LEVELS), ("u_prime", C.c_double * MAX_LEVELS),
                ("per_block", C.c_int32), ("leaf_stacked", C.c_int32)]


class BlockInfo(C.Structure):
    _fields_ = [("level", C.c_int32), ("rank", C.c_int32), ("row0", C.c_int64),
                ("nrows", C.c_int64), ("col0", C.c_int64), ("ncols", C.c_int64),
                ("dtype", C.c_int32), ("scaled", C.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2407_21637_amd.build first")
        L = C.CDLL(LIB_PATH)
        i32, i64, vp, dp = C.c_int32, C.c_int64, C.c_void_p, C.c_double
        L.hodlr_depth_for_leaf.argtypes = [i64, i64]
        L.hodlr_depth_for_leaf.restype = i32
        L.hodlr_tree_bounds.argtypes = [i64, i32, vp, vp]
        L.hodlr_tree_blocks.argtypes = [i64, i32, vp, vp]
        L.hodlr_create.argtypes = [C.POINTER(vp), i64, i32, vp, vp, vp, vp, i32]
        L.hodlr_assign_precision.argtypes = [vp, dp, vp, i32, vp, vp, C.c_uint32]
        L.hodlr_set_level_precisions.argtypes = [vp, vp, C.c_uint32]
        L.hodlr_get_level.argtypes = [vp, i32, vp, vp, vp, vp]
        L.hodlr_get_info.argtypes = [vp, vp]
        L.hodlr_get_block.argtypes = [vp, i32, vp]
        L.hodlr_query.argtypes = [vp, vp, vp, vp]
        L.hodlr_build_kernel.argtypes = [C.POINTER(vp), i64, i32, vp, vp, dp, C.c_uint64, i32, vp]
        L.hodlr_get_norms.argtypes = [vp, vp]
        L.hodlr_lu.argtypes = [vp, dp, vp]
        L.hodlr_solve.argtypes = [vp, vp, i64, vp, i64, i32, i32, vp]
        L.hodlr_lu_dense.argtypes = [vp, vp, i64, vp, i64]
        L.hodlr_export_block.argtypes = [vp, i32, vp, vp, vp, vp, i32]
        L.hodlr_matvec.argtypes = [vp, vp, i64, vp, i64, i32, i32, vp]
        L.hodlr_matvec_noalloc.argtypes = [vp, vp, i64, vp, i64, i32, i32, vp]
        L.hodlr_matvec_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.hodlr_profile.argtypes = [vp, i32]
        L.hodlr_profile_read.argtypes = [vp, vp, vp]
        L.hodlr_destroy.argtypes = [vp]
        L.hodlr_status_string.argtypes = [i32]
        L.hodlr_status_string.restype = C.c_char_p
        L.hodlr_last_error.argtypes = []
        L.hodlr_last_error.restype = C.c_char_p
        L.hodlr_last_error_message.argtypes = []
        L.hodlr_last_error_message.restype = C.c_char_p
        for name in EXPORTS:
            if name not in _NON_STATUS:
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise HodlrError(st, lib().hodlr_last_error_message().decode())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def depth_for_leaf(n: int, leaf: int) -> int:
    return int(lib().hodlr_depth_for_leaf(n, leaf))


def tree_bounds(n: int, depth: int, leaf_bounds=None) -> list:
    out = np.zeros((1 << (depth + 1)) + depth, dtype=np.int64)
    lb = None if leaf_bounds is None else np.ascontiguousarray(leaf_bounds, dtype=np.int64)
    _check(lib().hodlr_tree_bounds(n, depth, _ptr(lb), _ptr(out)))
    levels, off = [], 0
    for k in range(depth + 1):
        levels.append(out[off:off + (1 << k) + 1].copy())
        off += (1 << k) + 1
    return levels


def tree_blocks(n: int, depth: int, leaf_bounds=None) -> np.ndarray:
    """(nblocks, 5) int64: level, row0, nrows, col0, ncols (canonical order)."""
    nb = (1 << (depth + 1)) - 2
    out = np.zeros((max(nb, 1), 5), dtype=np.int64)
    lb = None if leaf_bounds is None else np.ascontiguousarray(leaf_bounds, dtype=np.int64)
    _check(lib().hodlr_tree_blocks(n, depth, _ptr(lb), _ptr(out)))
    return out[:nb]


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _colmajor(t, n):
    """(pointer, ld, nrhs) of a torch tensor holding an n x nrhs column-major
    matrix: shape (n,) or (n, nrhs) with stride (1, ld)."""
    if t.dim() == 1:
        if t.shape[0] != n or t.stride(0) != 1:
            raise ValueError("vector must have n contiguous entries")
        return t.data_ptr(), n, 1
    if t.dim() != 2 or t.shape[0] != n or (n > 1 and t.stride(0) != 1):
        raise ValueError("matrix must be (n, nrhs) column-major (stride (1, ld))")
    ld = t.stride(1) if t.shape[1] > 1 else n
    return t.data_ptr(), ld, t.shape[1]


def colmajor_empty(n, nrhs, dtype, device):
    import torch
    return torch.empty((nrhs, n), dtype=dtype, device=device).t()


class Operator:
    """A HODLR operator held by the library (see ``include/hodlr.h``)."""

    @classmethod
    def _adopt(cls, handle, n, depth, device):
        self = cls.__new__(cls)
        self._h = handle
        self.n, self.depth, self.nblocks, self.device = n, depth, (1 << (depth + 1)) - 2, device
        return self

    def __init__(self, n, depth, leaves, U, V, device=0, leaf_bounds=None):
        self._h = C.c_void_p()
        nl, nb = 1 << depth, (1 << (depth + 1)) - 2
        if len(leaves) != nl or len(U) != nb or len(V) != nb:
            raise ValueError("need 2^depth leaves and 2^(depth+1)-2 blocks")
        keep = []
        lp = (C.c_void_p * nl)()
        ld = np.zeros(nl, dtype=np.int64)
        for i, D in enumerate(leaves):
            D = np.asfortranarray(D, dtype=np.float64)
            keep.append(D)
            lp[i] = D.ctypes.data if D.size else None
            ld[i] = max(1, D.shape[0])
        blks = (LowRank * max(nb, 1))()
        for b in range(nb):
            u = np.asfortranarray(U[b], dtype=np.float64)
            v = np.asfortranarray(V[b], dtype=np.float64)
            keep += [u, v]
            blks[b].rank = u.shape[1]
            blks[b].U = u.ctypes.data if u.size else None
            blks[b].ldu = max(1, u.shape[0])
            blks[b].V = v.ctypes.data if v.size else None
            blks[b].ldv = max(1, v.shape[0])
        lb = None if leaf_bounds is None else np.ascontiguousarray(leaf_bounds, dtype=np.int64)
        _check(lib().hodlr_create(C.byref(self._h), n, depth, _ptr(lb),
                                  C.cast(lp, C.c_void_p), _ptr(ld), C.cast(blks, C.c_void_p), device))
        self.n, self.depth, self.nblocks, self.device = n, depth, nb, device

    @property
    def handle(self):
        return self._h

    def assign_precision(self, eps, allowed, norms2=None, flags=0, xi=None):
        """Alg. "Adaptive-precision HODLR Format" (``hodlr_assign_precision``);
        xi: optional per-level xi_1..xi_depth used as given."""
        al = np.array([DTYPES[a] if isinstance(a, str) else int(a) for a in allowed] or [0],
                      dtype=np.int32)
        nr = None if norms2 is None else np.ascontiguousarray(norms2, dtype=np.float64)
        if nr is not None and nr.size != 1 + self.nblocks:
            raise ValueError("norms2 needs 1 + nblocks values")
        xa = None if xi is None else np.ascontiguousarray(xi, dtype=np.float64)
        if xa is not None and xa.size != self.depth:
            raise ValueError("xi needs depth values")
        _check(lib().hodlr_assign_precision(self._h, float(eps), _ptr(al), len(allowed), _ptr(xa), _ptr(nr),
                                            flags))

    def set_level_precisions(self, per_level, flags=0):
        pl = np.array([DTYPES[a] if isinstance(a, str) else int(a) for a in per_level] or [0],
                      dtype=np.int32)
        _check(lib().hodlr_set_level_precisions(self._h, _ptr(pl), flags))

    def level(self, k):
        dt, nb = C.c_int32(), C.c_int32()
        xi, up = C.c_double(), C.c_double()
        _check(lib().hodlr_get_level(self._h, k, C.byref(dt), C.byref(xi), C.byref(up), C.byref(nb)))
        return DTYPE_NAMES[dt.value], xi.value, up.value, bool(nb.value)

    def levels(self):
        return [self.level(k) for k in range(1, self.depth + 1)]

    def info(self):
        inf = Info()
        _check(lib().hodlr_get_info(self._h, C.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in Info._fields_}
        d["acc_dtype"] = DTYPE_NAMES[d["acc_dtype"]]
        return d

    def query(self):
        """``hodlr_query``: info, per-level format / xi / u' / insufficient,
        leaf bounds and ranks in one call."""
        q = QueryInfo()
        lb = np.zeros((1 << self.depth) + 1, dtype=np.int64)
        rk = np.zeros(max(self.nblocks, 1), dtype=np.int32)
        _check(lib().hodlr_query(self._h, C.byref(q), _ptr(lb), _ptr(rk)))
        d = {f: getattr(q.info, f) for f, _ in Info._fields_}
        d["acc_dtype"] = DTYPE_NAMES[d["acc_dtype"]]
        L = self.depth
        d["levels"] = [(DTYPE_NAMES[q.level_dtype[k]], q.xi[k], q.u_prime[k], bool(q.insufficient[k]))
                       for k in range(L)]
        d["per_block"] = bool(q.per_block)
        d["leaf_stacked"] = bool(q.leaf_stacked)
        d["leaf_bounds"] = lb
        d["ranks"] = rk[:self.nblocks]
        return d

    def norms2(self):
        """``hodlr_get_norms``: ||A||_F^2 and ||A_b||_F^2 of the original matrix
        (operators made by ``build_kernel`` only)."""
        out = np.zeros(1 + self.nblocks)
        _check(lib().hodlr_get_norms(self._h, _ptr(out)))
        return out

    def block(self, b):
        bi = BlockInfo()
        _check(lib().hodlr_get_block(self._h, b, C.byref(bi)))
        d = {f: getattr(bi, f) for f, _ in BlockInfo._fields_}
        d["dtype"] = DTYPE_NAMES[d["dtype"]]
        return d

    def export_block(self, b, from_device=False):
        bi = self.block(b)
        dt = CODE_NP[DTYPES[bi["dtype"]]]
        p = bi["rank"]
        uc = np.zeros((bi["nrows"], p), dtype=dt, order="F")
        vc = np.zeros((bi["ncols"], p), dtype=dt, order="F")
        ue = np.zeros(max(p, 1), dtype=np.int8)
        ve = np.zeros(max(p, 1), dtype=np.int8)
        _check(lib().hodlr_export_block(self._h, b, _ptr(uc), _ptr(ue), _ptr(vc), _ptr(ve),
                                        1 if from_device else 0))
        return uc, ue[:p].astype(np.int64), vc, ve[:p].astype(np.int64)

    def _xy(self, X, Y):
        """Checked (X pointer, ldx, Y, Y pointer, ldy, nrhs, dtype code)."""
        code = _xy_code(X)
        xp, ldx, nrhs = _colmajor(X, self.n)
        if Y is None:
            import torch
            Y = torch.empty(self.n, dtype=X.dtype, device=X.device) if X.dim() == 1 else \
                colmajor_empty(self.n, nrhs, X.dtype, X.device)
        if Y.dtype != X.dtype:
            raise TypeError("Y must have X's dtype")
        yp, ldy, ny = _colmajor(Y, self.n)
        if ny != nrhs:
            raise ValueError("Y has a different nrhs")
        _on_device(X, self.device, "X")
        _on_device(Y, self.device, "Y")
        return xp, ldx, Y, yp, ldy, nrhs, code

    def matvec(self, X, Y=None, stream=None):
        """Y = A_H X for torch tensors on the operator's GPU; X is (n,) or
        (n, nrhs) column-major.  float64 / float32 X: the product as
        hodlr_matvec defines it for those dtypes; bfloat16 / float16 X: the
        product in that low working precision.  Returns Y (allocated if None)."""
        xp, ldx, Y, yp, ldy, nrhs, code = self._xy(X, Y)
        _check(lib().hodlr_matvec(self._h, C.c_void_p(xp), ldx, C.c_void_p(yp), ldy, nrhs, code,
                                  _stream_ptr(stream)))
        return Y

    def matvec_noalloc(self, X, Y, stream=None):
        """``hodlr_matvec_noalloc``: the fp64 / fp32 product with the workspace
        in the library's static scratch array (Y must be given)."""
        xp, ldx, Y, yp, ldy, nrhs, code = self._xy(X, Y)
        _check(lib().hodlr_matvec_noalloc(self._h, C.c_void_p(xp), ldx, C.c_void_p(yp), ldy, nrhs, code,
                                          _stream_ptr(stream)))
        return Y

    def lu(self, eps=0.0):
        """``hodlr_lu``: factor the stored operator, H = L U (Schur complements
        truncated at eps); returns the report as a dict."""
        rep = LuReport()
        _check(lib().hodlr_lu(self._h, float(eps), C.byref(rep)))
        return {f: getattr(rep, f) for f, _ in LuReport._fields_ if f != "reserved_"}

    def solve(self, B, X=None, stream=None):
        """``hodlr_solve``: X = U^-1 L^-1 B on the GPU for float64 / float32
        torch tensors ((n,) or (n, nrhs) column-major); X allocated if None."""
        bp, ldb, X, xp, ldx, nrhs, code = self._xy(B, X)
        _check(lib().hodlr_solve(self._h, C.c_void_p(bp), ldb, C.c_void_p(xp), ldx, nrhs, code,
                                 _stream_ptr(stream)))
        return X

    def lu_dense(self):
        """``hodlr_lu_dense``: the factors as dense (L, U) numpy arrays."""
        L = np.zeros((self.n, self.n), order="F")
        U = np.zeros((self.n, self.n), order="F")
        _check(lib().hodlr_lu_dense(self._h, _ptr(L), self.n, _ptr(U), self.n))
        return L, U

    def profile(self, capacity):
        """Record per-phase event timings for the next ``capacity`` products."""
        _check(lib().hodlr_profile(self._h, capacity))

    def profile_read(self):
        """{phase: (total_ms, launches)} of the recorded products; clears them."""
        ms = np.zeros(4)
        cnt = np.zeros(4, dtype=np.int64)
        _check(lib().hodlr_profile_read(self._h, _ptr(ms), _ptr(cnt)))
        return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(PHASES)}

    def close(self):
        if self._h:
            _check(lib().hodlr_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        # during interpreter shutdown the HIP runtime may already be gone:
        # leave the handle to the process exit instead of calling into it
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def build_kernel(points, depth, kind, a=0.0, diag_shift=0.0, diag_value=None, eps=1e-6, seed=0, device=0):
    """``hodlr_build_kernel``: the eps-HODLR operator of the kernel matrix
    k(p_i, p_j) (``kind`` a key of KERNELS) built on the GPU.  Returns the
    Operator and the build report as a dict."""
    P = np.ascontiguousarray(points, dtype=np.float64)
    if P.ndim == 1:
        P = P[:, None]
    n, dim = P.shape
    K = Kernel(KERNELS[kind] if isinstance(kind, str) else int(kind), dim, float(a), float(diag_shift),
               0.0 if diag_value is None else float(diag_value), 0 if diag_value is None else 1, 0)
    rep = BuildReport()
    h = C.c_void_p()
    _check(lib().hodlr_build_kernel(C.byref(h), n, depth, _ptr(P), C.byref(K), float(eps), C.c_uint64(seed), device,
                                    C.byref(rep)))
    return Operator._adopt(h, n, depth, device), {f: getattr(rep, f) for f, _ in BuildReport._fields_}


def _xy_code(X):
    """hodlr_dtype code of a torch tensor's dtype (TypeError for any other)."""
    import torch
    codes = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2, torch.float16: 3}
    if X.dtype not in codes:
        raise TypeError("X must be float64, float32, bfloat16 or float16")
    return codes[X.dtype]


def _on_device(t, device, what):
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{what} must be on the operator's GPU (cuda:{device}), not {t.device}")


def matvec_batched(ops, Xs, Ys, stream=None):
    """Y_i = A_i X_i for every operator, one call (``hodlr_matvec_batched``)."""
    k = len(ops)
    if len(Xs) != k or len(Ys) != k:
        raise ValueError("need one X and one Y per operator")
    hp = (C.c_void_p * k)(*[o.handle.value for o in ops])
    xp = (C.c_void_p * k)()
    yp = (C.c_void_p * k)()
    ldx = np.zeros(k, dtype=np.int64)
    ldy = np.zeros(k, dtype=np.int64)
    nr = np.zeros(k, dtype=np.int32)
    dt = np.zeros(k, dtype=np.int32)
    for i, (o, X, Y) in enumerate(zip(ops, Xs, Ys)):
        if Y is None:
            raise ValueError("matvec_batched needs every Y")
        xp[i], ldx[i], _, yp[i], ldy[i], nr[i], dt[i] = o._xy(X, Y)
    _check(lib().hodlr_matvec_batched(C.cast(hp, C.c_void_p), k, C.cast(xp, C.c_void_p), _ptr(ldx),
                                      C.cast(yp, C.c_void_p), _ptr(ldy), _ptr(nr), _ptr(dt),
                                      _stream_ptr(stream)))
