"""ctypes binding of the C ABI declared in include/mlbicgstab.h.

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch supplies device memory and streams.  If the built library is missing
this module raises at import time; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlbicgstab.so")

MLB_CONVERGED, MLB_MAXIT, MLB_BREAKDOWN = 0, 1, -1
MLB_EINVAL, MLB_ENOMEM, MLB_EHIP, MLB_EUNSUPPORTED = -2, -3, -4, -5
MLB_R64, MLB_C128 = 0, 1
MLB_CSR, MLB_BSR3 = 0, 1
MLB_PREC_FP64, MLB_PREC_FP32_IR = 0, 1
MLB_PRECOND_NONE, MLB_PRECOND_JACOBI, MLB_PRECOND_ILU0 = 0, 1, 2
MLB_ORDER_FUSED, MLB_ORDER_LITERAL = 0, 1
MLB_OP_A, MLB_OP_AH, MLB_OP_MINV, MLB_OP_MINVH = 0, 1, 2, 3
MLB_MAX_N = 32
MLB_MAX_INDEX = 2 ** 31 - 2 ** 20   # largest nrows and nnz
MLB_KERNEL_SPMV_STEP, MLB_KERNEL_ALPHA_STEP, MLB_KERNEL_COMBINE, MLB_KERNEL_RECOMBINE = 0, 1, 2, 3
MLB_SERVE_FIFO, MLB_SERVE_SMALLEST = 0, 1


class mlb_matrix(ctypes.Structure):
    _fields_ = [
        ("format", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("nrows", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("values", ctypes.c_void_p),
    ]


class mlb_options(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int64),
        ("kappa", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("max_outer", ctypes.c_int32),
        ("record_iterates", ctypes.c_int32),
        ("iterates", ctypes.c_void_p),
        ("precond", ctypes.c_int32),
        ("transpose_free", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("max_restarts", ctypes.c_int32),
    ]


class mlb_result(ctypes.Structure):
    _fields_ = [
        ("flag", ctypes.c_int32),
        ("iter", ctypes.c_int64),
        ("outer_iters", ctypes.c_int32),
        ("fp64_iters", ctypes.c_int64),
        ("err_recursive", ctypes.c_double),
        ("err_true", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
    ]


class mlb_server_options(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32), ("small_n_max", ctypes.c_int32),
                ("order", ctypes.c_int32), ("max_wait_ms", ctypes.c_double)]


class mlb_request_timing(ctypes.Structure):
    _fields_ = [
        ("queued_ms", ctypes.c_double),
        ("run_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
        ("footprint_bytes", ctypes.c_uint64),
        ("n_used", ctypes.c_int32),
    ]


class mlb_server_stats_t(ctypes.Structure):
    _fields_ = [
        ("budget_bytes", ctypes.c_uint64),
        ("used_bytes", ctypes.c_uint64),
        ("peak_used_bytes", ctypes.c_uint64),
        ("queued", ctypes.c_int64),
        ("running", ctypes.c_int32),
        ("peak_running", ctypes.c_int32),
        ("completed", ctypes.c_int64),
    ]


mlb_handle = ctypes.c_void_p
mlb_server_handle = ctypes.c_void_p

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

_lib.mlbicgstab_create.argtypes = [ctypes.POINTER(mlb_matrix), ctypes.POINTER(mlb_options), ctypes.c_void_p,
                                   ctypes.POINTER(mlb_handle)]
_lib.mlbicgstab_create.restype = ctypes.c_int
_lib.mlbicgstab_workspace_size.argtypes = [ctypes.POINTER(mlb_matrix), ctypes.POINTER(mlb_options),
                                           ctypes.POINTER(ctypes.c_size_t)]
_lib.mlbicgstab_workspace_size.restype = ctypes.c_int
_lib.mlbicgstab_solve.argtypes = [mlb_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.POINTER(mlb_result)]
_lib.mlbicgstab_solve.restype = ctypes.c_int
_lib.mlbicgstab_destroy.argtypes = [mlb_handle]
_lib.mlbicgstab_destroy.restype = ctypes.c_int
_lib.mlbicgstab_last_error.argtypes = []
_lib.mlbicgstab_last_error.restype = ctypes.c_char_p
_lib.mlbicgstab_matvec.argtypes = [mlb_handle, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
_lib.mlbicgstab_matvec.restype = ctypes.c_int
_lib.mlbicgstab_time_kernel.argtypes = [mlb_handle, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
_lib.mlbicgstab_time_kernel.restype = ctypes.c_int
_lib.mlbicgstab_solve_batch.argtypes = [ctypes.POINTER(mlb_handle), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(mlb_result)]
_lib.mlbicgstab_solve_batch.restype = ctypes.c_int
mlb_sequence_handle = ctypes.c_void_p
_lib.mlb_sequence_next_n.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32]
_lib.mlb_sequence_next_n.restype = ctypes.c_int32
_lib.mlb_sequence_create.argtypes = [ctypes.POINTER(mlb_matrix), ctypes.POINTER(mlb_options), ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.POINTER(mlb_sequence_handle)]
_lib.mlb_sequence_create.restype = ctypes.c_int
_lib.mlb_sequence_solve.argtypes = [mlb_sequence_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.POINTER(mlb_result), ctypes.POINTER(ctypes.c_int32)]
_lib.mlb_sequence_solve.restype = ctypes.c_int
_lib.mlb_sequence_destroy.argtypes = [mlb_sequence_handle]
_lib.mlb_sequence_destroy.restype = ctypes.c_int
_lib.mlbicgstab_solve_noalloc.argtypes = [ctypes.POINTER(mlb_matrix), ctypes.POINTER(mlb_options), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.POINTER(mlb_result)]
_lib.mlbicgstab_solve_noalloc.restype = ctypes.c_int
MLB_NOALLOC_SCRATCH_BYTES = 64 << 20
_lib.mlb_server_create.argtypes = [ctypes.POINTER(mlb_server_options), ctypes.POINTER(mlb_server_handle)]
_lib.mlb_server_create.restype = ctypes.c_int
_lib.mlb_server_submit.argtypes = [mlb_server_handle, ctypes.POINTER(mlb_matrix), ctypes.POINTER(mlb_options),
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)]
_lib.mlb_server_submit.restype = ctypes.c_int
_lib.mlb_server_submit_sequence.argtypes = [mlb_server_handle, ctypes.c_uint64, ctypes.POINTER(mlb_matrix),
                                            ctypes.POINTER(mlb_options), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
_lib.mlb_server_submit_sequence.restype = ctypes.c_int
_lib.mlb_server_end_sequence.argtypes = [mlb_server_handle, ctypes.c_uint64]
_lib.mlb_server_end_sequence.restype = ctypes.c_int
for _f in ("mlb_server_poll", "mlb_server_wait"):
    getattr(_lib, _f).argtypes = [mlb_server_handle, ctypes.c_int64, ctypes.POINTER(mlb_result),
                                  ctypes.POINTER(mlb_request_timing)]
    getattr(_lib, _f).restype = ctypes.c_int
_lib.mlb_server_stats.argtypes = [mlb_server_handle, ctypes.POINTER(mlb_server_stats_t)]
_lib.mlb_server_stats.restype = ctypes.c_int
_lib.mlb_server_destroy.argtypes = [mlb_server_handle]
_lib.mlb_server_destroy.restype = ctypes.c_int


class MlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mlbicgstab error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc <= -2:
        raise MlbError(rc, mlbicgstab_last_error())
    return rc


# ---- the C entry points, same names ---------------------------------------------


def mlbicgstab_create(A: mlb_matrix, opt: mlb_options, hip_stream: int = 0):
    h = mlb_handle()
    _check(_lib.mlbicgstab_create(ctypes.byref(A), ctypes.byref(opt), ctypes.c_void_p(hip_stream), ctypes.byref(h)))
    return h


def mlbicgstab_workspace_size(A: mlb_matrix, opt: mlb_options) -> int:
    out = ctypes.c_size_t()
    _check(_lib.mlbicgstab_workspace_size(ctypes.byref(A), ctypes.byref(opt), ctypes.byref(out)))
    return out.value


def mlbicgstab_solve(h, b_ptr: int, x_ptr: int, q_ptr: int, ldq: int) -> mlb_result:
    res = mlb_result()
    _check(_lib.mlbicgstab_solve(h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), ctypes.c_void_p(q_ptr),
                                 ctypes.c_int64(ldq), ctypes.byref(res)))
    return res


def mlbicgstab_solve_batch(handles, b_ptrs, x_ptrs, q_ptrs, ldqs):
    """One launch for all systems (one workgroup each); returns the list of mlb_result."""
    k = len(handles)
    hs = (mlb_handle * k)(*handles)
    ptrs = lambda v: (ctypes.c_void_p * k)(*[ctypes.c_void_p(p) for p in v])
    res = (mlb_result * k)()
    _check(_lib.mlbicgstab_solve_batch(hs, k, ptrs(b_ptrs), ptrs(x_ptrs), ptrs(q_ptrs), (ctypes.c_int64 * k)(*ldqs),
                                       res))
    return list(res)


def mlbicgstab_destroy(h) -> int:
    return _check(_lib.mlbicgstab_destroy(h))


def mlbicgstab_solve_noalloc(A: mlb_matrix, opt: mlb_options, hip_stream: int, b_ptr: int, x_ptr: int, q_ptr: int,
                             ldq: int) -> mlb_result:
    res = mlb_result()
    _check(_lib.mlbicgstab_solve_noalloc(ctypes.byref(A), ctypes.byref(opt), ctypes.c_void_p(hip_stream),
                                         ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), ctypes.c_void_p(q_ptr),
                                         ctypes.c_int64(ldq), ctypes.byref(res)))
    return res


def mlbicgstab_last_error() -> str:
    return _lib.mlbicgstab_last_error().decode()


def mlbicgstab_matvec(h, op: int, x_ptr: int, y_ptr: int) -> None:
    _check(_lib.mlbicgstab_matvec(h, op, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)))


def mlbicgstab_time_kernel(h, kernel: int, reps: int) -> float:
    ms = ctypes.c_double()
    _check(_lib.mlbicgstab_time_kernel(h, kernel, reps, ctypes.byref(ms)))
    return ms.value


def mlb_sequence_next_n(n: int, t_prev_ms: float, t_cur_ms: float, step: int, n_min: int, n_max: int) -> int:
    return _lib.mlb_sequence_next_n(n, t_prev_ms, t_cur_ms, step, n_min, n_max)


def mlb_sequence_create(A: mlb_matrix, opt: mlb_options, n_min: int, n_max: int, step: int, hip_stream: int = 0):
    h = mlb_sequence_handle()
    _check(_lib.mlb_sequence_create(ctypes.byref(A), ctypes.byref(opt), n_min, n_max, step,
                                    ctypes.c_void_p(hip_stream), ctypes.byref(h)))
    return h


def mlb_sequence_solve(h, b_ptr: int, x_ptr: int, q_ptr: int, ldq: int):
    """(result, n used)."""
    res, n = mlb_result(), ctypes.c_int32()
    _check(_lib.mlb_sequence_solve(h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), ctypes.c_void_p(q_ptr),
                                   ctypes.c_int64(ldq), ctypes.byref(res), ctypes.byref(n)))
    return res, n.value


def mlb_sequence_destroy(h) -> int:
    return _check(_lib.mlb_sequence_destroy(h))


def mlb_server_create(budget_bytes: int, max_inflight: int, small_n_max: int = 0, order: int = MLB_SERVE_FIFO,
                      max_wait_ms: float = 0.0):
    h = mlb_server_handle()
    _check(_lib.mlb_server_create(ctypes.byref(mlb_server_options(budget_bytes, max_inflight, small_n_max, order,
                                                                  max_wait_ms)),
                                  ctypes.byref(h)))
    return h


def mlb_server_submit(s, A: mlb_matrix, opt: mlb_options, b_ptr: int, x_ptr: int, q_ptr: int, ldq: int) -> int:
    t = ctypes.c_int64()
    _check(_lib.mlb_server_submit(s, ctypes.byref(A), ctypes.byref(opt), ctypes.c_void_p(b_ptr),
                                  ctypes.c_void_p(x_ptr), ctypes.c_void_p(q_ptr), ctypes.c_int64(ldq),
                                  ctypes.byref(t)))
    return t.value


def mlb_server_submit_sequence(s, key: int, A: mlb_matrix, opt: mlb_options, n_min: int, n_max: int, step: int,
                               b_ptr: int, x_ptr: int, q_ptr: int, ldq: int) -> int:
    t = ctypes.c_int64()
    _check(_lib.mlb_server_submit_sequence(s, ctypes.c_uint64(key), ctypes.byref(A), ctypes.byref(opt), n_min, n_max,
                                           step, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr),
                                           ctypes.c_void_p(q_ptr), ctypes.c_int64(ldq), ctypes.byref(t)))
    return t.value


def mlb_server_end_sequence(s, key: int) -> int:
    return _check(_lib.mlb_server_end_sequence(s, ctypes.c_uint64(key)))


def mlb_server_poll(s, ticket: int):
    """(done, result, timing); done False while pending."""
    res, tim = mlb_result(), mlb_request_timing()
    rc = _check(_lib.mlb_server_poll(s, ticket, ctypes.byref(res), ctypes.byref(tim)))
    return rc == 1, res, tim


def mlb_server_wait(s, ticket: int):
    res, tim = mlb_result(), mlb_request_timing()
    _check(_lib.mlb_server_wait(s, ticket, ctypes.byref(res), ctypes.byref(tim)))
    return res, tim


def mlb_server_stats(s) -> mlb_server_stats_t:
    st = mlb_server_stats_t()
    _check(_lib.mlb_server_stats(s, ctypes.byref(st)))
    return st


def mlb_server_destroy(s) -> int:
    return _check(_lib.mlb_server_destroy(s))


def raw_call(name, *args):
    """The raw C function (for tests of the error paths)."""
    return getattr(_lib, name)(*args)


# ---- torch convenience layer (marshalling only) ----------------------------------


@dataclass
class DeviceMatrix:
    """Device arrays of one sparse matrix (torch tensors) plus its descriptor."""
    row_ptr: object
    col_idx: object
    values: object
    nrows: int
    fmt: int
    dtype: int

    def descriptor(self) -> mlb_matrix:
        nnz = int(self.col_idx.numel())
        return mlb_matrix(self.fmt, self.dtype, self.nrows, nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                          self.values.data_ptr())


def to_device(A, device="cuda"):
    """Upload a scipy CSR or BSR (3x3 blocks) matrix as int32 / float64 or complex128 tensors."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    if sp.isspmatrix_bsr(A) or isinstance(A, sp.bsr_array):
        if A.blocksize != (3, 3):
            raise ValueError("BSR matrices must have 3x3 blocks")
        fmt = MLB_BSR3
        vals = np.ascontiguousarray(A.data)
    else:
        A = A.tocsr()
        fmt = MLB_CSR
        vals = np.ascontiguousarray(A.data)
    cplx = np.iscomplexobj(vals)
    vals = vals.astype(np.complex128 if cplx else np.float64)
    rp = torch.from_numpy(np.ascontiguousarray(A.indptr.astype(np.int32))).to(device)
    ci = torch.from_numpy(np.ascontiguousarray(A.indices.astype(np.int32))).to(device)
    v = torch.from_numpy(vals.reshape(-1)).to(device)
    return DeviceMatrix(rp, ci, v, A.shape[0], fmt, MLB_C128 if cplx else MLB_R64)


def column_major(Q, device="cuda"):
    """An N x n torch tensor with column-major strides (1, N) holding Q."""
    import numpy as np
    import torch

    Qf = np.asarray(Q)
    t = torch.from_numpy(np.ascontiguousarray(Qf.T)).to(device)   # n x N row-major == N x n column-major
    return t.t()


def q_layout(Q, N: int, n: int) -> int:
    """Checks that Q is an N x n column-major tensor (any stride on a dimension of size 1) and returns ldq."""
    if Q.dim() != 2 or Q.shape[0] != N or Q.shape[1] != n or (N > 1 and Q.stride(0) != 1):
        raise ValueError("Q must be an N x n column-major tensor")
    ldq = Q.stride(1) if n > 1 else N
    if ldq < N:
        raise ValueError("Q's columns overlap (leading dimension < N)")
    return ldq


class Solver:
    """One handle: create() on construction, solve() per right-hand side, destroy() on close()."""

    def __init__(self, dmat: DeviceMatrix, n: int, tol: float = 1e-10, maxit: int = 1000, kappa: float = 0.0,
                 precision: int = MLB_PREC_FP64, inner_tol: float = 0.0, max_outer: int = 0,
                 record_iterates: int = 0, iterates=None, stream=None, precond: int = MLB_PRECOND_NONE,
                 transpose_free: bool = False, order: int = MLB_ORDER_FUSED, max_restarts: int = 0):
        import torch

        self.dmat = dmat
        self.n = n
        self.iterates = iterates
        self.opt = mlb_options(n, tol, maxit, kappa, precision, inner_tol, max_outer, record_iterates,
                               iterates.data_ptr() if iterates is not None else None, precond, int(transpose_free),
                               order, max_restarts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = mlbicgstab_create(dmat.descriptor(), self.opt, self.stream.cuda_stream)

    def solve(self, b, x, Q) -> mlb_result:
        N = self.dmat.nrows
        ldq = q_layout(Q, N, self.n)
        if b.numel() != N or x.numel() != N or not x.is_contiguous() or not b.is_contiguous():
            raise ValueError("b and x must be contiguous vectors of length N")
        return mlbicgstab_solve(self.h, b.data_ptr(), x.data_ptr(), Q.data_ptr(), ldq)

    def ldq_of(self, Q):
        return q_layout(Q, self.dmat.nrows, self.n)

    def time_kernel(self, kernel: int, reps: int) -> float:
        return mlbicgstab_time_kernel(self.h, kernel, reps)

    def matvec(self, x, y, op: int = MLB_OP_A) -> None:
        """y = A x (op = MLB_OP_A) or y = A^H x (op = MLB_OP_AH) on the library's SpMV kernels; with an
        ILU(0) preconditioner also y = M^{-1} x (MLB_OP_MINV) and y = M^{-H} x (MLB_OP_MINVH)."""
        N = self.dmat.nrows
        if x.numel() != N or y.numel() != N or not x.is_contiguous() or not y.is_contiguous():
            raise ValueError("x and y must be contiguous vectors of length N")
        mlbicgstab_matvec(self.h, op, x.data_ptr(), y.data_ptr())

    def close(self):
        if self.h:
            mlbicgstab_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_noalloc(dmat: DeviceMatrix, b, x, Q, n: int, tol: float = 1e-10, maxit: int = 1000, kappa: float = 0.0,
                  record_iterates: int = 0, iterates=None, stream=None, transpose_free: bool = False,
                  order: int = MLB_ORDER_FUSED, max_restarts: int = 0) -> mlb_result:
    """mlbicgstab_solve_noalloc: one fp64 solve with every library buffer in the static device scratch."""
    import torch

    N = dmat.nrows
    ldq = q_layout(Q, N, n)
    if b.numel() != N or x.numel() != N or not x.is_contiguous() or not b.is_contiguous():
        raise ValueError("b and x must be contiguous vectors of length N")
    opt = mlb_options(n, tol, maxit, kappa, MLB_PREC_FP64, 0.0, 0, record_iterates,
                      iterates.data_ptr() if iterates is not None else None, MLB_PRECOND_NONE, int(transpose_free),
                      order, max_restarts)
    st = stream if stream is not None else torch.cuda.current_stream()
    return mlbicgstab_solve_noalloc(dmat.descriptor(), opt, st.cuda_stream, b.data_ptr(), x.data_ptr(),
                                    Q.data_ptr(), ldq)


def solve_batch(solvers, bs, xs, Qs):
    """mlbicgstab_solve_batch over Solver objects (same stream, CSR, fp64, no preconditioner)."""
    for sv, b, x, Q in zip(solvers, bs, xs, Qs):
        N = sv.dmat.nrows
        q_layout(Q, N, sv.n)
        if b.numel() != N or x.numel() != N or not x.is_contiguous() or not b.is_contiguous():
            raise ValueError("b and x must be contiguous vectors of length N")
    return mlbicgstab_solve_batch([sv.h for sv in solvers], [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                  [Q.data_ptr() for Q in Qs], [sv.ldq_of(Q) for sv, Q in zip(solvers, Qs)])


class Sequence:
    """Systems with the same A, n chosen from one system to the next (Section 5.2)."""

    def __init__(self, dmat: DeviceMatrix, n: int, n_min: int, n_max: int, step: int, tol: float = 1e-10,
                 maxit: int = 1000, kappa: float = 0.0, precision: int = MLB_PREC_FP64, stream=None,
                 precond: int = MLB_PRECOND_NONE, transpose_free: bool = False, order: int = MLB_ORDER_FUSED,
                 max_restarts: int = 0):
        import torch

        self.dmat = dmat
        self.n_max = n_max
        self.opt = mlb_options(n, tol, maxit, kappa, precision, 0.0, 0, 0, None, precond, int(transpose_free), order,
                               max_restarts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = mlb_sequence_create(dmat.descriptor(), self.opt, n_min, n_max, step, self.stream.cuda_stream)

    def solve(self, b, x, Q):
        """Q: N x n_max column-major.  Returns (result, n used)."""
        N = self.dmat.nrows
        ldq = q_layout(Q, N, self.n_max)
        if b.numel() != N or x.numel() != N or not x.is_contiguous() or not b.is_contiguous():
            raise ValueError("b and x must be contiguous vectors of length N")
        return mlb_sequence_solve(self.h, b.data_ptr(), x.data_ptr(), Q.data_ptr(), ldq)

    def close(self):
        if self.h:
            mlb_sequence_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching front end: submit() solves, wait()/poll() for their results."""

    def __init__(self, budget_bytes: int, max_inflight: int = 4, small_n_max: int = 0, order: int = MLB_SERVE_FIFO,
                 max_wait_ms: float = 0.0):
        self.h = mlb_server_create(budget_bytes, max_inflight, small_n_max, order, max_wait_ms)
        self._keep = {}

    def submit(self, dmat: DeviceMatrix, b, x, Q, n: int, tol: float = 1e-10, maxit: int = 1000, kappa: float = 0.0,
               precision: int = MLB_PREC_FP64, inner_tol: float = 0.0, precond: int = MLB_PRECOND_NONE,
               transpose_free: bool = False, order: int = MLB_ORDER_FUSED, max_restarts: int = 0) -> int:
        N = dmat.nrows
        ldq = q_layout(Q, N, n)
        opt = mlb_options(n, tol, maxit, kappa, precision, inner_tol, 0, 0, None, precond, int(transpose_free),
                          order, max_restarts)
        t = mlb_server_submit(self.h, dmat.descriptor(), opt, b.data_ptr(), x.data_ptr(), Q.data_ptr(), ldq)
        self._keep[t] = (dmat, b, x, Q)
        return t

    def submit_sequence(self, key: int, dmat: DeviceMatrix, b, x, Q, n: int, n_min: int, n_max: int, step: int,
                        tol: float = 1e-10, maxit: int = 1000, kappa: float = 0.0, precision: int = MLB_PREC_FP64,
                        inner_tol: float = 0.0, precond: int = MLB_PRECOND_NONE, transpose_free: bool = False,
                        order: int = MLB_ORDER_FUSED, max_restarts: int = 0) -> int:
        """A request of sequence `key` (same A throughout; Q is N x n_max, n is the first request's)."""
        N = dmat.nrows
        ldq = q_layout(Q, N, n_max)
        opt = mlb_options(n, tol, maxit, kappa, precision, inner_tol, 0, 0, None, precond, int(transpose_free),
                          order, max_restarts)
        t = mlb_server_submit_sequence(self.h, key, dmat.descriptor(), opt, n_min, n_max, step, b.data_ptr(),
                                       x.data_ptr(), Q.data_ptr(), ldq)
        self._keep[t] = (dmat, b, x, Q)
        return t

    def end_sequence(self, key: int) -> None:
        mlb_server_end_sequence(self.h, key)

    def wait(self, ticket: int):
        try:
            return mlb_server_wait(self.h, ticket)
        finally:
            self._keep.pop(ticket, None)

    def poll(self, ticket: int):
        done, res, tim = mlb_server_poll(self.h, ticket)
        if done:
            self._keep.pop(ticket, None)
        return done, res, tim

    def stats(self) -> mlb_server_stats_t:
        return mlb_server_stats(self.h)

    def close(self):
        if self.h:
            mlb_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
