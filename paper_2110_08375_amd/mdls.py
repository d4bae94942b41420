"""ctypes binding of the C ABI in ``include/mdls.h`` (argument marshalling only).

Tensors follow the library's storage: a matrix of P-limb numbers with ``rows`` rows and
``cols`` columns is a contiguous ``torch.float64`` tensor of shape ``(P, cols, rows)`` on the
GPU (P column-major planes, leading dimension ``rows``); a vector is ``(P, length)``.  Every
call is enqueued on the current torch stream.  Nothing here computes: if the HIP library is
missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmdls.so")

MDLS_F64, MDLS_DD, MDLS_QD, MDLS_OD = 1, 2, 4, 8
MDLS_EHIP, MDLS_EUNSUPPORTED, MDLS_ESCRATCH = -100, -101, -102
MDLS_NOALLOC_SCRATCH_BYTES = 64 << 20
MDLS_TUNE_LOOKAHEAD, MDLS_TUNE_PANEL_VARIANT, MDLS_TUNE_APPLY_GRID_CAP = 1, 2, 3
MDLS_TUNE_APPLY_WIDE_ROWS, MDLS_TUNE_SPIN_LIMIT, MDLS_TUNE_SPLIT_UPDATE = 4, 5, 6
MDLS_TUNE_CPANEL = 7

# every symbol include/mdls.h declares
EXPORTS = ("mdls_init", "mdls_finalize", "mdls_set_tuning", "mdls_get_tuning", "mdls_max_rows", "mdls_workspace_bytes", "mdls_qr", "mdls_apply_qt", "mdls_form_w",
           "mdls_backsub", "mdls_solve", "mdls_status_string", "mdls_timing_enable", "mdls_timing_reset",
           "mdls_timing_query", "mdls_timing_kernels", "mdls_batch_workspace_bytes", "mdls_batch_plan",
           "mdls_solve_batched", "mdls_batch_variants", "mdls_batch_autotune", "mdls_wall_clock_khz",
           "mdls_refined_workspace_bytes", "mdls_solve_refined", "mdls_apply_q", "mdls_form_q",
           "mdls_cworkspace_bytes", "mdls_cqr", "mdls_capply_qh", "mdls_cbacksub", "mdls_csolve",
           "mdls_dd_gemm_tn_workspace_bytes", "mdls_dd_gemm_tn", "mdls_capply_q", "mdls_cform_q",
           "mdls_solve_noalloc")


class BatchDesc(ctypes.Structure):
    """mdls_batch_desc: problem shape and offsets (in doubles) into the A, b, x pools."""
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("a_off", ctypes.c_longlong),
                ("b_off", ctypes.c_longlong), ("x_off", ctypes.c_longlong)]

_lib = None


class MdlsError(RuntimeError):
    pass


def lib():
    """Load ``libmdls.so``; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise MdlsError("libmdls.so is not built (run paper_2110_08375_amd/build.py); "
                            "there is no CPU fallback")
        L = ctypes.CDLL(_LIB_PATH)
        i, sz, vp = ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p
        L.mdls_init.argtypes = []
        L.mdls_finalize.argtypes = []
        L.mdls_set_tuning.argtypes = [i, ctypes.c_long]
        L.mdls_get_tuning.argtypes = [i]
        L.mdls_get_tuning.restype = ctypes.c_long
        L.mdls_max_rows.argtypes = [i]
        L.mdls_max_rows.restype = i
        L.mdls_workspace_bytes.argtypes = [i, i, i, i]
        L.mdls_workspace_bytes.restype = sz
        L.mdls_qr.argtypes = [i, i, i, i, vp, i, vp, vp, i, vp, sz, vp, vp]
        L.mdls_apply_qt.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, i, vp, sz, vp]
        L.mdls_form_w.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, vp]
        L.mdls_apply_q.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, i, vp, sz, vp]
        L.mdls_form_q.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, i, vp, sz, vp]
        L.mdls_backsub.argtypes = [i, i, i, vp, i, vp, vp, sz, vp, vp]
        L.mdls_solve.argtypes = [i, i, i, i, vp, i, vp, vp, vp, sz, vp, vp]
        L.mdls_solve_noalloc.argtypes = [i, i, i, i, vp, i, vp, vp, vp, vp]
        L.mdls_status_string.argtypes = [i]
        L.mdls_status_string.restype = ctypes.c_char_p
        L.mdls_timing_enable.argtypes = [i]
        L.mdls_timing_reset.argtypes = []
        L.mdls_timing_query.argtypes = [ctypes.c_char_p, i, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_double)]
        L.mdls_timing_kernels.argtypes = [ctypes.c_char_p, i]
        L.mdls_batch_workspace_bytes.argtypes = [i, i]
        L.mdls_batch_workspace_bytes.restype = sz
        L.mdls_batch_plan.argtypes = [i, i, ctypes.POINTER(BatchDesc), vp, sz, vp]
        L.mdls_solve_batched.argtypes = [i, i, vp, vp, vp, i, vp, sz, vp, vp, vp]
        L.mdls_batch_variants.argtypes = [i]
        L.mdls_batch_autotune.argtypes = [i, i, vp, vp, sz, sz, vp, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_float),
                                          vp]
        L.mdls_wall_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
        L.mdls_refined_workspace_bytes.argtypes = [i, i, i, i]
        L.mdls_refined_workspace_bytes.restype = sz
        L.mdls_solve_refined.argtypes = [i, i, i, i, vp, i, vp, vp, i, vp, vp, sz, vp, vp, vp]
        L.mdls_cworkspace_bytes.argtypes = [i, i, i, i]
        L.mdls_cworkspace_bytes.restype = sz
        L.mdls_cqr.argtypes = [i, i, i, i, vp, i, vp, i, vp, sz, vp]
        L.mdls_capply_qh.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, i, vp, sz, vp]
        L.mdls_cbacksub.argtypes = [i, i, i, vp, i, vp, vp, sz, vp, vp]
        L.mdls_capply_q.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, i, vp, sz, vp]
        L.mdls_cform_q.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, i, vp, sz, vp]
        L.mdls_csolve.argtypes = [i, i, i, i, vp, i, vp, vp, vp, sz, vp, vp]
        L.mdls_dd_gemm_tn_workspace_bytes.argtypes = [i, i]
        L.mdls_dd_gemm_tn_workspace_bytes.restype = sz
        L.mdls_dd_gemm_tn.argtypes = [i, i, i, i, vp, i, vp, i, vp, i, vp, sz, vp]
        for f in ("mdls_init", "mdls_finalize", "mdls_set_tuning", "mdls_capply_q", "mdls_cform_q", "mdls_dd_gemm_tn", "mdls_cqr", "mdls_capply_qh", "mdls_cbacksub", "mdls_csolve", "mdls_qr", "mdls_apply_qt", "mdls_apply_q", "mdls_form_q", "mdls_form_w", "mdls_backsub",
                  "mdls_solve", "mdls_timing_enable", "mdls_timing_reset", "mdls_timing_query", "mdls_timing_kernels",
                  "mdls_batch_plan", "mdls_solve_batched", "mdls_batch_variants", "mdls_batch_autotune",
                  "mdls_wall_clock_khz", "mdls_solve_refined"):
            getattr(L, f).restype = i
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().mdls_status_string(status).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise MdlsError("%s failed with status %d (%s)" % (what, rc, status_string(rc)))


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _mat(t, P, name):
    import torch

    if t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 3 or t.shape[0] != P:
        raise ValueError("%s must be a contiguous float64 tensor of shape (P, cols, rows)" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    return t.shape[2], t.shape[1]  # rows (= ld), cols


def _vec(t, P, name, length):
    import torch

    if (t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 2 or t.shape[0] != P
            or t.shape[1] != length or not t.is_cuda):
        raise ValueError("%s must be a contiguous float64 GPU tensor of shape (%d, %d)" % (name, P, length))


def init():
    """mdls_init on the calling thread and the current device (the look-ahead side stream)."""
    _check(lib().mdls_init(), "mdls_init")


def finalize():
    _check(lib().mdls_finalize(), "mdls_finalize")


def set_tuning(option: int, value: int):
    _check(lib().mdls_set_tuning(option, value), "mdls_set_tuning")


def get_tuning(option: int) -> int:
    return lib().mdls_get_tuning(option)


def max_rows(p: int) -> int:
    return lib().mdls_max_rows(p)


def workspace_bytes(p: int, m: int, n: int, tile: int) -> int:
    return lib().mdls_workspace_bytes(p, m, n, tile)


def workspace(p: int, m: int, n: int, tile: int, device="cuda"):
    import torch

    nb = workspace_bytes(p, m, n, tile)
    if nb == 0:
        raise ValueError("invalid sizes for a workspace")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def qr(p: int, A, tile: int, T=None, ws=None, beta=None, info=None):
    """In-place QR of A (P, n, m); T (P, n, ldt) or None receives the tile T factors, beta (P, n)
    or None the betas, info (one int32) or None the barrier status."""
    m, n = _mat(A, p, "A")
    if ws is None:
        ws = workspace(p, m, n, tile, A.device)
    ldt = 0
    if T is not None:
        ldt, _ = _mat(T, p, "T")
    if beta is not None:
        _vec(beta, p, "beta", n)
    rc = lib().mdls_qr(p, m, n, tile, _ptr(A), m, _ptr(beta), _ptr(T), ldt, _ptr(ws), ws.numel(), _ptr(info),
                       _stream())
    _check(rc, "mdls_qr")
    return A, T


def apply_qt(p: int, A, T, B, tile: int, ws=None):
    """B (P, nrhs, m) := Q^T B, in place."""
    m, n = _mat(A, p, "A")
    ldt, _ = _mat(T, p, "T")
    ldb, nrhs = _mat(B, p, "B")
    if ws is None:
        ws = workspace(p, m, n, tile, A.device)
    rc = lib().mdls_apply_qt(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(B), ldb, nrhs, _ptr(ws),
                             ws.numel(), _stream())
    _check(rc, "mdls_apply_qt")
    return B


def apply_q(p: int, A, T, B, tile: int, ws=None):
    """B (P, nrhs, m) := Q B, in place."""
    m, n = _mat(A, p, "A")
    ldt, _ = _mat(T, p, "T")
    ldb, nrhs = _mat(B, p, "B")
    if ws is None:
        ws = workspace(p, m, n, tile, A.device)
    rc = lib().mdls_apply_q(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(B), ldb, nrhs, _ptr(ws), ws.numel(),
                            _stream())
    _check(rc, "mdls_apply_q")
    return B


def form_q(p: int, A, T, tile: int, Q, ws=None):
    """Q (P, ncols, m) := the first ncols columns of the explicit orthogonal factor."""
    m, n = _mat(A, p, "A")
    ldt, _ = _mat(T, p, "T")
    ldq, ncols = _mat(Q, p, "Q")
    if ws is None:
        ws = workspace(p, m, n, tile, A.device)
    rc = lib().mdls_form_q(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(Q), ldq, ncols, _ptr(ws), ws.numel(),
                           _stream())
    _check(rc, "mdls_form_q")
    return Q


def form_w(p: int, A, T, tile: int, W):
    """W (P, n, m) := the paper's W factors, W_k = -Y_k T_k."""
    m, n = _mat(A, p, "A")
    ldt, _ = _mat(T, p, "T")
    ldw, _ = _mat(W, p, "W")
    rc = lib().mdls_form_w(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(W), ldw, _stream())
    _check(rc, "mdls_form_w")
    return W


def backsub(p: int, R, x, tile: int, n: int | None = None, ws=None, info=None):
    """Solve R x = y for the n x n upper triangle of R (P, n, ldr); x (P, n) holds y on entry.
    Returns (x, info tensor).  The library takes R's plane stride as ldr * n, so R must have
    exactly n columns."""
    import torch

    if n is not None and R.dim() == 3 and n != R.shape[1]:
        raise ValueError("R must have exactly n columns (its limb planes are ldr * n apart)")
    ldr, n = _mat(R, p, "R")
    _vec(x, p, "x", n)
    if ws is None:
        ws = workspace(p, n, n, tile, R.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=R.device)
    rc = lib().mdls_backsub(p, n, tile, _ptr(R), ldr, _ptr(x), _ptr(ws), ws.numel(), _ptr(info), _stream())
    _check(rc, "mdls_backsub")
    return x, info


def solve(p: int, A, b, tile: int, x=None, ws=None, info=None):
    """Least squares: A (P, n, m) and b (P, m) are overwritten; returns (x, info)."""
    import torch

    m, n = _mat(A, p, "A")
    _vec(b, p, "b", m)
    if x is None:
        x = torch.empty((p, n), dtype=torch.float64, device=A.device)
    _vec(x, p, "x", n)
    if ws is None:
        ws = workspace(p, m, n, tile, A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = lib().mdls_solve(p, m, n, tile, _ptr(A), m, _ptr(b), _ptr(x), _ptr(ws), ws.numel(), _ptr(info),
                          _stream())
    _check(rc, "mdls_solve")
    return x, info


def solve_noalloc(p: int, A, b, tile: int, x, info):
    """mdls_solve on the library's static scratch: A (P, n, m) and b (P, m) are overwritten,
    x (P, n) and info (one int32) are caller-allocated; nothing is allocated here."""
    import torch

    m, n = _mat(A, p, "A")
    _vec(b, p, "b", m)
    _vec(x, p, "x", n)
    if info is None or info.dtype != torch.int32 or info.numel() < 1 or info.device != A.device:
        raise MdlsError("info must be an int32 tensor on the device of A")
    rc = lib().mdls_solve_noalloc(p, m, n, tile, _ptr(A), m, _ptr(b), _ptr(x), _ptr(info), _stream())
    _check(rc, "mdls_solve_noalloc")
    return x, info


def dd_gemm_tn(method: int, Y, C, S=None, ws=None):
    """S (2, c, w) := Y^T C for double-double Y (2, w, h) and C (2, c, h): method 0 on the
    vector units, 1 on the matrix cores by exact slicing."""
    import torch

    h, w = _mat(Y, 2, "Y")
    hc, c = _mat(C, 2, "C")
    if hc != h:
        raise ValueError("Y and C need the same number of rows")
    if S is None:
        S = torch.empty((2, c, w), dtype=torch.float64, device=Y.device)
    lds, sc = _mat(S, 2, "S")
    if sc != c:
        raise ValueError("S must have c columns")
    if ws is None and method == 1:
        ws = torch.empty(lib().mdls_dd_gemm_tn_workspace_bytes(w, c), dtype=torch.uint8, device=Y.device)
    rc = lib().mdls_dd_gemm_tn(method, h, w, c, _ptr(Y), h, _ptr(C), h, _ptr(S), lds, _ptr(ws),
                               0 if ws is None else ws.numel(), _stream())
    _check(rc, "mdls_dd_gemm_tn")
    return S


# ------------------------------------------------------------------------------ complex
# A complex matrix is a contiguous float64 tensor of shape (2, P, cols, rows): the P limb
# planes of the real parts, then those of the imaginary parts.  A complex vector: (2, P, n).
def _cmat(t, P, name):
    import torch

    if t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 4 or t.shape[0] != 2 or t.shape[1] != P:
        raise ValueError("%s must be a contiguous float64 tensor of shape (2, P, cols, rows)" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    return t.shape[3], t.shape[2]  # rows (= ld), cols


def _cvec(t, P, name, length):
    import torch

    if (t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 3 or t.shape[0] != 2 or t.shape[1] != P
            or t.shape[2] != length or not t.is_cuda):
        raise ValueError("%s must be a contiguous float64 GPU tensor of shape (2, %d, %d)" % (name, P, length))


def cworkspace_bytes(p: int, m: int, n: int, tile: int) -> int:
    return lib().mdls_cworkspace_bytes(p, m, n, tile)


def cworkspace(p: int, m: int, n: int, tile: int, device="cuda"):
    import torch

    nb = cworkspace_bytes(p, m, n, tile)
    if nb == 0:
        raise ValueError("invalid sizes for a workspace")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def cqr(p: int, A, tile: int, T=None, ws=None):
    """In-place complex QR of A (2, P, n, m); T (2, P, n, ldt) or None receives the T_k."""
    m, n = _cmat(A, p, "A")
    if ws is None:
        ws = cworkspace(p, m, n, tile, A.device)
    ldt = 0
    if T is not None:
        ldt, tc = _cmat(T, p, "T")
        if tc != n:
            raise ValueError("T must have n columns")
    rc = lib().mdls_cqr(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(ws), ws.numel(), _stream())
    _check(rc, "mdls_cqr")
    return A, T


def capply_qh(p: int, A, T, B, tile: int, ws=None):
    """B (2, P, nrhs, m) := Q^H B, in place."""
    m, n = _cmat(A, p, "A")
    ldt, tc = _cmat(T, p, "T")
    if tc != n:
        raise ValueError("T must have n columns")
    ldb, nrhs = _cmat(B, p, "B")
    if ws is None:
        ws = cworkspace(p, m, n, tile, A.device)
    rc = lib().mdls_capply_qh(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(B), ldb, nrhs, _ptr(ws), ws.numel(),
                              _stream())
    _check(rc, "mdls_capply_qh")
    return B


def capply_q(p: int, A, T, B, tile: int, ws=None):
    """B (2, P, nrhs, m) := Q B, in place."""
    m, n = _cmat(A, p, "A")
    ldt, tc = _cmat(T, p, "T")
    if tc != n:
        raise ValueError("T must have n columns")
    ldb, nrhs = _cmat(B, p, "B")
    if ws is None:
        ws = cworkspace(p, m, n, tile, A.device)
    rc = lib().mdls_capply_q(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(B), ldb, nrhs, _ptr(ws), ws.numel(),
                             _stream())
    _check(rc, "mdls_capply_q")
    return B


def cform_q(p: int, A, T, tile: int, Q, ws=None):
    """Q (2, P, ncols, m) := the first ncols columns of the explicit unitary factor."""
    m, n = _cmat(A, p, "A")
    ldt, tc = _cmat(T, p, "T")
    if tc != n:
        raise ValueError("T must have n columns")
    ldq, ncols = _cmat(Q, p, "Q")
    if ws is None:
        ws = cworkspace(p, m, n, tile, A.device)
    rc = lib().mdls_cform_q(p, m, n, tile, _ptr(A), m, _ptr(T), ldt, _ptr(Q), ldq, ncols, _ptr(ws), ws.numel(),
                            _stream())
    _check(rc, "mdls_cform_q")
    return Q


def cbacksub(p: int, R, x, tile: int, ws=None, info=None):
    """Solve R x = y for the complex n x n upper triangle of R (2, P, n, ldr); x (2, P, n)
    holds y on entry.  Returns (x, info tensor)."""
    import torch

    ldr, n = _cmat(R, p, "R")
    _cvec(x, p, "x", n)
    if ws is None:
        ws = cworkspace(p, n, n, tile, R.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=R.device)
    rc = lib().mdls_cbacksub(p, n, tile, _ptr(R), ldr, _ptr(x), _ptr(ws), ws.numel(), _ptr(info), _stream())
    _check(rc, "mdls_cbacksub")
    return x, info


def csolve(p: int, A, b, tile: int, x=None, ws=None, info=None):
    """Complex least squares: A (2, P, n, m) and b (2, P, m) are overwritten; returns (x, info)."""
    import torch

    m, n = _cmat(A, p, "A")
    _cvec(b, p, "b", m)
    if x is None:
        x = torch.empty((2, p, n), dtype=torch.float64, device=A.device)
    _cvec(x, p, "x", n)
    if ws is None:
        ws = cworkspace(p, m, n, tile, A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = lib().mdls_csolve(p, m, n, tile, _ptr(A), m, _ptr(b), _ptr(x), _ptr(ws), ws.numel(), _ptr(info), _stream())
    _check(rc, "mdls_csolve")
    return x, info


def timing_enable(on: bool = True):
    lib().mdls_timing_enable(1 if on else 0)


def timing_reset():
    lib().mdls_timing_reset()


def timing_kernels():
    buf = ctypes.create_string_buffer(4096)
    lib().mdls_timing_kernels(buf, 4096)
    return [n for n in buf.value.decode().split("\n") if n]


def timing_query(name: str = "", p: int = 0):
    """(total milliseconds, launches, algorithmic md multiply-adds) of the recorded launches."""
    ms = ctypes.c_double(0)
    cnt = ctypes.c_long(0)
    work = ctypes.c_double(0)
    _check(lib().mdls_timing_query(name.encode(), p, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(work)),
           "mdls_timing_query")
    return ms.value, cnt.value, work.value


# ----------------------------------------------------------------------------- batched solves
def batch_descs(p: int, shapes):
    """Descriptors for problems packed back to back: A pool (P planes of m x n each), b pool
    (P planes of m), x pool (P planes of n).  Returns (descs, a_len, b_len, x_len)."""
    descs = (BatchDesc * len(shapes))()
    a = b = x = 0
    for k, (m, n) in enumerate(shapes):
        descs[k] = BatchDesc(int(m), int(n), a, b, x)
        a += p * m * n
        b += p * m
        x += p * n
    return descs, a, b, x


def batch_workspace(p: int, count: int, device="cuda"):
    import torch

    nb = lib().mdls_batch_workspace_bytes(p, count)
    if nb == 0:
        raise ValueError("invalid precision or count for a batch workspace")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def batch_plan(p: int, descs, ws):
    _check(lib().mdls_batch_plan(p, len(descs), descs, _ptr(ws), ws.numel(), _stream()), "mdls_batch_plan")


def batch_variants(p: int) -> int:
    return lib().mdls_batch_variants(p)


def solve_batched(p: int, count: int, A, b, x, variant: int, ws, info, times=None):
    """Solve the planned batch in one persistent launch on the current stream."""
    _check(lib().mdls_solve_batched(p, count, _ptr(A), _ptr(b), _ptr(x), variant, _ptr(ws), ws.numel(), _ptr(info),
                                    _ptr(times), _stream()), "mdls_solve_batched")
    return x, info


def batch_autotune(p: int, count: int, A_src, b_src, A, b, x, ws, info):
    """Time every kernel variant on copies of the batch; returns (best variant, ms per variant)."""
    nv = batch_variants(p)
    ms = (ctypes.c_float * max(nv, 1))()
    rc = lib().mdls_batch_autotune(p, count, _ptr(A_src), _ptr(b_src), A_src.numel(), b_src.numel(), _ptr(A), _ptr(b),
                                   _ptr(x), _ptr(ws), ws.numel(), _ptr(info), ms, _stream())
    if rc < 0:
        _check(rc, "mdls_batch_autotune")
    return rc, [ms[i] for i in range(nv)]


def wall_clock_khz() -> int:
    k = ctypes.c_int(0)
    _check(lib().mdls_wall_clock_khz(ctypes.byref(k)), "mdls_wall_clock_khz")
    return k.value


# ----------------------------------------------------------------------------- refined solve
def refined_workspace(p_out: int, m: int, n: int, tile: int, device="cuda"):
    import torch

    nb = lib().mdls_refined_workspace_bytes(p_out, m, n, tile)
    if nb == 0:
        raise ValueError("invalid sizes for a refined-solve workspace")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def solve_refined(p_out: int, A, b, tile: int, iters: int, x=None, F=None, ws=None, info=None, norms=None):
    """x (p_out, n) from a double-double factorisation of A (2, n, m) and at most iters refinement
    steps with residuals in p_out limbs; b (p_out, m).  Returns (x, info, norms); norms (2 iters)
    holds max |correction| and max |x| per step taken, -1 for steps not taken."""
    import torch

    m, n = _mat(A, 2, "A")
    _vec(b, p_out, "b", m)
    if x is None:
        x = torch.empty((p_out, n), dtype=torch.float64, device=A.device)
    _vec(x, p_out, "x", n)
    if F is None:
        F = torch.empty_like(A)
    if ws is None:
        ws = refined_workspace(p_out, m, n, tile, A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if norms is None:
        norms = torch.zeros(2 * iters, dtype=torch.float64, device=A.device)
    rc = lib().mdls_solve_refined(p_out, m, n, tile, _ptr(A), m, _ptr(b), _ptr(x), iters, _ptr(F), _ptr(ws), ws.numel(),
                                  _ptr(info), _ptr(norms), _stream())
    _check(rc, "mdls_solve_refined")
    return x, info, norms
