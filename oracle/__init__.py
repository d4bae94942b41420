"""Python bindings of the CPU oracle (``mdls_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg use this
package.  It never imports the GPU package and the GPU package never imports it.

Arrays follow the paper's limb-major staging (after Algorithm 1): a matrix of P-limb
multiple doubles is a numpy float64 array of shape ``(P, cols, rows)`` (P column-major
planes), a vector has shape ``(P, n)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, l = ctypes.c_int, ctypes.c_long
        for name in ("orc_md_add", "orc_md_sub", "orc_md_mul", "orc_md_div"):
            getattr(L, name).argtypes = [i, dp, dp, dp]
        L.orc_md_sqrt.argtypes = [i, dp, dp]
        L.orc_md_round.argtypes = [i, i, dp, dp]
        lp = ctypes.POINTER(ctypes.c_long)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_qr.argtypes = [i, i, i, dp, i, l, dp, lp, i]
        L.orc_apply_qt.argtypes = [i, i, i, dp, i, l, dp, dp, i, l, i, lp, i]
        L.orc_backsub.argtypes = [i, i, dp, i, l, dp, l, dp, l, ip, lp]
        L.orc_lstsq.argtypes = [i, i, i, dp, i, l, dp, l, dp, l, dp, ip, lp, i]
        L.orc_explicit_q.argtypes = [i, i, i, dp, i, l, dp, dp, i, l, i]
        L.orc_matvec.argtypes = [i, i, i, i, i, i, i, dp, i, l, dp, l, dp, l, dp, l, i]
        L.orc_cmd_mul.argtypes = [i, dp, dp, dp]
        L.orc_cmd_div.argtypes = [i, dp, dp, dp]
        L.orc_cqr.argtypes = [i, i, i, dp, i, l, dp, lp, i]
        L.orc_capply_qh.argtypes = [i, i, i, dp, i, l, dp, dp, i, l, i, lp, i]
        L.orc_cbacksub.argtypes = [i, i, dp, i, l, dp, l, dp, l, ip, lp]
        L.orc_clstsq.argtypes = [i, i, i, dp, i, l, dp, l, dp, l, dp, ip, lp, i]
        L.orc_cexplicit_q.argtypes = [i, i, i, dp, i, l, dp, dp, i, l, i]
        L.orc_cmatvec.argtypes = [i, i, i, i, i, i, i, dp, i, l, dp, l, dp, l, dp, l, i]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _md(x, P):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(P))
    return a


def _nthreads(nthreads):
    if nthreads is not None:
        return int(nthreads)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# ------------------------------------------------------------------------------ md scalars
def md_add(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_md_add(a.size, _p(a), _p(b), _p(r))
    return r


def md_sub(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_md_sub(a.size, _p(a), _p(b), _p(r))
    return r


def md_mul(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_md_mul(a.size, _p(a), _p(b), _p(r))
    return r


def md_div(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_md_div(a.size, _p(a), _p(b), _p(r))
    return r


def md_sqrt(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_md_sqrt(a.size, _p(a), _p(r))
    return r


def md_round(P: int, terms):
    """Exact sum of the doubles in ``terms``, truncated to P limbs."""
    t = np.ascontiguousarray(np.asarray(terms, dtype=np.float64).ravel())
    r = np.zeros(P, dtype=np.float64)
    lib().orc_md_round(P, t.size, _p(t), _p(r))
    return r


# ------------------------------------------------------------------------------ matrices
def qr(A: np.ndarray, nthreads=None, tally=False):
    """Unblocked Householder QR. Returns (factored A copy, beta (P, n)[, tally])."""
    P, n, m = A.shape
    F = np.array(A, dtype=np.float64, order="C", copy=True)
    beta = np.zeros((P, n), dtype=np.float64)
    t = (ctypes.c_long * 4)()
    rc = lib().orc_qr(P, m, n, _p(F), m, m * n, _p(beta), t, _nthreads(nthreads))
    if rc:
        raise ValueError("orc_qr rejected its arguments (%d)" % rc)
    if tally:
        return F, beta, list(t)
    return F, beta


def apply_qt(F: np.ndarray, beta: np.ndarray, B: np.ndarray, nthreads=None):
    """Q^T B for B of shape (P, nrhs, m) (or (P, m) for one vector)."""
    P, n, m = F.shape
    vec = B.ndim == 2
    Bm = np.array(B.reshape(P, 1, m) if vec else B, dtype=np.float64, order="C", copy=True)
    nrhs = Bm.shape[1]
    rc = lib().orc_apply_qt(P, m, n, _p(np.ascontiguousarray(F)), m, m * n,
                            _p(np.ascontiguousarray(beta)), _p(Bm), m, m * nrhs, nrhs, None,
                            _nthreads(nthreads))
    if rc:
        raise ValueError("orc_apply_qt rejected its arguments (%d)" % rc)
    return Bm.reshape(P, m) if vec else Bm


def backsub(R: np.ndarray, y: np.ndarray, n: int | None = None):
    """Solve R(0:n,0:n) x = y(0:n). R has shape (P, cols, ldr). Returns (x, info)."""
    P, cols, ldr = R.shape
    if n is None:
        n = cols
    Rc = np.ascontiguousarray(R)
    yc = np.ascontiguousarray(y[:, :n])
    x = np.zeros((P, n), dtype=np.float64)
    info = ctypes.c_int(0)
    rc = lib().orc_backsub(P, n, _p(Rc), ldr, ldr * cols, _p(yc), n, _p(x), n,
                           ctypes.byref(info), None)
    if rc:
        raise ValueError("orc_backsub rejected its arguments (%d)" % rc)
    return x, info.value


def lstsq(A: np.ndarray, b: np.ndarray, nthreads=None, tally=False):
    """Least squares via unblocked Householder QR.

    Returns dict with x (P, n), qtb (P, m), F (factored A), beta, info[, tally].
    """
    P, n, m = A.shape
    F = np.array(A, dtype=np.float64, order="C", copy=True)
    bb = np.array(b, dtype=np.float64, order="C", copy=True).reshape(P, m)
    x = np.zeros((P, n), dtype=np.float64)
    beta = np.zeros((P, n), dtype=np.float64)
    info = ctypes.c_int(0)
    t = (ctypes.c_long * 4)()
    rc = lib().orc_lstsq(P, m, n, _p(F), m, m * n, _p(bb), m, _p(x), n, _p(beta),
                         ctypes.byref(info), t, _nthreads(nthreads))
    if rc:
        raise ValueError("orc_lstsq rejected its arguments (%d)" % rc)
    out = dict(x=x, qtb=bb, F=F, beta=beta, info=info.value)
    if tally:
        out["tally"] = list(t)
    return out


def explicit_q(F: np.ndarray, beta: np.ndarray, nthreads=None):
    """The m x m orthogonal factor, shape (P, m, m)."""
    P, n, m = F.shape
    Q = np.zeros((P, m, m), dtype=np.float64)
    rc = lib().orc_explicit_q(P, m, n, _p(np.ascontiguousarray(F)), m, m * n,
                              _p(np.ascontiguousarray(beta)), _p(Q), m, m * m,
                              _nthreads(nthreads))
    if rc:
        raise ValueError("orc_explicit_q rejected its arguments (%d)" % rc)
    return Q


def matvec(A: np.ndarray, x: np.ndarray, P_out: int, c: np.ndarray | None = None,
           trans: bool = False, nthreads=None):
    """Exactly accumulated ``op(A) x`` (or ``c - op(A) x``), truncated to P_out limbs.

    A: (Pa, cols, rows); x: (Px, len); c: (Pc, len_out).
    """
    Pa, cols, rows = A.shape
    Ac = np.ascontiguousarray(A)
    xc = np.ascontiguousarray(x)
    Px, xl = xc.shape
    nout = cols if trans else rows
    y = np.zeros((P_out, nout), dtype=np.float64)
    if c is not None:
        cc = np.ascontiguousarray(c)
        Pc, cl = cc.shape
        cp = _p(cc)
    else:
        Pc, cl, cp = 1, nout, None
    rc = lib().orc_matvec(1 if trans else 0, Pa, Px, Pc, P_out, rows, cols, _p(Ac), rows,
                          rows * cols, _p(xc), xl, cp, cl, _p(y), nout, _nthreads(nthreads))
    if rc:
        raise ValueError("orc_matvec rejected its arguments (%d)" % rc)
    return y


def rhs_for(A: np.ndarray, x_true: np.ndarray, P_out: int | None = None):
    """b = A x_true accumulated exactly and truncated to the working precision."""
    P = A.shape[0]
    return matvec(A, x_true, P if P_out is None else P_out)


# ------------------------------------------------------------------------------ complex
# A complex matrix of P-limb numbers is an array of shape (2, P, cols, rows): the real parts'
# limb planes, then the imaginary parts' (the paper keeps real and imaginary parts in
# separate arrays, end of Section 2).  A complex vector has shape (2, P, n).
def cmd_mul(a, b):
    """Complex product of two complex md scalars given as (2, P) arrays."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_cmd_mul(a.shape[-1], _p(a), _p(b), _p(r))
    return r


def cmd_div(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros_like(a)
    lib().orc_cmd_div(a.shape[-1], _p(a), _p(b), _p(r))
    return r


def cqr(A: np.ndarray, nthreads=None, tally=False):
    """Unblocked complex Householder QR. Returns (factored A copy, beta (P, n)[, tally])."""
    _, P, n, m = A.shape
    F = np.array(A, dtype=np.float64, order="C", copy=True)
    beta = np.zeros((P, n), dtype=np.float64)
    t = (ctypes.c_long * 4)()
    rc = lib().orc_cqr(P, m, n, _p(F), m, m * n, _p(beta), t, _nthreads(nthreads))
    if rc:
        raise ValueError("orc_cqr rejected its arguments (%d)" % rc)
    if tally:
        return F, beta, list(t)
    return F, beta


def capply_qh(F: np.ndarray, beta: np.ndarray, B: np.ndarray, nthreads=None):
    """Q^H B for B of shape (2, P, nrhs, m) (or (2, P, m) for one vector)."""
    _, P, n, m = F.shape
    vec = B.ndim == 3
    Bm = np.array(B.reshape(2, P, 1, m) if vec else B, dtype=np.float64, order="C", copy=True)
    nrhs = Bm.shape[2]
    rc = lib().orc_capply_qh(P, m, n, _p(np.ascontiguousarray(F)), m, m * n,
                             _p(np.ascontiguousarray(beta)), _p(Bm), m, m * nrhs, nrhs, None,
                             _nthreads(nthreads))
    if rc:
        raise ValueError("orc_capply_qh rejected its arguments (%d)" % rc)
    return Bm.reshape(2, P, m) if vec else Bm


def cbacksub(R: np.ndarray, y: np.ndarray, n: int | None = None):
    """Solve R(0:n,0:n) x = y(0:n), complex. R: (2, P, cols, ldr), y: (2, P, >= n)."""
    _, P, cols, ldr = R.shape
    if n is None:
        n = cols
    Rc = np.ascontiguousarray(R)
    yc = np.ascontiguousarray(y[:, :, :n])
    x = np.zeros((2, P, n), dtype=np.float64)
    info = ctypes.c_int(0)
    rc = lib().orc_cbacksub(P, n, _p(Rc), ldr, ldr * cols, _p(yc), n, _p(x), n, ctypes.byref(info), None)
    if rc:
        raise ValueError("orc_cbacksub rejected its arguments (%d)" % rc)
    return x, info.value


def clstsq(A: np.ndarray, b: np.ndarray, nthreads=None, tally=False):
    """Complex least squares via unblocked Householder QR.

    A: (2, P, n, m), b: (2, P, m).  Returns dict with x (2, P, n), qhb (2, P, m), F, beta,
    info[, tally].
    """
    _, P, n, m = A.shape
    F = np.array(A, dtype=np.float64, order="C", copy=True)
    bb = np.array(b, dtype=np.float64, order="C", copy=True).reshape(2, P, m)
    x = np.zeros((2, P, n), dtype=np.float64)
    beta = np.zeros((P, n), dtype=np.float64)
    info = ctypes.c_int(0)
    t = (ctypes.c_long * 4)()
    rc = lib().orc_clstsq(P, m, n, _p(F), m, m * n, _p(bb), m, _p(x), n, _p(beta), ctypes.byref(info), t,
                          _nthreads(nthreads))
    if rc:
        raise ValueError("orc_clstsq rejected its arguments (%d)" % rc)
    out = dict(x=x, qhb=bb, F=F, beta=beta, info=info.value)
    if tally:
        out["tally"] = list(t)
    return out


def cexplicit_q(F: np.ndarray, beta: np.ndarray, nthreads=None):
    """The m x m unitary factor, shape (2, P, m, m)."""
    _, P, n, m = F.shape
    Q = np.zeros((2, P, m, m), dtype=np.float64)
    rc = lib().orc_cexplicit_q(P, m, n, _p(np.ascontiguousarray(F)), m, m * n, _p(np.ascontiguousarray(beta)),
                               _p(Q), m, m * m, _nthreads(nthreads))
    if rc:
        raise ValueError("orc_cexplicit_q rejected its arguments (%d)" % rc)
    return Q


def cmatvec(A: np.ndarray, x: np.ndarray, P_out: int, c: np.ndarray | None = None, trans: bool = False,
            nthreads=None):
    """Exactly accumulated complex ``op(A) x`` (or ``c - op(A) x``), op(A) = A or A^H.

    A: (2, Pa, cols, rows); x: (2, Px, len); c: (2, Pc, len_out).
    """
    _, Pa, cols, rows = A.shape
    Ac = np.ascontiguousarray(A)
    xc = np.ascontiguousarray(x)
    _, Px, xl = xc.shape
    nout = cols if trans else rows
    y = np.zeros((2, P_out, nout), dtype=np.float64)
    if c is not None:
        cc = np.ascontiguousarray(c)
        _, Pc, cl = cc.shape
        cp = _p(cc)
    else:
        Pc, cl, cp = 1, nout, None
    rc = lib().orc_cmatvec(1 if trans else 0, Pa, Px, Pc, P_out, rows, cols, _p(Ac), rows, rows * cols, _p(xc), xl,
                           cp, cl, _p(y), nout, _nthreads(nthreads))
    if rc:
        raise ValueError("orc_cmatvec rejected its arguments (%d)" % rc)
    return y


# ------------------------------------------------------------------------------ md <-> exact
def to_fraction(limbs):
    """Exact rational value of one md number (sequence of doubles)."""
    from fractions import Fraction

    return sum((Fraction(float(v)) for v in limbs), Fraction(0))


def md_to_mpf(limbs):
    import mpmath

    s = mpmath.mpf(0)
    for v in limbs:
        s += mpmath.mpf(float(v))
    return s
