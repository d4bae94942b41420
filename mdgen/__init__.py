"""Seeded, counter-based synthetic inputs for multiple-double least-squares problems.

This module is shared by the tests, the benchmark and the oracle harness. It holds no
multiple-double arithmetic: it only draws uniform numbers and scales them by exact powers
of two, so every limb it emits is an exactly representable double and the limbs of one
value are non-overlapping by construction.

Generator of record
-------------------
Each value is a pure function of ``(seed, stream, k)`` where ``k`` is the element's linear
counter inside its array.  The 64-bit word is the SplitMix64 output function (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to the
Weyl sequence point ``base + (k + 1) * GAMMA`` with ``base = mix(seed * GAMMA ^ stream *
STREAM_MUL)``.  The top 53 bits give a uniform ``u = (z >> 11) * 2**-52 - 1`` in ``[-1, 1)``
with resolution ``2**-52``.

Multiple-double entries (P limbs, limb 0 most significant) follow the paper's random
inputs (Section 4.1, notes on the implementation): limb 0 is ``u``; limb k >= 1 is
``u_k * 2**(e_{k-1} - 53)`` where ``2**e_{k-1} <= |limb_{k-1}| < 2**(e_{k-1}+1)``, i.e. a
uniform fraction of half an ulp of the limb above, so ``|limb_k| <= ulp(limb_{k-1}) / 2``.
A zero limb forces all lower limbs to zero.

Layout: arrays are returned limb-major (structure of arrays), shape ``(P, cols, rows)``,
C-contiguous, which is ``P`` column-major planes with leading dimension ``rows`` and plane
stride ``rows * cols`` — the storage the paper prescribes after Algorithm 1.

Two backends produce bit-identical values: numpy on the host and torch (any device), the
latter used to fill large matrices directly in device memory.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
STREAM_MUL = 0xD1B54A32D192ED03
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# Streams: one per logical array of a problem, so arrays never share counters.
STREAM_A = 1
STREAM_X = 2
STREAM_B = 3
STREAM_DIAG = 4
STREAM_U = 7
STREAM_V = 8
STREAM_IM = 16  # added to a stream number for the imaginary parts of complex data


def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def _base(seed: int, stream: int) -> int:
    return _mix_int(((seed * GAMMA) & MASK64) ^ ((stream * STREAM_MUL) & MASK64))


def uniform_scalar(seed: int, stream: int, k: int) -> float:
    """Reference (pure Python) value of counter ``k``; used to pin the vectorised paths."""
    z = _mix_int(_base(seed, stream) + (k + 1) * GAMMA)
    return (z >> 11) * 2.0 ** -52 - 1.0


# ----------------------------------------------------------------------------- numpy backend
def _uniform_np(seed: int, stream: int, k0: int, count: int) -> np.ndarray:
    base = np.uint64(_base(seed, stream))
    k = np.arange(k0 + 1, k0 + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = base + k * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


# ----------------------------------------------------------------------------- torch backend
def _to_i64(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(z, s: int):
    """Logical right shift of int64 tensors holding uint64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _uniform_torch(seed: int, stream: int, k0: int, count: int, device):
    import torch

    k = torch.arange(k0 + 1, k0 + 1 + count, dtype=torch.int64, device=device)
    z = k * _to_i64(GAMMA) + _to_i64(_base(seed, stream))
    z = (z ^ _srl(z, 30)) * _to_i64(MIX1)
    z = (z ^ _srl(z, 27)) * _to_i64(MIX2)
    z = z ^ _srl(z, 31)
    return _srl(z, 11).to(torch.float64) * 2.0 ** -52 - 1.0


def uniform(seed: int, stream: int, count: int, k0: int = 0, device=None):
    """``count`` consecutive uniforms in [-1, 1) starting at counter ``k0``.

    ``device=None`` returns numpy; otherwise a torch float64 tensor on ``device``.
    """
    if device is None:
        return _uniform_np(seed, stream, k0, count)
    return _uniform_torch(seed, stream, k0, count, device)


def _lower_limb(prev, u, xp):
    """u * 2**(e - 53) with 2**e <= |prev| < 2**(e+1).

    Zero where ``prev`` is zero or where the scale would leave the normal range, so every
    limb is a normal double (or zero) and the scaling is exact on both backends.
    """
    if xp == "np":
        _, ex = np.frexp(prev)  # prev = m * 2**ex with 0.5 <= |m| < 1, so e = ex - 1
        e = ex.astype(np.int64) - 54
        ok = (prev != 0.0) & (e >= -1022)
        scale = ((np.clip(e, -1022, 1023) + 1023) << 52).astype(np.int64).view(np.float64)
        return np.where(ok, u * scale, 0.0)
    import torch

    _, ex = torch.frexp(prev)
    e = ex.to(torch.int64) - 54
    ok = (prev != 0.0) & (e >= -1022)
    scale = ((torch.clamp(e, -1022, 1023) + 1023) << 52).view(torch.float64)
    return torch.where(ok, u * scale, torch.zeros_like(u))


def md_from_leading(lead, P: int, seed: int, stream: int, k0: int, device=None):
    """Attach P-1 lower limbs (drawn after counter block k0) to leading limbs ``lead``.

    Returns an array of shape ``(P,) + lead.shape``.  Lower limb k uses counters
    ``k0 + k * lead.size + idx``.
    """
    size = int(np.prod(lead.shape)) if device is None else lead.numel()
    if device is None:
        out = np.empty((P,) + tuple(lead.shape), dtype=np.float64)
        out[0] = lead
        for k in range(1, P):
            u = uniform(seed, stream, size, k0 + k * size).reshape(lead.shape)
            out[k] = _lower_limb(out[k - 1], u, "np")
        return out
    import torch

    out = torch.empty((P,) + tuple(lead.shape), dtype=torch.float64, device=device)
    out[0] = lead
    for k in range(1, P):
        u = uniform(seed, stream, size, k0 + k * size, device=device).reshape(lead.shape)
        out[k] = _lower_limb(out[k - 1], u, "torch")
    return out


def md_uniform(P: int, rows: int, cols: int, seed: int, stream: int, device=None):
    """Dense md matrix, entries as the module docstring; shape (P, cols, rows)."""
    n = rows * cols
    lead = uniform(seed, stream, n, 0, device=device).reshape(cols, rows)
    return md_from_leading(lead, P, seed, stream, 0, device=device)


def md_vector(P: int, n: int, seed: int, stream: int, device=None):
    """md vector, shape (P, n)."""
    return md_uniform(P, n, 1, seed, stream, device=device).reshape(P, n)


def md_ones(P: int, n: int, device=None):
    """The all-ones md vector (limbs 1, 0, ..., 0), shape (P, n)."""
    if device is None:
        out = np.zeros((P, n), dtype=np.float64)
        out[0] = 1.0
        return out
    import torch

    out = torch.zeros((P, n), dtype=torch.float64, device=device)
    out[0] = 1.0
    return out


def upper_triangular(P: int, n: int, seed: int, well_conditioned: bool = False, device=None):
    """Upper-triangular md matrix, shape (P, n, n) (column-major planes, ld = n).

    Off-diagonal entries above the diagonal are uniform in [-1, 1) (scaled by the exact
    power of two 2**-ceil(log2 n) when ``well_conditioned``); the diagonal's leading limb is
    ``fl(1 + (u + 1) / 2)`` in [1, 2]; entries below the diagonal are zero.
    """
    a = md_uniform(P, n, n, seed, STREAM_A, device=device)
    d = uniform(seed, STREAM_DIAG, n, 0, device=device)
    if device is None:
        dlead = 1.0 + (d + 1.0) * 0.5
        dmd = md_from_leading(dlead, P, seed, STREAM_DIAG, 0)
        i = np.arange(n)
        upper = (i[None, :] < i[:, None])  # [col, row]: row < col
        if well_conditioned:
            a = a * 2.0 ** -math.ceil(math.log2(n)) if n > 1 else a
        a = np.where(upper[None, :, :], a, 0.0)
        a[:, i, i] = dmd
        return np.ascontiguousarray(a)
    import torch

    dlead = 1.0 + (d + 1.0) * 0.5
    dmd = md_from_leading(dlead, P, seed, STREAM_DIAG, 0, device=device)
    if well_conditioned and n > 1:
        a.mul_(2.0 ** -math.ceil(math.log2(n)))
    i = torch.arange(n, device=device)
    upper = i[None, :] < i[:, None]
    a.mul_(upper[None, :, :].to(torch.float64))
    a[:, i, i] = dmd
    return a


def upper_triangular_exact(P: int, n: int, seed: int, device=None):
    """Upper-triangular R (P, n, n) and b = R * ones (P, n) with b exact by construction.

    Only limb 0 is nonzero.  Off-diagonal entries are uniforms rounded to multiples of 2**-25
    and scaled by 2**-s, s = ceil(log2 n); the diagonal is 1 + (u + 1)/2 rounded to a multiple
    of 2**-25, in [1, 2].  Every entry is a multiple of 2**-(25 + s) and every partial row sum
    is below 3, so for s <= 26 each row sum is exact in one double whatever the summation
    order, and the solution of R x = b is exactly the all-ones vector.  ||D^-1 N||_inf <=
    n 2**-s <= 1 keeps R well conditioned (the well-conditioned variant of the paper's
    back-substitution test, Section 4.1).
    """
    s = math.ceil(math.log2(n)) if n > 1 else 0
    assert s <= 26, "row sums would no longer be exact"
    lead = uniform(seed, STREAM_A, n * n, 0, device=device).reshape(n, n)  # [col, row]
    d = uniform(seed, STREAM_DIAG, n, 0, device=device)
    if device is None:
        q = np.round(lead * 2.0 ** 25) * 2.0 ** (-25 - s)
        i = np.arange(n)
        q = np.where(i[None, :] < i[:, None], q, 0.0)
        q[i, i] = 1.0 + np.round((d + 1.0) * 2.0 ** 24) * 2.0 ** -25
        R = np.zeros((P, n, n), dtype=np.float64)
        R[0] = q
        bv = np.zeros((P, n), dtype=np.float64)
        bv[0] = q.sum(axis=0)
        return R, bv
    import torch

    q = torch.round(lead * 2.0 ** 25) * 2.0 ** (-25 - s)
    i = torch.arange(n, device=device)
    q.mul_((i[None, :] < i[:, None]).to(torch.float64))
    q[i, i] = 1.0 + torch.round((d + 1.0) * 2.0 ** 24) * 2.0 ** -25
    R = torch.zeros((P, n, n), dtype=torch.float64, device=device)
    R[0] = q
    del q, lead
    bv = torch.zeros((P, n), dtype=torch.float64, device=device)
    bv[0] = R[0].sum(dim=0)
    return R, bv


def conditioned(P: int, m: int, n: int, seed: int, kappa: float = 1e8, reflectors: int = 8):
    """A = U diag(s) V^T (m x n) with s log-spaced from 1 down to 1/kappa, U and V products of
    `reflectors` Householder reflectors I - 2 u u^T / u^T u with uniform u (the precision-form
    workload); formed in float64 (numpy) as limb 0, lower limbs drawn as in md_uniform.
    Shape (P, n, m)."""
    s = np.logspace(0.0, -math.log10(kappa), n)
    M = np.zeros((m, n))
    M[np.arange(n), np.arange(n)] = s
    for k in range(reflectors):
        u = uniform(seed, STREAM_U, m, k * m)
        M -= np.outer(u, (2.0 / (u @ u)) * (u @ M))
    for k in range(reflectors):
        v = uniform(seed, STREAM_V, n, k * n)
        M -= np.outer((2.0 / (v @ v)) * (M @ v), v)
    return md_from_leading(np.ascontiguousarray(M.T), P, seed, STREAM_A, 0)


def conditioned_exact(P: int, m: int, n: int, seed: int, kappa: float = 1e8, reflectors: int = 8):
    """The precision-form matrix with a right-hand side that is exact by construction.

    A is the leading limb of ``conditioned`` rounded to a multiple of 2**-50 (a change below
    2**-51 per entry, which moves the singular values by less than 2**-51 sqrt(m n), far below
    1/kappa for the sizes used), stored as one nonzero limb of P; x_true has entries that are
    multiples of 1/16 in [-1, 1]; b = A x_true is formed in exact integer arithmetic (every
    product is an integer multiple of 2**-54) and split into its two leading doubles, which
    represent it exactly.  Returns A (P, n, m), x_true (P, n), b (P, m), all numpy."""
    A0 = conditioned(1, m, n, seed, kappa, reflectors)[0]          # (n, m) = [col, row]
    ia = np.round(A0 * 2.0 ** 50).astype(np.int64)                  # |A| <= 1, so |ia| <= 2**50
    ix = np.round(uniform(seed, STREAM_X, n) * 16.0).astype(np.int64)  # |ix| <= 16
    # sum_j ia_ij ix_j with ia = hi 2**25 + lo: two int64 products (|.| < 2**44 each), then Python ints
    hi = ia >> 25
    lo = ia - (hi << 25)
    s_hi = hi.T @ ix
    s_lo = lo.T @ ix
    A = np.zeros((P, n, m), dtype=np.float64)
    A[0] = ia.astype(np.float64) * 2.0 ** -50
    x = np.zeros((P, n), dtype=np.float64)
    x[0] = ix.astype(np.float64) / 16.0
    b = np.zeros((P, m), dtype=np.float64)
    for i in range(m):
        S = (int(s_hi[i]) << 25) + int(s_lo[i])                     # b_i = S 2**-54 exactly
        h = float(S)
        r = S - int(h)
        lo_d = float(r)
        assert r - int(lo_d) == 0, "b_i does not fit two doubles"
        b[0, i] = math.ldexp(h, -54)
        if P > 1:
            b[1, i] = math.ldexp(lo_d, -54)
    return A, x, b


def ls_problem(P: int, m: int, n: int, seed: int, ones_solution: bool = False, device=None):
    """A (P, n, m) and x_true (P, n) for a least-squares test problem."""
    A = md_uniform(P, m, n, seed, STREAM_A, device=device)
    x = md_ones(P, n, device=device) if ones_solution else md_vector(P, n, seed, STREAM_X, device=device)
    return A, x


def cmd_uniform(P: int, rows: int, cols: int, seed: int, stream: int, device=None):
    """Complex md matrix, shape (2, P, cols, rows): real parts drawn from ``stream``,
    imaginary parts from ``stream + STREAM_IM`` (real and imaginary parts in separate
    arrays, the paper's staging of complex data at the end of Section 2)."""
    re = md_uniform(P, rows, cols, seed, stream, device=device)
    im = md_uniform(P, rows, cols, seed, stream + STREAM_IM, device=device)
    if device is None:
        return np.stack([re, im])
    import torch

    return torch.stack([re, im]).contiguous()


def cmd_vector(P: int, n: int, seed: int, stream: int, device=None):
    """Complex md vector, shape (2, P, n)."""
    return cmd_uniform(P, n, 1, seed, stream, device=device).reshape(2, P, n)


def cls_problem(P: int, m: int, n: int, seed: int, device=None):
    """Complex A (2, P, n, m) and x_true (2, P, n) for a least-squares test problem."""
    return (cmd_uniform(P, m, n, seed, STREAM_A, device=device),
            cmd_vector(P, n, seed, STREAM_X, device=device))


def batch_shapes(count: int, seed: int, m_lo: int = 32, m_hi: int = 512, n_lo: int = 16):
    """(m, n) pairs with m uniform in [m_lo, m_hi] and n uniform in [n_lo, m]."""
    u1 = uniform(seed, 5, count)
    u2 = uniform(seed, 6, count)
    ms = m_lo + np.floor((u1 + 1.0) * 0.5 * (m_hi - m_lo + 1)).astype(np.int64)
    ms = np.minimum(ms, m_hi)
    ns = n_lo + np.floor((u2 + 1.0) * 0.5 * (ms - n_lo + 1)).astype(np.int64)
    ns = np.minimum(ns, ms)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]
