"""Operation counts for reporting throughput the way the paper does.

The paper converts multiple-double operations into double-precision operations with its
Table 1 (Section 1.1) and divides the tally by kernel time (Section 4).  The weights below
restate that table: double-precision operations per multiple-double add, multiply and
divide.

``ls_md_fmas(m, n)`` is the algorithmic size of the least-squares solve in multiple-double
multiply-add pairs: Householder QR of an m x n matrix (m n^2 - n^3/3), Q^T b (2 m n - n^2)
and back substitution (n (n - 1) / 2).  ``ls_double_ops`` weights it with Table 1 and adds
3 n divisions (beta and the Householder vector per column, the back-substitution divide;
the square root is weighted as a division).  This algorithmic count deliberately leaves out
the extra work an implementation does (compact-WY factors, tile inversions), so it is the
same for every implementation of the method.
"""
from __future__ import annotations

# precision (limbs) -> (add, mul, div) double operations, paper Table 1
TABLE1 = {
    2: (20, 23, 70),
    4: (89, 336, 893),
    8: (269, 1742, 5126),
}
NAMES = {1: "d", 2: "dd", 4: "qd", 8: "od"}


def weights(p: int):
    if p == 1:
        return (1, 1, 1)
    return TABLE1[p]


def ls_md_fmas(m: int, n: int) -> float:
    return (m * n * n - n ** 3 / 3.0) + (2.0 * m * n - n * n) + n * (n - 1) / 2.0


def ls_double_ops(p: int, m: int, n: int) -> float:
    wa, wm, wd = weights(p)
    return (wa + wm) * ls_md_fmas(m, n) + 3.0 * n * wd


def backsub_double_ops(p: int, n: int) -> float:
    """Back substitution of an n x n triangular system: n(n-1)/2 md multiply-adds and n divisions
    (the algorithmic count; the tile inversions the method adds are not counted)."""
    wa, wm, wd = weights(p)
    return (wa + wm) * n * (n - 1) / 2.0 + n * wd


def cqr_double_ops(p: int, m: int, n: int) -> float:
    """Complex Householder QR of an m x n matrix: a complex multiply-add is four real ones
    (4 multiplications, 4 additions), so four times the real count (m n^2 - n^3/3 md
    multiply-adds and 2 n divisions); the paper gives the same factor of about four for
    complex data (Section 4, before Table 5)."""
    wa, wm, wd = weights(p)
    return 4.0 * ((wa + wm) * (m * n * n - n ** 3 / 3.0) + 2.0 * n * wd)


def md_fma_double_ops(p: int) -> int:
    wa, wm, _ = weights(p)
    return wa + wm


# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
