"""The double-double update product S = Y^T C on the FP64 vector units and on the FP64 matrix
cores by exact slicing (the precision form's split-limb products; Section 3's GEMM-shaped
update stage), through the C ABI, against the oracle's exactly accumulated Y^T C.

Tolerance (normwise, per entry): |S - S_exact| <= 2^-98 * sum_k |Y(k,l)| |C(k,c)|: the slicing
leaves at most h * 2^-112 of max|Y| max|C| and the final rounding 2^-105 of |S|; the vector
method's lazy accumulation stays within a few units of 2^-104 per term.
"""
import numpy as np
import pytest

import mdgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def M():
    import paper_2110_08375_amd as M

    M.lib()
    return M


def exact_tn(orc, Y, C):
    """S (2, c, w) = Y^T C, each entry the exact sum rounded to dd (the oracle's matvec)."""
    _, w, h = Y.shape
    c = C.shape[1]
    S = np.zeros((2, c, w))
    for j in range(c):
        S[:, j, :] = orc.matvec(Y, np.ascontiguousarray(C[:, j, :]), 2, trans=True)
    return S


def check(S, Sx, Y, C, what):
    d = (S[1] - Sx[1]) + (S[0] - Sx[0])
    bound = 2.0 ** -98 * (np.abs(C[0]) @ np.abs(Y[0]).T)  # (c, w): sum_k |C(k,j)| |Y(k,l)|
    bound = np.maximum(bound, 1e-300)
    ratio = float(np.max(np.abs(d) / bound))
    print("%s max err / bound = %.3e" % (what, ratio), flush=True)
    assert ratio <= 1.0


@pytest.mark.parametrize("h,w,c", [(1024, 16, 1008), (333, 5, 37), (4, 16, 16), (1000, 16, 65), (2048, 16, 48)])
def test_split_and_vector_match_exact(M, orc, h, w, c):
    print("case dd_gemm_tn h=%d w=%d c=%d" % (h, w, c), flush=True)
    Y = mdgen.md_uniform(2, h, w, 4100 + h, mdgen.STREAM_A)
    C = mdgen.md_uniform(2, h, c, 4100 + h, mdgen.STREAM_B)
    C[:, :, :h // 3] *= 2.0 ** -40  # rows of very different size in each column
    Sx = exact_tn(orc, Y, C)
    Yg, Cg = torch.from_numpy(Y).to(dev()), torch.from_numpy(C).to(dev())
    for method in (0, 1):
        S = M.dd_gemm_tn(method, Yg, Cg)
        torch.cuda.synchronize()
        check(S.cpu().numpy(), Sx, Y, C, "method %d" % method)


def test_split_zero_column_and_limits(M):
    h, w, c = 64, 16, 20
    Y = mdgen.md_uniform(2, h, w, 4200, mdgen.STREAM_A)
    C = mdgen.md_uniform(2, h, c, 4200, mdgen.STREAM_B)
    C[:, 7, :] = 0.0
    S = M.dd_gemm_tn(1, torch.from_numpy(Y).to(dev()), torch.from_numpy(C).to(dev()))
    torch.cuda.synchronize()
    assert np.all(S.cpu().numpy()[:, 7, :] == 0.0)
    big = torch.zeros((2, 1, 2049), dtype=torch.float64, device=dev())
    with pytest.raises(Exception):
        M.dd_gemm_tn(1, big, big)  # h above the exactness bound is refused on the host
