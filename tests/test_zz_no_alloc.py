"""The allocation-free solve (mdls_solve_noalloc, static device scratch) against mdls_solve
(caller workspace) through the C ABI: the same kernels in the same order, so A's factors, Q^T b,
x and info must agree bit for bit.  Two calls in a row per precision, the second smaller than
the first, so the second runs on the scratch the first left behind."""
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

    M.lib()  # raises if the HIP library is missing: there is no fallback
    torch.zeros(1, device=dev())
    return M


def problem(P, m, n, seed):
    A, _ = mdgen.ls_problem(P, m, n, seed)
    b = mdgen.md_vector(P, m, seed, mdgen.STREAM_B)
    return (torch.from_numpy(np.ascontiguousarray(A)).to(dev()),
            torch.from_numpy(np.ascontiguousarray(b)).to(dev()))


def run_pair(M, P, m, n, tile, seed):
    A, b = problem(P, m, n, seed)
    A1, b1 = A.clone(), b.clone()
    x1 = torch.full((P, n), float("nan"), dtype=torch.float64, device=dev())
    i1 = torch.full((1,), 7, dtype=torch.int32, device=dev())
    M.solve_noalloc(P, A1, b1, tile, x1, i1)
    A2, b2 = A.clone(), b.clone()
    x2, i2 = M.solve(P, A2, b2, tile)
    torch.cuda.synchronize()
    assert int(i1.item()) == 0 and int(i2.item()) == 0
    assert torch.equal(x1, x2), "x differs from mdls_solve"
    assert torch.equal(A1, A2), "factors differ from mdls_solve"
    assert torch.equal(b1, b2), "Q^T b differs from mdls_solve"
    assert bool(torch.isfinite(x1).all())


@pytest.mark.parametrize("P", [2, 4, 8])
def test_noalloc_matches_solve_twice(M, P):
    # a larger call, then a smaller one on the scratch it left behind
    for (m, n, tile, seed) in ((640, 384, 128, 900 + P), (96, 64, 16, 950 + P)):
        print("case noalloc P=%d m=%d n=%d tile=%d seed=%d" % (P, m, n, tile, seed), flush=True)
        run_pair(M, P, m, n, tile, seed)


def test_noalloc_headline_then_small(M):
    # the square n = 1024 double-double solve, then a small one
    for (m, n, tile, seed) in ((1024, 1024, 128, 990), (128, 128, 32, 991)):
        print("case noalloc P=2 m=%d n=%d tile=%d" % (m, n, tile), flush=True)
        run_pair(M, 2, m, n, tile, seed)


def test_noalloc_rejects_oversized(M):
    P, m, n, tile = 8, 4096, 2048, 256
    assert M.workspace_bytes(P, m, n, tile) > M.MDLS_NOALLOC_SCRATCH_BYTES
    A = torch.zeros((P, 1, 1), dtype=torch.float64, device=dev())
    one = int(A.data_ptr())
    rc = M.lib().mdls_solve_noalloc(P, m, n, tile, one, m, one, one, one, None)
    assert rc == M.MDLS_ESCRATCH
