"""GPU parity of the complex path (paper Section 3: Hermitian transpose in Algorithm 2;
Section 4, Table 5: complex double double QR of dimension 512 for tiles 32..256) through
the C ABI against the complex CPU oracle, element by element on seeded inputs.

Tolerance: ||x_gpu - x_or|| / ||x_or|| <= TOL[P] * max(1, kappa_2(A)) as for real data, and
the tight bound 64 n u_P kappa of the real full-size tests;
R, the Householder vectors and Q^H b against the oracle's at TOL[P] * max(1, kappa) relative
to the largest entry (the factors are unique once the phase convention of the diagonal is
fixed, which both sides share).
"""
import numpy as np
import pytest

import mdgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {1: 1e-12, 2: 1e-28, 4: 1e-58, 8: 1e-118}


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def M():
    import paper_2110_08375_amd as M

    M.lib()  # raises if the HIP library is missing: there is no fallback
    return M


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def limb_sum(d):
    """(P, ...) limb differences summed from the bottom limb up"""
    out = np.zeros(d.shape[1:])
    for k in range(d.shape[0] - 1, -1, -1):
        out = out + d[k]
    return out


def cerr(x, ref):
    """max-norm relative error of complex md arrays (2, P, ...)"""
    dre = limb_sum(x[0] - ref[0])
    dim = limb_sum(x[1] - ref[1])
    scale = max(float(np.max(np.abs(ref[0, 0]) + np.abs(ref[1, 0]))), 1e-300)
    return float(np.max(np.abs(dre) + np.abs(dim))) / scale


def kappa(A):
    return float(np.linalg.cond(A[0, 0].T + 1j * A[1, 0].T))


def upper(F, n):
    """upper triangle of the leading n x n block, (2, P, n, n) in column-major planes"""
    out = F[:, :, :n, :n].copy()
    for j in range(n):
        out[:, :, j, j + 1:] = 0.0
    return out


def lower(F, n):
    """strictly lower part (the Householder vectors), (2, P, n, m)"""
    out = F.copy()
    for j in range(n):
        out[:, :, j, :j + 1] = 0.0
    return out


def unit(P):
    """u_P = 2^-(53P - (P - 1)) (the tolerance unit of each precision)"""
    return 2.0 ** -(53 * P - (P - 1))


def report(case, err, bound, uk=None):
    if uk:
        print("%s err=%.3e bound=%.3e (%.2f u kappa)" % (case, err, bound, err / uk), flush=True)
    else:
        print("%s err=%.3e bound=%.3e" % (case, err, bound), flush=True)


CASES = [
    # P, m, n, tile
    (2, 128, 128, 32),   # square, 4 tiles, sigma = 0 in the last column
    (2, 200, 96, 32),    # tall
    (2, 300, 64, 16),    # more rows than threads per workgroup, ragged
    (2, 700, 40, 8),     # column steps with 3-4 rows per thread in registers
    (4, 1100, 32, 16),   # columns taller than the register-resident step (loop path)
    (2, 40, 24, 8),
    (4, 96, 64, 16),
    (4, 70, 70, 14),
    (8, 64, 48, 16),
    (8, 33, 20, 10),
    (8, 544, 64, 32),    # octo double: the first panel taller than the persistent panel's LDS column
    (4, 200, 128, 64),   # blocked T inversion (64-column tiles), quad double
    (8, 128, 128, 64),   # blocked T inversion and back-substitution tiles, octo double
    (4, 256, 256, 256),  # one 256-column panel: 256 persistent workgroups, 8 x 32 diagonal blocks
    (4, 900, 32, 16),    # quad double persistent panels of 900 and 884 rows (four rows per thread)
    (1, 128, 96, 32),
]


@pytest.fixture
def tuning(M):
    """set_tuning, with the complex panel form and the spin limit restored afterwards"""
    from paper_2110_08375_amd import mdls

    opts = (mdls.MDLS_TUNE_CPANEL, mdls.MDLS_TUNE_SPIN_LIMIT)
    saved = {o: M.get_tuning(o) for o in opts}
    yield M.set_tuning
    torch.cuda.synchronize()
    for o, v in saved.items():
        M.set_tuning(o, v)


@pytest.mark.parametrize("P,m,n,tile", CASES)
def test_csolve_matches_oracle(M, orc, P, m, n, tile):
    check_csolve(M, orc, P, m, n, tile)


@pytest.mark.parametrize("P,m,n,tile", [(2, 128, 128, 32), (2, 700, 40, 8), (4, 96, 64, 16), (8, 64, 48, 16)])
def test_csolve_per_column_panels(M, orc, tuning, P, m, n, tile):
    """The panel as one launch per column (the default for double and dd, and the form for
    columns taller than the persistent panel's LDS column) against the oracle."""
    from paper_2110_08375_amd import mdls

    tuning(mdls.MDLS_TUNE_CPANEL, 0)
    check_csolve(M, orc, P, m, n, tile)


@pytest.mark.parametrize("P,m,n,tile", [(2, 128, 128, 32), (2, 200, 96, 32), (2, 300, 64, 16), (2, 700, 40, 8),
                                        (2, 40, 24, 8), (1, 128, 96, 32), (4, 1100, 32, 16)])
def test_csolve_persistent_panels(M, orc, tuning, P, m, n, tile):
    """The persistent panel forced for every precision (its default is qd and od only) against
    the oracle, including sigma = 0 columns, ragged row counts and, for qd at 1100 rows, the
    first panel left to the per-column form."""
    from paper_2110_08375_amd import mdls

    tuning(mdls.MDLS_TUNE_CPANEL, 1)
    check_csolve(M, orc, P, m, n, tile)


def test_cpanel_wait_timeout(M, orc, tuning):
    """A persistent panel whose waits give up at once (spin limit 0, forced from the host:
    every kernel still ends): csolve reports info = -1 and cqr leaves R(0,0) = NaN; with the
    default limit the same calls succeed."""
    from paper_2110_08375_amd import mdls

    P, m, n, tile = 8, 64, 64, 64
    print("case cpanel timeout P=%d m=%d n=%d tile=%d" % (P, m, n, tile), flush=True)
    A, _ = mdgen.cls_problem(P, m, n, 3800)
    b = mdgen.cmd_vector(P, m, 3800, mdgen.STREAM_B)
    tuning(mdls.MDLS_TUNE_CPANEL, 1)
    tuning(mdls.MDLS_TUNE_SPIN_LIMIT, 0)
    x, info = M.csolve(P, to_gpu(A), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == -1
    Ag = to_gpu(A)
    M.cqr(P, Ag, tile)
    torch.cuda.synchronize()
    assert np.isnan(Ag.cpu().numpy()[0, 0, 0, 0])
    tuning(mdls.MDLS_TUNE_SPIN_LIMIT, 1 << 22)
    x, info = M.csolve(P, to_gpu(A), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert np.all(np.isfinite(x.cpu().numpy()))


@pytest.mark.parametrize("P", (2, 4, 8))
def test_cnan_input_propagates(M, tuning, P):
    """A NaN in A comes out as NaN in x through both panel forms (one launch per column, and the
    persistent panel whose hand-off counts arrivals, not values): every kernel exits, info stays
    0 (NaN is not an exact zero), and the next solve on the same stream is finite.  The same for
    a NaN in R given to the back substitution."""
    from paper_2110_08375_amd import mdls

    m, n, tile = 300, 96, 32
    A, _ = mdgen.cls_problem(P, m, n, 3900 + P)
    b = mdgen.cmd_vector(P, m, 3900 + P, mdgen.STREAM_B)
    An = A.copy()
    An[0, 0, 3, 5] = np.nan
    for cp in (0, 1):
        print("case cnan P=%d m=%d n=%d tile=%d cpanel=%d" % (P, m, n, tile, cp), flush=True)
        tuning(mdls.MDLS_TUNE_CPANEL, cp)
        x, info = M.csolve(P, to_gpu(An), to_gpu(b), tile)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert np.isnan(x.cpu().numpy()).any()
        x2, info2 = M.csolve(P, to_gpu(A), to_gpu(b), tile)
        torch.cuda.synchronize()
        assert int(info2.item()) == 0
        assert np.isfinite(x2.cpu().numpy()).all()
    R = mdgen.cmd_uniform(P, n, n, 3950 + P, mdgen.STREAM_A)
    R[1, 0, 70, 20] = np.nan  # imaginary part of R(20, 70), above the diagonal
    y, info3 = M.cbacksub(P, to_gpu(R), to_gpu(mdgen.cmd_vector(P, n, 3950 + P, mdgen.STREAM_B)), tile)
    torch.cuda.synchronize()
    assert int(info3.item()) == 0
    assert np.isnan(y.cpu().numpy()).any()


def check_csolve(M, orc, P, m, n, tile):
    print("case csolve P=%d m=%d n=%d tile=%d" % (P, m, n, tile), flush=True)
    A, _ = mdgen.cls_problem(P, m, n, 3000 + m + n)
    b = mdgen.cmd_vector(P, m, 3000 + m + n, mdgen.STREAM_B)
    ref = orc.clstsq(A, b)
    Ag, bg = to_gpu(A), to_gpu(b)
    x, info = M.csolve(P, Ag, bg, tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = kappa(A)
    bound = TOL[P] * max(1.0, k)
    uk = unit(P) * k
    tight = 64 * n * uk  # the tight bound of the real path's full-size tests
    Fg = Ag.cpu().numpy()
    for name, e in (("x", cerr(x.cpu().numpy(), ref["x"])), ("R", cerr(upper(Fg, n), upper(ref["F"], n))),
                    ("V", cerr(lower(Fg, n), lower(ref["F"], n))), ("Q^H b", cerr(bg.cpu().numpy(), ref["qhb"]))):
        report(name, e, bound, uk)
        assert e <= bound
        assert e <= tight


@pytest.mark.parametrize("P,m,n,tile,nrhs", [(2, 96, 64, 16, 3), (4, 80, 48, 16, 70), (8, 48, 32, 8, 2)])
def test_cqr_then_capply_qh(M, orc, P, m, n, tile, nrhs):
    """T from mdls_cqr applied by mdls_capply_qh to several right-hand sides (more than one
    chunk of columns for nrhs = 70) equals the oracle's Q^H B."""
    print("case cqr+capply P=%d m=%d n=%d tile=%d nrhs=%d" % (P, m, n, tile, nrhs), flush=True)
    A = mdgen.cmd_uniform(P, m, n, 3100 + m, mdgen.STREAM_A)
    B = mdgen.cmd_uniform(P, m, nrhs, 3100 + m, mdgen.STREAM_B)
    Fo, beta = orc.cqr(A)
    QhB = orc.capply_qh(Fo, beta, B)
    Ag, Bg = to_gpu(A), to_gpu(B)
    T = torch.zeros((2, P, n, tile), dtype=torch.float64, device=dev())
    M.cqr(P, Ag, tile, T=T)
    M.capply_qh(P, Ag, T, Bg, tile)
    torch.cuda.synchronize()
    bound = TOL[P] * max(1.0, kappa(A))
    e = cerr(Bg.cpu().numpy(), QhB)
    report("Q^H B", e, bound)
    assert e <= bound
    # diag(T_k) = beta
    Tn = T.cpu().numpy()
    for j in range(n):
        tj = Tn[:, :, j, j % tile]
        assert abs(limb_sum((tj[0] - beta[:, j])[:, None])[0]) <= bound * max(1.0, float(beta[0, j]))
        assert np.all(tj[1] == 0.0)


@pytest.mark.parametrize("P,n,tile", [(2, 96, 32), (4, 64, 16), (8, 40, 8), (2, 256, 256), (4, 192, 64), (8, 128, 128)])
def test_cbacksub_matches_oracle(M, orc, P, n, tile):
    print("case cbacksub P=%d n=%d tile=%d" % (P, n, tile), flush=True)
    R = mdgen.cmd_uniform(P, n, n, 3200 + n, mdgen.STREAM_A)
    for j in range(n):
        R[:, :, j, j + 1:] = 0.0
        R[0, 0, j, j] += 3.0 if R[0, 0, j, j] >= 0 else -3.0
    y = mdgen.cmd_vector(P, n, 3200 + n, mdgen.STREAM_B)
    xo, info = orc.cbacksub(R, y)
    assert info == 0
    Rg, xg = to_gpu(R), to_gpu(y)
    x, dinfo = M.cbacksub(P, Rg, xg, tile)
    torch.cuda.synchronize()
    assert int(dinfo.item()) == 0
    k = float(np.linalg.cond(R[0, 0].T + 1j * R[1, 0].T))
    e = cerr(x.cpu().numpy(), xo)
    report("x", e, TOL[P] * k, unit(P) * k)
    assert e <= TOL[P] * max(1.0, k)
    assert e <= 64 * n * unit(P) * max(1.0, k)


def test_cbacksub_zero_diagonal_info(M):
    P, n, tile = 2, 64, 16
    R = mdgen.cmd_uniform(P, n, n, 3300, mdgen.STREAM_A)
    R[:, :, 37, 37] = 0.0
    _, info = M.cbacksub(P, to_gpu(R), to_gpu(mdgen.cmd_vector(P, n, 3300, mdgen.STREAM_B)), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 38


def test_real_data_matches_real_path(M):
    """Zero imaginary parts: the complex solve's x equals the real solve's x."""
    P, m, n, tile = 4, 96, 64, 16
    A, _ = mdgen.ls_problem(P, m, n, 3400)
    b = mdgen.md_vector(P, m, 3400, mdgen.STREAM_B)
    xr, _ = M.solve(P, to_gpu(A), to_gpu(b), tile)
    Ac = to_gpu(np.stack([A, np.zeros_like(A)]))
    bc = to_gpu(np.stack([b, np.zeros_like(b)]))
    xc, info = M.csolve(P, Ac, bc, tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = float(np.linalg.cond(A[0].T))
    xr = xr.cpu().numpy()
    xc = xc.cpu().numpy()
    d = limb_sum(xc[0] - xr)
    assert float(np.max(np.abs(d))) / float(np.max(np.abs(xr[0]))) <= TOL[P] * max(1.0, k)
    assert float(np.max(np.abs(limb_sum(xc[1])))) / float(np.max(np.abs(xr[0]))) <= TOL[P] * max(1.0, k)


def test_table5_complex_dd_512(M, orc):
    """The paper's complex workload at full size: complex double double QR of a 512 x 512
    matrix (Table 5), here as a least-squares solve, for the four tile sizes of the table,
    each compared element by element with the oracle (x and R)."""
    P, n = 2, 512
    print("case table5 complex dd n=512", flush=True)
    A, _ = mdgen.cls_problem(P, n, n, 3500)
    b = mdgen.cmd_vector(P, n, 3500, mdgen.STREAM_B)
    ref = orc.clstsq(A, b)
    k = kappa(A)
    bound = TOL[P] * max(1.0, k)
    uk = unit(P) * k
    for tile in (128, 32, 64, 256):
        print("  tile %d" % tile, flush=True)
        Ag, bg = to_gpu(A), to_gpu(b)
        x, info = M.csolve(P, Ag, bg, tile)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        for name, e in (("x", cerr(x.cpu().numpy(), ref["x"])), ("R", cerr(upper(Ag.cpu().numpy(), n), upper(ref["F"], n)))):
            report("%s tile %d" % (name, tile), e, bound, uk)
            assert e <= bound
            assert e <= 64 * n * uk


def test_csolve_graph_replay(M, orc):
    """The complex solve captured into a HIP graph and replayed gives the eager result."""
    P, m, n, tile = 2, 128, 64, 32
    A, _ = mdgen.cls_problem(P, m, n, 3600)
    b = mdgen.cmd_vector(P, m, 3600, mdgen.STREAM_B)
    A0, b0 = to_gpu(A), to_gpu(b)
    Ag, bg = A0.clone(), b0.clone()
    ws = M.cworkspace(P, m, n, tile, dev())
    x = torch.empty((2, P, n), dtype=torch.float64, device=dev())
    info = torch.zeros(1, dtype=torch.int32, device=dev())
    M.csolve(P, Ag, bg, tile, x=x, ws=ws, info=info)
    torch.cuda.synchronize()
    x_eager = x.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Ag.copy_(A0)
        bg.copy_(b0)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            M.csolve(P, Ag, bg, tile, x=x, ws=ws, info=info)
    for _ in range(3):
        Ag.copy_(A0)
        bg.copy_(b0)
        x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, x_eager)


@pytest.mark.parametrize("P,m,n,tile", [(2, 48, 32, 16), (4, 40, 24, 8), (8, 24, 16, 8)])
def test_cform_q_matches_oracle(M, orc, P, m, n, tile):
    """The explicit unitary factor (the paper's Algorithm 2 forms Q) against the oracle's."""
    print("case cform_q P=%d m=%d n=%d tile=%d" % (P, m, n, tile), flush=True)
    A = mdgen.cmd_uniform(P, m, n, 3700 + m, mdgen.STREAM_A)
    Fo, beta = orc.cqr(A)
    Qo = orc.cexplicit_q(Fo, beta)
    Ag = to_gpu(A)
    T = torch.zeros((2, P, n, tile), dtype=torch.float64, device=dev())
    M.cqr(P, Ag, tile, T=T)
    Q = torch.zeros((2, P, m, m), dtype=torch.float64, device=dev())
    M.cform_q(P, Ag, T, tile, Q)
    torch.cuda.synchronize()
    bound = TOL[P] * max(1.0, kappa(A))
    e = cerr(Q.cpu().numpy(), Qo)
    report("Q", e, bound)
    assert e <= bound


def test_q_unitary_on_gpu(M):
    """Q^H Q = I for the 256 x 256 double double case, Q formed and applied on the GPU, and
    Q (Q^H B) = B."""
    P, n, tile = 2, 256, 64
    A = mdgen.cmd_uniform(P, n, n, 3800, mdgen.STREAM_A)
    Ag = to_gpu(A)
    T = torch.zeros((2, P, n, tile), dtype=torch.float64, device=dev())
    M.cqr(P, Ag, tile, T=T)
    Q = torch.zeros((2, P, n, n), dtype=torch.float64, device=dev())
    M.cform_q(P, Ag, T, tile, Q)
    QhQ = M.capply_qh(P, Ag, T, Q.clone(), tile)
    B = to_gpu(mdgen.cmd_uniform(P, n, 5, 3800, mdgen.STREAM_B))
    B2 = M.capply_q(P, Ag, T, M.capply_qh(P, Ag, T, B.clone(), tile), tile)
    torch.cuda.synchronize()
    I = np.zeros((2, P, n, n))
    for i in range(n):
        I[0, 0, i, i] = 1.0
    e = cerr(QhQ.cpu().numpy(), I)
    report("Q^H Q - I", e, 1e-28)
    assert e <= 1e-28
    e = cerr(B2.cpu().numpy(), B.cpu().numpy())
    report("Q Q^H B - B", e, 1e-28)
    assert e <= 1e-28
