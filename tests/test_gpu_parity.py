"""GPU parity: the HIP library (through its C ABI) against the CPU oracle, element by element,
on seeded synthetic inputs.

Tolerance (forward error of x): ||x_gpu - x_ref|| / ||x_ref|| <= TOL[P] * max(1, kappa_2(A)),
with TOL = 1e-28 (dd), 1e-58 (qd), 1e-118 (od) and kappa_2 from the leading limbs in FP64.
The unit roundoffs are 2^-105, 2^-209 and 2^-417, so the tolerance leaves room for the
O(n) growth of rounding errors in QR and back substitution.  Beside it, the oracle comparisons
apply a tight bound, err <= 64 n u_P kappa (u_P = 2^-(53P - P + 1)), which a loss of 20
low-order bits anywhere in the path would break, and print err / (u_P kappa).
"""
import os

import numpy as np
import pytest

import mdgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {1: 1e-12, 2: 1e-28, 4: 1e-58, 8: 1e-118}


def unit(P):
    """u_P = 2^-(53P - (P - 1)) (the tolerance unit of each precision)"""
    return 2.0 ** -(53 * P - (P - 1))


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def M():
    import paper_2110_08375_amd as M

    M.lib()  # raises if the HIP library is missing: there is no fallback
    torch.zeros(1, device=dev())
    M.init()  # the look-ahead side stream of this thread
    return M


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def md_err(x, ref):
    """max-norm relative error of md vectors (P, n), in float via limb sums of the difference"""
    d = np.zeros(ref.shape[1])
    # difference limb-wise then summed from the bottom: exact enough for an error estimate
    for k in range(ref.shape[0] - 1, -1, -1):
        d = d + (x[k] - ref[k])
    return np.max(np.abs(d)) / max(np.max(np.abs(ref[0])), 1e-300)


def kappa(A):
    return float(np.linalg.cond(A[0].T))


def report(case, err, bound):
    print("%s err=%.3e bound=%.3e" % (case, err, bound), flush=True)


CASES = [
    # P, m, n, tile, ones_solution
    (2, 128, 128, 32, True),    # the small square double-double case (4 tiles)
    (2, 200, 96, 32, False),    # tall
    (2, 77, 40, 8, False),      # ragged rows
    (4, 96, 64, 16, False),
    (4, 100, 36, 12, False),
    (8, 64, 48, 16, False),
    (8, 50, 30, 10, False),     # ragged last panel
    (1, 128, 96, 32, False),
]


@pytest.mark.parametrize("P,m,n,tile,ones", CASES)
def test_solve_matches_oracle(M, orc, P, m, n, tile, ones):
    print("case solve P=%d m=%d n=%d tile=%d" % (P, m, n, tile), flush=True)
    A, xt = mdgen.ls_problem(P, m, n, 1000 + m + n, ones_solution=ones)
    b = orc.rhs_for(A, xt) if ones else mdgen.md_vector(P, m, 7 + n, mdgen.STREAM_B)
    ref = orc.lstsq(A, b)
    Ag, bg = to_gpu(A), to_gpu(b)
    x, info = M.solve(P, Ag, bg, tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    xg = x.cpu().numpy()
    k = kappa(A)
    tight = 64 * n * unit(P) * k  # beside the contract, the tight bound of the full-size tests
    err = md_err(xg, ref["x"])
    report("x", err, TOL[P] * max(1, k))
    assert err <= TOL[P] * max(1.0, k)
    assert err <= tight
    # R (upper triangle of the factored A) against the oracle's R
    Fg = Ag.cpu().numpy()
    Rg = np.stack([np.triu(Fg[l].T[:n, :]) for l in range(P)])
    Ro = np.stack([np.triu(ref["F"][l].T[:n, :]) for l in range(P)])
    dR = np.zeros_like(Rg[0])
    for l in range(P - 1, -1, -1):
        dR = dR + (Rg[l] - Ro[l])
    eR = np.max(np.abs(dR)) / np.max(np.abs(Ro[0]))
    assert eR <= TOL[P] * max(1, k)
    assert eR <= tight
    # Q^T b against the oracle (the part below n carries the residual)
    qerr = md_err(bg.cpu().numpy(), ref["qtb"])
    assert qerr <= TOL[P] * max(1, k)
    assert qerr <= tight
    print("  x %.2f, R %.2f, Q^T b %.2f u kappa" % (err / (unit(P) * k), eR / (unit(P) * k), qerr / (unit(P) * k)),
          flush=True)


@pytest.fixture
def tuning(M):
    """set_tuning inside a test; every option is restored afterwards"""
    from paper_2110_08375_amd import mdls

    opts = (mdls.MDLS_TUNE_LOOKAHEAD, mdls.MDLS_TUNE_PANEL_VARIANT, mdls.MDLS_TUNE_APPLY_GRID_CAP,
            mdls.MDLS_TUNE_APPLY_WIDE_ROWS, mdls.MDLS_TUNE_SPIN_LIMIT)
    saved = {o: M.get_tuning(o) for o in opts}
    yield M.set_tuning
    torch.cuda.synchronize()
    for o, v in saved.items():
        M.set_tuning(o, v)


@pytest.mark.parametrize("P,variant", [(2, 0), (4, 0), (8, 1), (8, 0)])
def test_multi_workgroup_panel(M, orc, tuning, P, variant):
    """Small workgroups spread a 700-row panel over several workgroups (grid barrier), with
    and without the concurrent side-stream update."""
    from paper_2110_08375_amd import mdls

    tuning(mdls.MDLS_TUNE_PANEL_VARIANT, variant)
    m, n, tile = 700, 64, 16
    print("case multi-wg P=%d variant=%d" % (P, variant), flush=True)
    A, xt = mdgen.ls_problem(P, m, n, 55)
    b = orc.rhs_for(A, xt)
    ref = orc.lstsq(A, b)
    outs = []
    for la in (1, 0):
        tuning(mdls.MDLS_TUNE_LOOKAHEAD, la)
        x, info = M.solve(P, to_gpu(A), to_gpu(b), tile)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert md_err(x.cpu().numpy(), ref["x"]) <= TOL[P] * max(1, kappa(A))
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])  # same arithmetic in the same order


@pytest.mark.parametrize("P", (2, 4, 8))
def test_qr_t_apply_qt_and_w(M, orc, P):
    m, n, tile = 40, 16, 8
    print("case qr/T/W P=%d" % P, flush=True)
    A = mdgen.md_uniform(P, m, n, 77, mdgen.STREAM_A)
    B = mdgen.md_uniform(P, m, 3, 78, mdgen.STREAM_B)
    Fo, beta = orc.qr(A)
    qtb_ref = orc.apply_qt(Fo, beta, B)
    Ag = to_gpu(A)
    T = torch.zeros((P, n, tile), dtype=torch.float64, device=dev())
    bg = torch.full((P, n), 7.0, dtype=torch.float64, device=dev())
    info = torch.full((1,), 5, dtype=torch.int32, device=dev())
    M.qr(P, Ag, tile, T=T, beta=bg, info=info)
    Bg = to_gpu(B)
    M.apply_qt(P, Ag, T, Bg, tile)
    W = torch.zeros((P, n, m), dtype=torch.float64, device=dev())
    M.form_w(P, Ag, T, tile, W)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = kappa(A)
    # the betas against the oracle's
    assert md_err(bg.cpu().numpy(), beta) <= TOL[P] * max(1, k)
    Bq = Bg.cpu().numpy()
    for c in range(3):
        assert md_err(Bq[:, c, :], qtb_ref[:, c, :]) <= TOL[P] * max(1, k)
    # diag(T_k) = beta, T_k upper triangular
    Tn = T.cpu().numpy()
    for j in range(n):
        blk, jj = divmod(j, tile)
        assert md_err(Tn[:, j, jj:jj + 1], beta[:, j:j + 1]) <= TOL[P]
        assert np.all(Tn[:, j, jj + 1:] == 0.0)
    # P_WY = I + W_k Y_k^T equals the oracle's product of the block's reflectors (first block):
    # column c of I + W Y^T is e_c + W Y(c, :)^T, accumulated exactly by the oracle
    Fg = Ag.cpu().numpy()
    Wn = W.cpu().numpy()
    Qo = orc.explicit_q(Fo[:, :tile, :], beta[:, :tile])
    Wb = np.ascontiguousarray(Wn[:, :tile, :])
    for c in range(m):
        yrow = np.zeros((P, tile))
        for l in range(tile):
            if c > l:
                yrow[:, l] = Fg[:, l, c]
            elif c == l:
                yrow[0, l] = 1.0
        ec = np.zeros((P, m))
        ec[0, c] = 1.0
        col = orc.matvec(Wb, yrow, P, c=-ec)  # -e_c - W y  ->  negate
        assert md_err(-col, Qo[:, c, :]) <= TOL[P] * 10


@pytest.mark.parametrize("P,n,tile", [(2, 512, 128), (4, 384, 64), (8, 128, 32), (4, 256, 256)])
def test_backsub_matches_oracle(M, orc, P, n, tile):
    print("case backsub P=%d n=%d tile=%d" % (P, n, tile), flush=True)
    R = mdgen.upper_triangular(P, n, 5, well_conditioned=True)
    y = mdgen.md_vector(P, n, 5, mdgen.STREAM_B)
    xo, info_o = orc.backsub(R, y)
    assert info_o == 0
    x = to_gpu(y)
    x, info = M.backsub(P, to_gpu(R), x, tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    err = md_err(x.cpu().numpy(), xo)
    report("bs", err, TOL[P])
    assert err <= TOL[P] * 10
    k = float(np.linalg.cond(R[0].T))
    print("  %.2f u kappa (kappa %.2f)" % (err / (unit(P) * k), k), flush=True)
    assert err <= 64 * n * unit(P) * k


def test_zero_diagonal_sets_info(M):
    P, n, tile = 2, 64, 16
    R = mdgen.upper_triangular(P, n, 3, well_conditioned=True)
    R[:, 37, 37] = 0.0
    R[:, 50, 50] = 0.0
    x, info = M.backsub(P, to_gpu(R), to_gpu(mdgen.md_vector(P, n, 3, 3)), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 38
    A = mdgen.md_uniform(P, 80, n, 4, mdgen.STREAM_A)
    A[:, 9, :] = 0.0  # zero column: R(9,9) is exactly zero
    x, info = M.solve(P, to_gpu(A), to_gpu(mdgen.md_vector(P, 80, 4, 3)), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 10


def test_upper_triangular_input_gives_r_equal_a(M):
    """sigma = 0 in every column: beta = 0, R = A bit for bit (Golub-Van Loan 5.1.1)."""
    P, n = 4, 32
    R = mdgen.upper_triangular(P, n, 8)
    R[:, 5, 5] *= -1.0
    Ag = to_gpu(R)
    T = torch.zeros((P, n, 16), dtype=torch.float64, device=dev())
    M.qr(P, Ag, 16, T=T)
    torch.cuda.synchronize()
    assert np.array_equal(Ag.cpu().numpy(), R)
    assert np.all(T.cpu().numpy() == 0.0)


def test_run_to_run_bitwise(M):
    P, m, n, tile = 2, 300, 128, 32
    A, xt = mdgen.ls_problem(P, m, n, 4)
    b = mdgen.md_vector(P, m, 4, 3)
    outs = []
    for _ in range(2):
        x, info = M.solve(P, to_gpu(A), to_gpu(b), tile)
        torch.cuda.synchronize()
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def md_diff_max(X, Y):
    """max |X - Y| of two md arrays (limb axis first), the limb differences summed from the bottom"""
    d = np.zeros(X.shape[1:])
    for k in range(X.shape[0] - 1, -1, -1):
        d = d + (X[k] - Y[k])
    return float(np.max(np.abs(d)))


# The headline workload (Section 4, Table 11: least squares on 1024 x 1024, 8 tiles of 128) in
# dd and qd, its tall 2048 x 1024 variant in dd, and od at 768 x 768, the largest square size whose
# oracle run fits the test budget and still reaches the full-size paths of the factorisation:
# 256-row trailing-update units (at least 2 x 256 units in the first panels) and the od update's
# switch from 448 to 224 workgroups below 768 rows.
HEADLINE = [(2, 1024, 1024, 128), (4, 1024, 1024, 128), (2, 2048, 1024, 128), (8, 768, 768, 128)]


@pytest.mark.parametrize("P,m,n,tile", HEADLINE)
def test_full_size_matches_oracle(M, orc, P, m, n, tile):
    """R, Q^T b, x and the Householder vectors of the full-size solve against the oracle's
    unblocked solve of the same data, element by element, with the kappa-scaled contract and the tight bound 64 n u_P kappa;
    x also against x_true (b = A x_true formed exactly by the oracle, rounded to P limbs)."""
    print("case full-size oracle P=%d m=%d n=%d tile=%d" % (P, m, n, tile), flush=True)
    A, xt = mdgen.ls_problem(P, m, n, 2000 + P)
    b = orc.rhs_for(A, xt)
    ref = orc.lstsq(A, b)
    print("  oracle done", flush=True)
    Ag, bg = to_gpu(A), to_gpu(b)
    x, info = M.solve(P, Ag, bg, tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = kappa(A)
    u = unit(P)
    tight = 64 * n * u * k
    loose = TOL[P] * max(1.0, k)
    xg = x.cpu().numpy()
    ex = md_err(xg, ref["x"])
    et = md_err(xg, xt)
    Fg = Ag.cpu().numpy()
    Rg = np.stack([np.triu(Fg[l].T[:n, :]) for l in range(P)])
    Ro = np.stack([np.triu(ref["F"][l].T[:n, :]) for l in range(P)])
    eR = md_diff_max(Rg, Ro) / float(np.max(np.abs(Ro[0])))
    eq = md_err(bg.cpu().numpy(), ref["qtb"])
    # the Householder vectors below the diagonal (unit first entries implicit)
    Vg = np.stack([np.tril(Fg[l].T, -1) for l in range(P)])
    Vo = np.stack([np.tril(ref["F"][l].T, -1) for l in range(P)])
    ev = md_diff_max(Vg, Vo) / float(np.max(np.abs(Vo[0])))
    print("  kappa %.3e; x vs oracle %.3e (%.2f u kappa), x vs x_true %.3e (%.2f u kappa), "
          "R %.3e (%.2f u kappa), Q^T b %.3e (%.2f u kappa), v %.3e (%.2f u kappa); tight bound %.3e"
          % (k, ex, ex / (u * k), et, et / (u * k), eR, eR / (u * k), eq, eq / (u * k), ev, ev / (u * k), tight),
          flush=True)
    for e in (ex, et, eR, eq, ev):
        assert e <= loose
        assert e <= tight


@pytest.mark.parametrize("P", (2, 4, 8))
def test_nan_input_propagates(M, P):
    """A NaN in A comes out as NaN in x, every kernel exits, d_info stays 0 (NaN is not an
    exact zero), and the next solve on the same stream is unaffected."""
    m, n, tile = 300, 128, 32
    A, xt = mdgen.ls_problem(P, m, n, 31)
    b = mdgen.md_vector(P, m, 31, mdgen.STREAM_B)
    An = A.copy()
    An[0, 3, 5] = np.nan
    x, info = M.solve(P, to_gpu(An), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    xh = x.cpu().numpy()
    assert np.isnan(xh).any()
    x2, info2 = M.solve(P, to_gpu(A), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info2.item()) == 0
    assert np.isfinite(x2.cpu().numpy()).all()
    # back substitution with a NaN in R
    R = mdgen.upper_triangular(P, n, 5, well_conditioned=True)
    R[0, 70, 20] = np.nan
    y = to_gpu(mdgen.md_vector(P, n, 5, mdgen.STREAM_B))
    y, info3 = M.backsub(P, to_gpu(R), y, tile)
    torch.cuda.synchronize()
    assert int(info3.item()) == 0
    assert np.isnan(y.cpu().numpy()).any()


@pytest.mark.parametrize("P", (2, 8))
def test_barrier_timeout_reports_minus_one(M, orc, tuning, P):
    """With a spin limit of zero polls the panel's grid barriers give up at once: every kernel
    still exits, the solve and the QR report d_info = -1.  With the limit restored the same
    problem solves normally."""
    from paper_2110_08375_amd import mdls

    m, n, tile = 700, 64, 16  # 11 (dd) / 11 (od) panel workgroups
    A, xt = mdgen.ls_problem(P, m, n, 57)
    b = orc.rhs_for(A, xt)
    tuning(mdls.MDLS_TUNE_SPIN_LIMIT, 0)
    x, info = M.solve(P, to_gpu(A), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == -1
    qinfo = torch.full((1,), 9, dtype=torch.int32, device=dev())
    M.qr(P, to_gpu(A), tile, info=qinfo)
    torch.cuda.synchronize()
    assert int(qinfo.item()) == -1
    tuning(mdls.MDLS_TUNE_SPIN_LIMIT, 1 << 22)
    x, info = M.solve(P, to_gpu(A), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert md_err(x.cpu().numpy(), xt) <= TOL[P] * max(1.0, kappa(A))
    M.qr(P, to_gpu(A), tile, info=qinfo)
    torch.cuda.synchronize()
    assert int(qinfo.item()) == 0


def test_backsub_full_size_exact_rhs(M):
    """Back substitution at the largest size of the paper's back-substitution tests (upper
    triangular, quad double, n = 17 920, tile 256, Section 4.1): b = R * ones is exact by
    construction, so x must be all ones to the qd tolerance (kappa_inf(R) < 10 here)."""
    from fractions import Fraction

    from paper_2110_08375_amd import opcount

    P, n, tile = 4, 17920, 256
    print("case backsub full-size P=4 n=17920 tile=256", flush=True)
    R, b = mdgen.upper_triangular_exact(P, n, 11, device=dev())
    ws = M.workspace(P, n, n, tile, dev())
    info = torch.zeros(1, dtype=torch.int32, device=dev())
    ms = []
    for _ in range(2):
        x = b.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        M.backsub(P, R, x, tile, ws=ws, info=info)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    assert int(info.item()) == 0
    xh = x.cpu().numpy()
    err = md_err(xh, mdgen.md_ones(P, n))
    tf = opcount.backsub_double_ops(P, n) / (ms[-1] * 1e-3) / 1e12
    print("backsub n=17920 qd: %.3f ms, %.3f Table-1 TFLOP/s, err %.3e" % (ms[-1], tf, err), flush=True)
    assert err <= TOL[P] * 10
    for i in range(0, n, 997):  # exact check of a sample
        v = sum(Fraction(float(xh[k, i])) for k in range(P))
        assert abs(v - 1) <= Fraction(TOL[P] * 10)


def test_solve_graph_replay(M):
    """A least-squares solve (look-ahead side stream included) captured in a graph and replayed
    three times, with eager restores of A and b between replays: each replay equals the eager
    solve bit for bit."""
    P, m, n, tile = 4, 300, 128, 32
    A, _ = mdgen.ls_problem(P, m, n, 12)
    b = mdgen.md_vector(P, m, 12, 3)
    A0, b0 = to_gpu(A), to_gpu(b)
    Aw, bw = A0.clone(), b0.clone()
    x = torch.zeros((P, n), dtype=torch.float64, device=dev())
    ws = M.workspace(P, m, n, tile, dev())
    info = torch.zeros(1, dtype=torch.int32, device=dev())
    M.solve(P, Aw, bw, tile, x=x, ws=ws, info=info)
    torch.cuda.synchronize()
    ref = x.cpu().numpy().copy()
    Aw.copy_(A0)
    bw.copy_(b0)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        M.solve(P, Aw, bw, tile, x=x, ws=ws, info=info)
    torch.cuda.synchronize()
    for rep in range(3):
        Aw.copy_(A0)
        bw.copy_(b0)
        x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), ref), rep
        assert int(info.item()) == 0


@pytest.mark.parametrize("P", (2, 4, 8))
def test_form_q_matches_oracle(M, orc, P):
    """The explicit orthogonal factor (the paper's Algorithm 2 forms Q) against the oracle's
    backward accumulation of its own reflectors, column by column."""
    m, n, tile = 40, 16, 8
    print("case form_q P=%d" % P, flush=True)
    A = mdgen.md_uniform(P, m, n, 91, mdgen.STREAM_A)
    Fo, beta = orc.qr(A)
    Qo = orc.explicit_q(Fo, beta)
    Ag = to_gpu(A)
    T = torch.zeros((P, n, tile), dtype=torch.float64, device=dev())
    M.qr(P, Ag, tile, T=T)
    Q = torch.zeros((P, m, m), dtype=torch.float64, device=dev())
    M.form_q(P, Ag, T, tile, Q)
    torch.cuda.synchronize()
    Qn = Q.cpu().numpy()
    k = kappa(A)
    for c in range(m):
        assert md_err(Qn[:, c, :], Qo[:, c, :]) <= TOL[P] * max(1, k) * 10, c


@pytest.mark.parametrize("P", (2, 8))
def test_apply_q_inverts_apply_qt(M, P):
    """Q (Q^T B) = B on random right-hand sides (m = 300, n = 128, tile 32)."""
    m, n, tile = 300, 128, 32
    A = mdgen.md_uniform(P, m, n, 92, mdgen.STREAM_A)
    B = mdgen.md_uniform(P, m, 5, 93, mdgen.STREAM_B)
    Ag = to_gpu(A)
    T = torch.zeros((P, n, tile), dtype=torch.float64, device=dev())
    M.qr(P, Ag, tile, T=T)
    Bg = to_gpu(B)
    M.apply_qt(P, Ag, T, Bg, tile)
    M.apply_q(P, Ag, T, Bg, tile)
    torch.cuda.synchronize()
    Bn = Bg.cpu().numpy()
    for c in range(5):
        assert md_err(Bn[:, c, :], B[:, c, :]) <= TOL[P] * 100, c
