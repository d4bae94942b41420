"""GPU parity: the HIP library (through its C ABI) against the CPU oracle, element by element,
on seeded synthetic inputs.

Tolerance (forward error of x): ||x_gpu - x_ref|| / ||x_ref|| <= TOL[P] * max(1, kappa_2(A)),
with TOL = 1e-28 (dd), 1e-58 (qd), 1e-118 (od) and kappa_2 from the leading limbs in FP64.
The unit roundoffs are 2^-105, 2^-209 and 2^-417, so the tolerance leaves room for the
O(n) growth of rounding errors in QR and back substitution.
"""
import os

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
    err = md_err(xg, ref["x"])
    report("x", err, TOL[P] * max(1, k))
    assert err <= TOL[P] * max(1.0, k)
    # R (upper triangle of the factored A) against the oracle's R
    Fg = Ag.cpu().numpy()
    Rg = np.stack([np.triu(Fg[l].T[:n, :]) for l in range(P)])
    Ro = np.stack([np.triu(ref["F"][l].T[:n, :]) for l in range(P)])
    dR = np.zeros_like(Rg[0])
    for l in range(P - 1, -1, -1):
        dR = dR + (Rg[l] - Ro[l])
    assert np.max(np.abs(dR)) <= TOL[P] * max(1, k) * np.max(np.abs(Ro[0]))
    # Q^T b against the oracle (the part below n carries the residual)
    qerr = md_err(bg.cpu().numpy(), ref["qtb"])
    assert qerr <= TOL[P] * max(1, k)


@pytest.mark.parametrize("P,cfg", [(2, "512,2"), (4, "256,1"), (8, "256,2"), (8, "256,1")])
def test_multi_workgroup_panel(M, orc, monkeypatch, P, cfg):
    """Small workgroups spread a 700-row panel over several workgroups (grid barrier), with
    and without the concurrent side-stream update."""
    monkeypatch.setenv("MDLS_PANEL_CFG", cfg)
    if True:
        m, n, tile = 700, 64, 16
        print("case multi-wg P=%d cfg=%s" % (P, cfg), flush=True)
        A, xt = mdgen.ls_problem(P, m, n, 55)
        b = orc.rhs_for(A, xt)
        ref = orc.lstsq(A, b)
        outs = []
        for la in ("1", "0"):
            monkeypatch.setenv("MDLS_LOOKAHEAD", la)
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
    M.qr(P, Ag, tile, T=T)
    Bg = to_gpu(B)
    M.apply_qt(P, Ag, T, Bg, tile)
    W = torch.zeros((P, n, m), dtype=torch.float64, device=dev())
    M.form_w(P, Ag, T, tile, W)
    torch.cuda.synchronize()
    k = kappa(A)
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


@pytest.mark.parametrize("P,m,n,tile", [(2, 1024, 1024, 128), (2, 2048, 1024, 128), (4, 1024, 1024, 128),
                                        (4, 2048, 1024, 128), (8, 1024, 1024, 128), (8, 2048, 1024, 128)])
def test_full_size_recovers_x_true(M, orc, P, m, n, tile):
    """The n = 1024 headline sizes: b = A x_true formed exactly by the oracle and rounded to P
    limbs, so the computed x must match x_true to the kappa-scaled tolerance."""
    print("case full P=%d m=%d n=%d" % (P, m, n), flush=True)
    A, xt = mdgen.ls_problem(P, m, n, 2000 + P)
    b = orc.rhs_for(A, xt)
    x, info = M.solve(P, to_gpu(A), to_gpu(b), tile)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    k = kappa(A)
    err = md_err(x.cpu().numpy(), xt)
    report("full", err, TOL[P] * max(1, k))
    assert err <= TOL[P] * max(1.0, k)


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
