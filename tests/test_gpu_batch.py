"""GPU parity of the batched least-squares form (many uneven problems, one persistent launch)
against the CPU oracle, problem by problem, through the C ABI.

Tolerance as in test_gpu_parity: ||x - x_ref||_inf / ||x_ref||_inf <= TOL[P] * max(1, kappa_2(A)).
"""
import numpy as np
import pytest

import mdgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {2: 1e-28, 4: 1e-58}


def unit(P):
    """u_P = 2^-(53P - (P - 1)); beside TOL every x is also held to the tight bound 64 n u_P kappa"""
    return 2.0 ** -(53 * P - (P - 1))


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def M():
    import paper_2110_08375_amd as M

    M.lib()  # raises if the HIP library is missing: there is no fallback
    return M


def md_err(x, ref):
    d = np.zeros(ref.shape[1])
    for k in range(ref.shape[0] - 1, -1, -1):
        d = d + (x[k] - ref[k])
    return np.max(np.abs(d)) / max(np.max(np.abs(ref[0])), 1e-300)


def make_batch(M, P, shapes, seed, rhs):
    """Problems packed back to back; rhs(k, A) gives b for problem k (numpy, P x m)."""
    descs, a_len, b_len, x_len = M.batch_descs(P, shapes)
    A = np.zeros(a_len)
    b = np.zeros(b_len)
    mats = []
    for k, (m, n) in enumerate(shapes):
        Ak = mdgen.md_uniform(P, m, n, seed + k, mdgen.STREAM_A)
        bk = rhs(k, Ak)
        A[descs[k].a_off:descs[k].a_off + P * m * n] = Ak.ravel()
        b[descs[k].b_off:descs[k].b_off + P * m] = bk.ravel()
        mats.append((Ak, bk))
    return descs, A, b, x_len, mats


def x_of(M, descs, xg, P, k):
    d = descs[k]
    return xg[d.x_off:d.x_off + P * d.n].reshape(P, d.n)


def run_batch(M, P, descs, A, b, x_len, variant, ws, times=None):
    Ag = torch.from_numpy(A).to(dev())
    bg = torch.from_numpy(b).to(dev())
    xg = torch.zeros(x_len, dtype=torch.float64, device=dev())
    info = torch.full((len(descs),), -7, dtype=torch.int32, device=dev())
    M.solve_batched(P, len(descs), Ag, bg, xg, variant, ws, info, times)
    torch.cuda.synchronize()
    return xg.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("P", (2, 4))
def test_batched_matches_oracle(M, orc, P):
    shapes = mdgen.batch_shapes(13, 300 + P, m_lo=8, m_hi=96, n_lo=1) + [(1, 1), (7, 7), (96, 1), (64, 64)]
    print("case batched P=%d shapes=%s" % (P, shapes), flush=True)
    descs, A, b, x_len, mats = make_batch(M, P, shapes, 900, lambda k, Ak: mdgen.md_vector(P, Ak.shape[2], 77 + k, 3))
    refs = [orc.lstsq(Ak, bk)["x"] for Ak, bk in mats]
    kap = [float(np.linalg.cond(Ak[0].T)) for Ak, _ in mats]
    ws = M.batch_workspace(P, len(shapes), dev())
    M.batch_plan(P, descs, ws)
    outs = []
    for v in range(M.batch_variants(P)):
        xg, info = run_batch(M, P, descs, A, b, x_len, v, ws)
        assert np.all(info == 0), (v, info)
        for k in range(len(shapes)):
            err = md_err(x_of(M, descs, xg, P, k), refs[k])
            assert err <= TOL[P] * max(1.0, kap[k]), (v, k, shapes[k], err)
            assert err <= 64 * shapes[k][1] * unit(P) * max(1.0, kap[k]), (v, k, shapes[k], err)
        outs.append(xg)
    xg, _ = run_batch(M, P, descs, A, b, x_len, 0, ws)
    assert np.array_equal(xg, outs[0])  # run to run, bit for bit


def test_batched_zero_column_sets_info(M):
    P = 2
    shapes = [(40, 12), (30, 30), (50, 5)]

    def rhs(k, Ak):
        return mdgen.md_vector(P, Ak.shape[2], 5 + k, 3)

    descs, A, b, x_len, mats = make_batch(M, P, shapes, 70, rhs)
    d = descs[0]
    Ak = A[d.a_off:d.a_off + P * 40 * 12].reshape(P, 12, 40)
    Ak[:, 4, :] = 0.0  # zero column 4 of problem 0: R(4,4) is exactly zero
    ws = M.batch_workspace(P, len(shapes), dev())
    M.batch_plan(P, descs, ws)
    _, info = run_batch(M, P, descs, A, b, x_len, 0, ws)
    assert list(info) == [5, 0, 0]


@pytest.mark.parametrize("P", (2, 4))
def test_batched_nan_problem_is_isolated(M, P):
    """A NaN in one problem's A: that problem's x holds NaN with info 0 (NaN is not an exact
    zero), every kernel exits, and every other problem's x equals the clean batch's bit for bit
    in each kernel variant (teams share no values across problems)."""
    shapes = [(40, 12), (64, 32), (30, 30), (96, 17), (50, 5), (8, 8)]

    def rhs(k, Ak):
        return mdgen.md_vector(P, Ak.shape[2], 11 + k, 3)

    descs, A, b, x_len, _ = make_batch(M, P, shapes, 120 + P, rhs)
    An = A.copy()
    d = descs[1]
    An[d.a_off + 3 * 64 + 5] = np.nan  # problem 1, leading limb, column 3, row 5
    ws = M.batch_workspace(P, len(shapes), dev())
    M.batch_plan(P, descs, ws)
    for v in range(M.batch_variants(P)):
        print("case batched nan P=%d variant %d" % (P, v), flush=True)
        xc, ic = run_batch(M, P, descs, A, b, x_len, v, ws)
        xn, inn = run_batch(M, P, descs, An, b, x_len, v, ws)
        assert np.all(ic == 0) and np.all(inn == 0), (v, ic, inn)
        assert np.isfinite(xc).all()
        for k in range(len(shapes)):
            xk = x_of(M, descs, xn, P, k)
            if k == 1:
                assert np.isnan(xk).any(), v
            else:
                assert np.array_equal(xk, x_of(M, descs, xc, P, k)), (v, k)


@pytest.mark.parametrize("P", (2, 4))
def test_batched_full_size_recovers_ones(M, orc, P):
    """512 problems, m uniform in [32, 512], n uniform in [16, m] (the batched workload), b = A ones
    formed exactly by the oracle: every x must be ones within TOL * kappa; the autotuner's choice
    is used, and per-problem device timestamps are ordered."""
    shapes = mdgen.batch_shapes(512, 4000 + P)
    print("case batched full-size P=%d" % P, flush=True)
    descs, A, b, x_len, mats = make_batch(M, P, shapes, 6000, lambda k, Ak: orc.rhs_for(Ak, mdgen.md_ones(P, Ak.shape[1])))
    ws = M.batch_workspace(P, len(shapes), dev())
    M.batch_plan(P, descs, ws)
    A0 = torch.from_numpy(A).to(dev())
    b0 = torch.from_numpy(b).to(dev())
    Aw, bw = torch.empty_like(A0), torch.empty_like(b0)
    xg = torch.zeros(x_len, dtype=torch.float64, device=dev())
    info = torch.zeros(len(shapes), dtype=torch.int32, device=dev())
    best, ms = M.batch_autotune(P, len(shapes), A0, b0, Aw, bw, xg, ws, info)
    print("autotune P=%d variant %d ms %s" % (P, best, ms), flush=True)
    assert 0 <= best < M.batch_variants(P) and all(t > 0 for t in ms)
    times = torch.zeros(2 * len(shapes), dtype=torch.int64, device=dev())
    Aw.copy_(A0)
    bw.copy_(b0)
    M.solve_batched(P, len(shapes), Aw, bw, xg, best, ws, info, times)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    xh = xg.cpu().numpy()
    ones = None
    worst = 0.0
    for k, (m, n) in enumerate(shapes):
        ones = mdgen.md_ones(P, n)
        kap = float(np.linalg.cond(mats[k][0][0].T))
        err = md_err(x_of(M, descs, xh, P, k), ones)
        worst = max(worst, err / max(1.0, kap))
        assert err <= TOL[P] * max(1.0, kap), (k, m, n, err, kap)
        assert err <= 64 * n * unit(P) * max(1.0, kap), (k, m, n, err, kap)
    t = times.cpu().numpy().reshape(-1, 2)
    assert np.all(t[:, 1] > t[:, 0])
    print("batched P=%d: worst err/kappa %.3e (%.2f u), %.1f solves/s" % (P, worst, worst / unit(P), 512 / (min(ms) * 1e-3)),
          flush=True)


def test_batched_graph_replay(M):
    """The batched solve (counter reset + one persistent kernel) captured in a graph and replayed
    three times, with eager restores of A and b between replays: every replay equals the eager
    solve bit for bit."""
    P = 2
    shapes = mdgen.batch_shapes(40, 17, m_lo=16, m_hi=160, n_lo=4)
    descs, A, b, x_len, _ = make_batch(M, P, shapes, 400, lambda k, Ak: mdgen.md_vector(P, Ak.shape[2], 9 + k, 3))
    ws = M.batch_workspace(P, len(shapes), dev())
    M.batch_plan(P, descs, ws)
    A0 = torch.from_numpy(A).to(dev())
    b0 = torch.from_numpy(b).to(dev())
    Aw, bw = A0.clone(), b0.clone()
    xg = torch.zeros(x_len, dtype=torch.float64, device=dev())
    info = torch.zeros(len(shapes), dtype=torch.int32, device=dev())
    M.solve_batched(P, len(shapes), Aw, bw, xg, 0, ws, info)
    torch.cuda.synchronize()
    ref = xg.cpu().numpy().copy()
    Aw.copy_(A0)
    bw.copy_(b0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            M.solve_batched(P, len(shapes), Aw, bw, xg, 0, ws, info)
    torch.cuda.synchronize()
    for rep in range(3):
        Aw.copy_(A0)
        bw.copy_(b0)
        xg.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(xg.cpu().numpy(), ref), rep
        assert np.all(info.cpu().numpy() == 0)
