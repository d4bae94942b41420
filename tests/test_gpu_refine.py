"""GPU parity of the refined least-squares form (double-double factorisation, refinement with
quad- or octo-double residuals) through the C ABI, on kappa = 1e8 matrices (U diag(s) V^T):
with consistent right-hand sides b = A x_true formed exactly by the oracle and rounded to the
target precision, x must match x_true to TOL[P] * kappa, like the plain solver at that
precision; with an inconsistent b (a residual orthogonal to range(A)), x must match the
oracle's least-squares solution of the stored data at the target precision, to
TOL[P] kappa (1 + kappa rho), rho = ||r|| / (||A|| ||x||) (the least-squares perturbation bound)."""
import numpy as np
import pytest

import mdgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {4: 1e-58, 8: 1e-118}


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def M():
    import paper_2110_08375_amd as M

    M.lib()
    torch.zeros(1, device=dev())
    M.init()
    return M


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def md_err(x, ref):
    d = np.zeros(ref.shape[1])
    for k in range(ref.shape[0] - 1, -1, -1):
        d = d + (x[k] - ref[k])
    return np.max(np.abs(d)) / max(np.max(np.abs(ref[0])), 1e-300)


def steps_taken(norms):
    nr = norms.cpu().numpy().reshape(-1, 2)
    taken = nr[:, 0] >= 0
    k = int(np.argmin(taken)) if not taken.all() else len(taken)
    assert taken[:k].all() and not taken[k:].any()  # steps not taken are marked -1 at the end
    return nr[:k]


@pytest.mark.parametrize("P,m,n,tile,iters", [(4, 256, 256, 64, 8), (8, 256, 256, 64, 10), (8, 300, 128, 32, 10)])
def test_refined_recovers_x_true(M, orc, P, m, n, tile, iters):
    """Consistent b: x_true to the target tolerance, and the refinement stops by itself on its
    correction norms before the step limit."""
    print("case refined P=%d m=%d n=%d" % (P, m, n), flush=True)
    A = mdgen.conditioned(2, m, n, 40 + n, kappa=1e8)
    xt = mdgen.md_vector(P, n, 41, mdgen.STREAM_X)
    b = orc.matvec(A, xt, P)
    x, info, norms = M.solve_refined(P, to_gpu(A), to_gpu(b), tile, iters)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    kap = float(np.linalg.cond(A[0].T))
    err = md_err(x.cpu().numpy(), xt)
    nr = steps_taken(norms)
    rel = nr[:, 0] / nr[:, 1]
    u = 2.0 ** -(53 * P - (P - 1))
    print("refined P=%d err %.3e (%.2f u kappa) kappa %.3e steps %d corrections %s"
          % (P, err, err / (u * kap), kap, len(nr), rel), flush=True)
    assert err <= TOL[P] * max(1.0, kap)
    assert err <= 64 * n * u * max(1.0, kap)  # the tight bound of the plain path's oracle tests
    assert 3 <= len(nr) < iters  # stopped on the norms, not on the limit
    assert rel[1] < 1e-12 * rel[0] and rel[2] < rel[1]  # the corrections shrink geometrically
    # the stopping rule: the last step's correction, or its contraction estimate, is below u
    assert rel[-1] <= u or rel[-1] * (nr[-1, 0] / nr[-2, 0]) <= u


@pytest.mark.parametrize("P,m,n,tile", [(4, 512, 256, 64), (8, 512, 256, 64)])
def test_refined_inconsistent_matches_oracle(M, orc, P, m, n, tile):
    """Tall kappa = 1e8 system with a nonzero residual: b = A x_true + t r, r orthogonal to
    range(A) (from the FP64 least-squares residual of a random vector), formed exactly by the
    oracle at the target precision.  The refined x against the oracle's least-squares solution of
    the same (A promoted to P limbs, b) data."""
    print("case refined inconsistent P=%d m=%d n=%d" % (P, m, n), flush=True)
    A = mdgen.conditioned(2, m, n, 90 + P, kappa=1e8)
    xt = mdgen.md_vector(P, n, 91, mdgen.STREAM_X)
    A64 = A[0].T + A[1].T
    g = mdgen.md_vector(1, m, 92, mdgen.STREAM_B)[0]
    r = g - A64 @ np.linalg.lstsq(A64, g, rcond=None)[0]
    t = 1e-6 / np.linalg.norm(r)
    rv = np.zeros((P, m))
    rv[0] = t * r
    b = -orc.matvec(A, xt, P, c=-rv)  # c - A x with c = -t r, negated (exact)
    Ap = np.zeros((P, n, m))
    Ap[:2] = A
    ref = orc.lstsq(Ap, b)
    x, info, norms = M.solve_refined(P, to_gpu(A), to_gpu(b), tile, 12)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    kap = float(np.linalg.cond(A64))
    xo = ref["x"]
    rho = np.linalg.norm(t * r) / (np.linalg.norm(A64, 2) * np.linalg.norm(xo[0]))
    err = md_err(x.cpu().numpy(), xo)
    nr = steps_taken(norms)
    bound = TOL[P] * kap * (1.0 + kap * rho)
    u = 2.0 ** -(53 * P - (P - 1))
    tight = 64 * n * u * kap * (1.0 + kap * rho)
    print("refined inconsistent P=%d err vs oracle %.3e bound %.3e (%.2f u kappa (1 + kappa rho)) kappa %.3e rho %.3e "
          "steps %d" % (P, err, bound, err / (u * kap * (1.0 + kap * rho)), kap, rho, len(nr)), flush=True)
    assert err <= bound
    assert err <= tight
    assert len(nr) < 12


@pytest.mark.parametrize("P,iters", [(4, 4), (8, 6)])
def test_refined_full_size_vs_plain(M, orc, P, iters):
    """The precision-form workload: n = 2048 (tile 128), kappa = 1e8, factor in dd, refine to qd
    or od; the plain solver at the target precision on the same data for comparison."""
    from paper_2110_08375_amd import opcount

    m = n = 2048
    tile = 128
    print("case refined full-size P=%d" % P, flush=True)
    A = mdgen.conditioned(2, m, n, 77, kappa=1e8)
    xt = mdgen.md_vector(P, n, 78, mdgen.STREAM_X)
    b = orc.matvec(A, xt, P)
    kap = float(np.linalg.cond(A[0].T))
    Ag, bg = to_gpu(A), to_gpu(b)
    ws = M.refined_workspace(P, m, n, tile, dev())
    F = torch.empty_like(Ag)
    ms = []
    for _ in range(2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        x, info, norms = M.solve_refined(P, Ag, bg, tile, iters, F=F, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    assert int(info.item()) == 0
    err = md_err(x.cpu().numpy(), xt)
    # the plain solver at the target precision on the same data (A promoted to P limbs)
    Ap = np.zeros((P, n, m))
    Ap[:2] = A
    Apg = to_gpu(Ap)
    bp = bg.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    xp, infop = M.solve(P, Apg, bp, tile)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    errp = md_err(xp.cpu().numpy(), xt)
    F_ops = opcount.ls_double_ops(P, m, n)
    print("full-size P=%d: refined %.2f ms err %.3e; plain %.2f ms err %.3e; kappa %.3e; speedup %.1f; "
          "plain-equivalent %.2f Table-1 TFLOP/s" % (P, ms[-1], err, ms_plain, errp, kap, ms_plain / ms[-1],
                                                    F_ops / (ms[-1] * 1e-3) / 1e12), flush=True)
    assert err <= TOL[P] * max(1.0, kap)
    assert errp <= TOL[P] * max(1.0, kap)


@pytest.mark.parametrize("P,m,n,tile", [(4, 640, 384, 64), (8, 1280, 256, 128)])
def test_refined_split_update_matches_oracle(M, orc, P, m, n, tile):
    """The option that forms the factorisation's trailing-update products Y^T C on the FP64 matrix
    cores (exact slicing): the refined solution still matches the oracle's least-squares solution
    of the stored data (nonzero residual, kappa = 1e8) to the same bound, the matrix-core kernel
    ran, and the product rows above 1024 (the second case's first panels) take the same path."""
    print("case refined split update P=%d m=%d n=%d" % (P, m, n), flush=True)
    A = mdgen.conditioned(2, m, n, 190 + P, kappa=1e8)
    xt = mdgen.md_vector(P, n, 191, mdgen.STREAM_X)
    A64 = A[0].T + A[1].T
    g = mdgen.md_vector(1, m, 192, mdgen.STREAM_B)[0]
    r = g - A64 @ np.linalg.lstsq(A64, g, rcond=None)[0]
    t = 1e-6 / np.linalg.norm(r)
    rv = np.zeros((P, m))
    rv[0] = t * r
    b = -orc.matvec(A, xt, P, c=-rv)
    Ap = np.zeros((P, n, m))
    Ap[:2] = A
    ref = orc.lstsq(Ap, b)
    M.set_tuning(M.MDLS_TUNE_SPLIT_UPDATE, 1)
    try:
        M.timing_reset()
        M.timing_enable(True)
        x, info, norms = M.solve_refined(P, to_gpu(A), to_gpu(b), tile, 12)
        torch.cuda.synchronize()
        M.timing_enable(False)
        ms, cnt, work = M.timing_query("k_split_tn", 0)
    finally:
        M.set_tuning(M.MDLS_TUNE_SPLIT_UPDATE, 0)
    assert int(info.item()) == 0
    assert cnt > 0, "the matrix-core product did not run"
    kap = float(np.linalg.cond(A64))
    rho = np.linalg.norm(t * r) / (np.linalg.norm(A64, 2) * np.linalg.norm(ref["x"][0]))
    err = md_err(x.cpu().numpy(), ref["x"])
    nr = steps_taken(norms)
    bound = TOL[P] * kap * (1.0 + kap * rho)
    print("refined split update P=%d err vs oracle %.3e bound %.3e steps %d k_split_tn launches %d"
          % (P, err, bound, len(nr), cnt), flush=True)
    assert err <= bound
    assert len(nr) < 12
