"""The C ABI library loads and exports every entry point include/mdls.h declares, and
rejects invalid arguments on the host before anything is enqueued (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2110_08375_amd import build, mdls

    if not os.path.exists(mdls._LIB_PATH):
        build.build_library()
    return mdls.lib()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "mdls.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mdls_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    from paper_2110_08375_amd import mdls

    assert sorted(mdls.EXPORTS) == names


def test_workspace_and_limits(L):
    assert L.mdls_workspace_bytes(2, 1024, 1024, 128) > 0
    assert L.mdls_workspace_bytes(3, 1024, 1024, 128) == 0  # P not in {1,2,4,8}
    assert L.mdls_workspace_bytes(2, 10, 20, 4) == 0  # m < n
    assert L.mdls_workspace_bytes(2, 10, 10, 0) == 0
    for p in (1, 2, 4, 8):
        assert L.mdls_max_rows(p) >= 2048
    assert L.mdls_max_rows(5) == 0


def test_solve_argument_errors(L):
    vp = ctypes.c_void_p
    dummy = vp(16)  # never dereferenced: validation fails first
    ws = L.mdls_workspace_bytes(2, 64, 32, 16)
    s = L.mdls_solve
    assert s(3, 64, 32, 16, dummy, 64, dummy, dummy, dummy, ws, dummy, None) == -1
    assert s(2, 0, 32, 16, dummy, 64, dummy, dummy, dummy, ws, dummy, None) == -2
    assert s(2, 16, 32, 16, dummy, 64, dummy, dummy, dummy, ws, dummy, None) == -3
    assert s(2, 64, 32, 12, dummy, 64, dummy, dummy, dummy, ws, dummy, None) == -4  # n % tile
    assert s(2, 64, 32, 16, None, 64, dummy, dummy, dummy, ws, dummy, None) == -5
    assert s(2, 64, 32, 16, dummy, 63, dummy, dummy, dummy, ws, dummy, None) == -6
    assert s(2, 64, 32, 16, dummy, 64, None, dummy, dummy, ws, dummy, None) == -7
    assert s(2, 64, 32, 16, dummy, 64, dummy, None, dummy, ws, dummy, None) == -8
    assert s(2, 64, 32, 16, dummy, 64, dummy, dummy, None, ws, dummy, None) == -9
    assert s(2, 64, 32, 16, dummy, 64, dummy, dummy, dummy, ws - 1, dummy, None) == -10
    assert s(2, 64, 32, 16, dummy, 64, dummy, dummy, dummy, ws, None, None) == -11
    big = L.mdls_max_rows(2) + 1
    wsb = L.mdls_workspace_bytes(2, big, 32, 16)
    assert s(2, big, 32, 16, dummy, big, dummy, dummy, dummy, wsb, dummy, None) == -101


def test_noalloc_argument_errors(L):
    """mdls_solve_noalloc checks its arguments and its scratch limit on the host, before it looks
    up its static scratch or enqueues anything."""
    from paper_2110_08375_amd import mdls

    d = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    s = L.mdls_solve_noalloc
    assert s(3, 64, 32, 16, d, 64, d, d, d, None) == -1
    assert s(2, 64, 32, 12, d, 64, d, d, d, None) == -4
    assert s(2, 64, 32, 16, d, 63, d, d, d, None) == -6
    assert s(2, 64, 32, 16, d, 64, d, d, None, None) == -9
    # the largest workload that fits, and one that does not
    assert L.mdls_workspace_bytes(8, 2048, 2048, 128) <= mdls.MDLS_NOALLOC_SCRATCH_BYTES
    assert L.mdls_workspace_bytes(8, 4096, 2048, 256) > mdls.MDLS_NOALLOC_SCRATCH_BYTES
    assert s(8, 4096, 2048, 256, d, 4096, d, d, d, None) == mdls.MDLS_ESCRATCH
    assert "static scratch" in mdls.status_string(mdls.MDLS_ESCRATCH)


def test_other_entry_point_errors(L):
    vp = ctypes.c_void_p
    d = vp(16)
    ws = L.mdls_workspace_bytes(4, 64, 32, 16)
    assert L.mdls_qr(4, 64, 32, 12, d, 64, None, d, 12, d, ws, None, None) == -4  # T wants n % tile == 0
    assert L.mdls_qr(4, 64, 32, 16, d, 64, None, d, 8, d, ws, None, None) == -9  # ldt < tile
    assert L.mdls_qr(4, 64, 32, 16, d, 64, None, d, 16, None, ws, None, None) == -10
    assert L.mdls_qr(4, 64, 32, 16, d, 64, None, d, 16, d, ws - 1, None, None) == -11
    assert L.mdls_backsub(4, 30, 16, d, 30, d, d, ws, d, None) == -3
    assert L.mdls_backsub(4, 32, 16, d, 31, d, d, ws, d, None) == -5
    assert L.mdls_backsub(4, 32, 16, d, 32, d, d, ws, None, None) == -9
    assert L.mdls_apply_qt(4, 64, 32, 16, d, 64, None, 16, d, 64, 1, d, ws, None) == -7
    assert L.mdls_apply_qt(4, 64, 32, 16, d, 64, d, 16, d, 64, -1, d, ws, None) == -11
    assert L.mdls_form_w(4, 64, 32, 16, d, 64, d, 16, d, 63, None) == -10
    assert L.mdls_status_string(0) == b"success"
    assert b"invalid" in L.mdls_status_string(-3)


def test_tuning_options(L):
    """Tuning is explicit (no environment variables): defaults, range checks, round trip."""
    from paper_2110_08375_amd import mdls

    assert L.mdls_get_tuning(mdls.MDLS_TUNE_LOOKAHEAD) == 1
    assert L.mdls_get_tuning(mdls.MDLS_TUNE_PANEL_VARIANT) == 0
    assert L.mdls_get_tuning(mdls.MDLS_TUNE_SPIN_LIMIT) == 1 << 22
    assert L.mdls_get_tuning(mdls.MDLS_TUNE_CPANEL) == 2
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_CPANEL, 3) == -2
    assert L.mdls_get_tuning(99) == -1
    assert L.mdls_set_tuning(99, 0) == -1
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_PANEL_VARIANT, 2) == -2
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_SPIN_LIMIT, -1) == -2
    rows0 = L.mdls_max_rows(2)
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_PANEL_VARIANT, 1) == 0
    assert L.mdls_max_rows(2) == 4 * rows0  # 512 x 8 instead of 512 x 2 threads x rows
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_PANEL_VARIANT, 0) == 0
    assert L.mdls_max_rows(2) == rows0
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_SPIN_LIMIT, 7) == 0
    assert L.mdls_get_tuning(mdls.MDLS_TUNE_SPIN_LIMIT) == 7
    assert L.mdls_set_tuning(mdls.MDLS_TUNE_SPIN_LIMIT, 1 << 22) == 0


def test_no_environment_reads():
    """The library source reads no environment variable."""
    import glob

    for f in glob.glob(os.path.join(ROOT, "paper_2110_08375_amd", "csrc", "*")):
        assert "getenv" not in open(f).read(), f


def test_binding_refuses_cpu_tensors(L):
    torch = pytest.importorskip("torch")
    import paper_2110_08375_amd as M

    A = torch.zeros((2, 4, 8), dtype=torch.float64)
    b = torch.zeros((2, 8), dtype=torch.float64)
    with pytest.raises(ValueError):
        M.solve(2, A, b, 4)


def test_batched_entry_point_errors(L):
    from paper_2110_08375_amd import mdls

    vp = ctypes.c_void_p
    d = vp(16)
    assert L.mdls_batch_variants(2) >= 1 and L.mdls_batch_variants(4) >= 1
    assert L.mdls_batch_variants(8) == 0 and L.mdls_batch_variants(3) == 0
    assert L.mdls_batch_workspace_bytes(2, 512) > 0
    assert L.mdls_batch_workspace_bytes(8, 512) == 0 and L.mdls_batch_workspace_bytes(2, 0) == 0
    ws = L.mdls_batch_workspace_bytes(2, 3)
    good, _, _, _ = mdls.batch_descs(2, [(40, 20), (512, 512), (16, 1)])
    for bad in ([(10, 20), (40, 20), (16, 1)], [(513, 20), (40, 20), (16, 1)], [(40, 0), (40, 20), (16, 1)]):
        descs, _, _, _ = mdls.batch_descs(2, bad)
        assert L.mdls_batch_plan(2, 3, descs, d, ws, None) == -3
    assert L.mdls_batch_plan(8, 3, good, d, ws, None) == -1
    assert L.mdls_batch_plan(2, 0, good, d, ws, None) == -2
    assert L.mdls_batch_plan(2, 3, None, d, ws, None) == -3
    assert L.mdls_batch_plan(2, 3, good, None, ws, None) == -4
    assert L.mdls_batch_plan(2, 3, good, d, ws - 1, None) == -5
    sb = L.mdls_solve_batched
    assert sb(2, 3, d, d, d, L.mdls_batch_variants(2), d, ws, d, None, None) == -6
    assert sb(2, 3, d, d, d, -1, d, ws, d, None, None) == -6
    assert sb(2, 3, None, d, d, 0, d, ws, d, None, None) == -3
    assert sb(2, 3, d, d, d, 0, d, ws, None, None, None) == -9
    assert sb(4, 3, d, d, d, 0, d, L.mdls_batch_workspace_bytes(4, 3) - 1, d, None, None) == -8


def test_refined_entry_point_errors(L):
    d = ctypes.c_void_p(16)
    assert L.mdls_refined_workspace_bytes(8, 256, 256, 64) > L.mdls_workspace_bytes(2, 256, 256, 64)
    assert L.mdls_refined_workspace_bytes(2, 256, 256, 64) == 0
    ws = L.mdls_refined_workspace_bytes(8, 64, 32, 16)
    f = L.mdls_solve_refined
    assert f(2, 64, 32, 16, d, 64, d, d, 4, d, d, ws, d, d, None) == -1
    assert f(8, 64, 30, 16, d, 64, d, d, 4, d, d, ws, d, d, None) == -4
    assert f(8, 64, 32, 16, d, 63, d, d, 4, d, d, ws, d, d, None) == -6
    assert f(4, 64, 32, 16, d, 64, d, d, 0, d, d, ws, d, d, None) == -9
    assert f(8, 64, 32, 16, d, 64, d, d, 4, None, d, ws, d, d, None) == -10
    assert f(8, 64, 32, 16, d, 64, d, d, 4, d, d, ws - 1, d, d, None) == -12
    assert f(8, 64, 32, 16, d, 64, d, d, 4, d, d, ws, d, None, None) == -14


def test_explicit_q_entry_point_errors(L):
    d = ctypes.c_void_p(16)
    ws = L.mdls_workspace_bytes(4, 64, 32, 16)
    assert L.mdls_apply_q(4, 64, 32, 12, d, 64, d, 16, d, 64, 1, d, ws, None) == -4
    assert L.mdls_apply_q(4, 64, 32, 16, d, 64, None, 16, d, 64, 1, d, ws, None) == -7
    assert L.mdls_apply_q(4, 64, 32, 16, d, 64, d, 16, d, 64, -1, d, ws, None) == -11
    assert L.mdls_form_q(4, 64, 32, 16, d, 64, d, 16, None, 64, 64, d, ws, None) == -9
    assert L.mdls_form_q(4, 64, 32, 16, d, 64, d, 16, d, 63, 64, d, ws, None) == -10
    assert L.mdls_form_q(4, 64, 32, 16, d, 64, d, 16, d, 64, 65, d, ws, None) == -11
    assert L.mdls_form_q(4, 64, 32, 16, d, 64, d, 16, d, 64, 64, d, ws - 1, None) == -13


def test_complex_entry_point_errors(L):
    d = ctypes.c_void_p(16)
    ws = L.mdls_cworkspace_bytes(2, 64, 32, 16)
    assert ws > 0
    assert L.mdls_cworkspace_bytes(3, 64, 32, 16) == 0
    assert L.mdls_cworkspace_bytes(2, 16, 32, 16) == 0
    # the complex workspace holds twice the planes of the real one's blocks
    assert ws >= 2 * 8 * 2 * 16 * 32
    s = L.mdls_csolve
    assert s(5, 64, 32, 16, d, 64, d, d, d, ws, d, None) == -1
    assert s(2, 0, 32, 16, d, 64, d, d, d, ws, d, None) == -2
    assert s(2, 64, 65, 16, d, 64, d, d, d, ws, d, None) == -3
    assert s(2, 64, 32, 12, d, 64, d, d, d, ws, d, None) == -4
    assert s(2, 64, 32, 16, None, 64, d, d, d, ws, d, None) == -5
    assert s(2, 64, 32, 16, d, 63, d, d, d, ws, d, None) == -6
    assert s(2, 64, 32, 16, d, 64, None, d, d, ws, d, None) == -7
    assert s(2, 64, 32, 16, d, 64, d, None, d, ws, d, None) == -8
    assert s(2, 64, 32, 16, d, 64, d, d, None, ws, d, None) == -9
    assert s(2, 64, 32, 16, d, 64, d, d, d, ws - 1, d, None) == -10
    assert s(2, 64, 32, 16, d, 64, d, d, d, ws, None, None) == -11
    q = L.mdls_cqr
    assert q(2, 64, 32, 12, d, 64, None, 0, d, ws, None) == -4
    assert q(2, 64, 32, 16, d, 64, d, 15, d, ws, None) == -8
    assert q(2, 64, 32, 16, d, 64, None, 0, d, ws - 1, None) == -10
    a = L.mdls_capply_qh
    assert a(2, 64, 32, 16, d, 64, None, 16, d, 64, 1, d, ws, None) == -7
    assert a(2, 64, 32, 16, d, 64, d, 16, d, 63, 1, d, ws, None) == -10
    assert a(2, 64, 32, 16, d, 64, d, 16, d, 64, -1, d, ws, None) == -11
    assert a(2, 64, 32, 16, d, 64, d, 16, d, 64, 0, d, ws, None) == 0  # nothing to do
    wsb = L.mdls_cworkspace_bytes(4, 32, 32, 16)
    b = L.mdls_cbacksub
    assert b(4, 32, 12, d, 32, d, d, wsb, d, None) == -3
    assert b(4, 32, 16, d, 31, d, d, wsb, d, None) == -5
    assert b(4, 32, 16, d, 32, d, d, wsb - 1, d, None) == -8
    assert b(4, 32, 16, d, 32, d, d, wsb, None, None) == -9


def test_complex_binding_refuses_bad_tensors(L):
    import torch

    from paper_2110_08375_amd import mdls

    A = torch.zeros((2, 2, 16, 32), dtype=torch.float64)
    b = torch.zeros((2, 2, 32), dtype=torch.float64)
    with pytest.raises(ValueError):
        mdls.csolve(2, A, b, 16)  # CPU tensors
    with pytest.raises(ValueError):
        mdls.cqr(2, torch.zeros((2, 16, 32), dtype=torch.float64), 16)  # real layout


def test_backsub_binding_requires_n_columns(L):
    import torch

    from paper_2110_08375_amd import mdls

    R = torch.zeros((2, 64, 64), dtype=torch.float64)
    x = torch.zeros((2, 32), dtype=torch.float64)
    with pytest.raises(ValueError, match="exactly n columns"):
        mdls.backsub(2, R, x, 16, n=32)  # planes would be misread: refused before any call


def test_complex_explicit_q_entry_point_errors(L):
    d = ctypes.c_void_p(16)
    ws = L.mdls_cworkspace_bytes(2, 64, 32, 16)
    assert L.mdls_capply_q(2, 64, 32, 12, d, 64, d, 16, d, 64, 1, d, ws, None) == -4
    assert L.mdls_capply_q(2, 64, 32, 16, d, 64, None, 16, d, 64, 1, d, ws, None) == -7
    assert L.mdls_capply_q(2, 64, 32, 16, d, 64, d, 16, d, 64, 1, d, ws - 1, None) == -13
    assert L.mdls_cform_q(2, 64, 32, 16, d, 64, d, 16, None, 64, 64, d, ws, None) == -9
    assert L.mdls_cform_q(2, 64, 32, 16, d, 64, d, 16, d, 63, 64, d, ws, None) == -10
    assert L.mdls_cform_q(2, 64, 32, 16, d, 64, d, 16, d, 64, 65, d, ws, None) == -11
