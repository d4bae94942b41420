"""bench.py's command-line contract on the host: more than one GPU is refused with a message
(the library measures one GPU), before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_counter_summaries_read_back():
    """The committed counter summaries parse the way bench.py reads them (hardware flops per
    launch and per solve, HBM bytes per launch of the dominant kernel), whatever their source hash."""
    import json

    sys.path.insert(0, ROOT)
    import bench

    with open(os.path.join(ROOT, "profiles", "fp64_insts_ls_n1024.json")) as fh:
        hw = json.load(fh)
    assert bench.hw_flops_per_launch(hw, "k_panel<od>") > 0
    assert bench.hw_flops_per_launch(hw, "k_apply_s<od>") > 0
    assert bench.hw_flops_per_launch(hw, "no such kernel") is None
    assert bench.hw_flops_per_launch(hw, None) is None
    for p in ("dd", "qd", "od"):
        assert bench.hw_flops_per_solve(hw, p) > 0
    with open(os.path.join(ROOT, "profiles", "traffic_k_panel_od_n1024.json")) as fh:
        tr = json.load(fh)
    assert tr["kernel"] == "k_panel<od>" and tr["hbm_bytes_per_launch"] > 0
    # when the summaries were taken on these sources, bench.py finds them
    if hw["sources_sha256"] == bench.sources_digest():
        assert bench.measured_fp64() is not None
        assert bench.measured_traffic("k_panel<od>")[0] == tr["hbm_bytes_per_launch"]
