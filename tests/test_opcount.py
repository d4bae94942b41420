"""Table 1 of the paper (operation counts of md arithmetic), transcribed into the metric,
checked against the fixture copied from the paper and against the paper's own derived
numbers (row sums, averages, predicted overhead factors)."""
import os

import pytest

from paper_2110_08375_amd import opcount

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_opcounts.txt")
PREC = {"dd": 2, "qd": 4, "od": 8}


def load():
    rows, avg, fac = {}, {}, {}
    for ln in open(GOLDEN):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        f = ln.split()
        if f[0] == "average":
            avg[f[1]] = float(f[2])
        elif f[0] == "factor":
            fac[f[1]] = float(f[2])
        else:
            rows[(f[0], f[1])] = [int(v) for v in f[2:]]
    return rows, avg, fac


def test_rows_sum_and_match_weights():
    rows, _, _ = load()
    for (p, op), (a, s, m, d, tot) in rows.items():
        assert a + s + m + d == tot
        idx = {"add": 0, "mul": 1, "div": 2}[op]
        assert opcount.TABLE1[PREC[p]][idx] == tot


def test_averages_and_predicted_factors():
    rows, avg, fac = load()
    for p in ("dd", "qd", "od"):
        assert abs(sum(opcount.TABLE1[PREC[p]]) / 3 - avg[p]) < 0.05
    assert abs(sum(opcount.TABLE1[4]) / sum(opcount.TABLE1[2]) - fac["dd_qd"]) < 0.05
    assert abs(sum(opcount.TABLE1[8]) / sum(opcount.TABLE1[4]) - fac["qd_od"]) < 0.05


def test_ls_count_and_peak():
    # square n: m n^2 - n^3/3 = 2/3 n^3 leading term
    n = 1024
    assert abs(opcount.ls_md_fmas(n, n) / (2 / 3 * n ** 3) - 1) < 0.01
    assert opcount.ls_double_ops(2, n, n) == pytest.approx(43 * opcount.ls_md_fmas(n, n) + 3 * n * 70)
    assert opcount.FP64_PEAK_TFLOPS == pytest.approx(78.6, rel=1e-3)
