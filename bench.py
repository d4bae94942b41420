#!/usr/bin/env python3
"""Benchmark of the multiple-double least-squares hot path on one MI355X.

One step solves the square n = 1024 least-squares problem (tile 128) once in double double,
once in quad double and once in octo double: blocked Householder QR with Q^T b folded in,
then the tiled back substitution (paper Algorithms 2 and 1, Section 4 Table 11 workload).
Inputs are seeded synthetic matrices generated directly in device memory; every step
restores the pristine A and b (device-to-device copies of 16 + 32 + 64 MiB) before solving.

``value`` is the paper's throughput measure: the algorithmic double-operation count of the
three solves (Table 1 weights, see paper_2110_08375_amd/opcount.py) divided by the wall time
of the step, in TFLOP/s; the step is captured once as a HIP graph and replayed (``--no-graph``
times eager launches), the per-precision times come from events around eager solves.  The JSON line also carries, per precision, the solve time and its
fraction of the FP64 peak; a roofline entry for the kernel that takes the most device time
(per-kernel HIP-event timing inside the library, on the solve's stream); and the CPU oracle
timed on a bounded sample of the same workload; and the batched form (512 uneven dd and qd
problems in one persistent launch: solves/s, p50/p99 per-problem latency) against the plain
solver called once per problem; and the precision form (n = 2048, kappa = 1e8: double-double
factorisation refined with qd/od residuals) against the plain qd/od solver.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "double-op TFLOP/s QR+backsub n=1024 dd/qd/od vs FP64 peak; batched solves/s"
PNAME = {1: "d", 2: "dd", 4: "qd", 8: "od"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_problem(P, m, n, seed, device):
    import mdgen

    A = mdgen.md_uniform(P, m, n, seed, mdgen.STREAM_A, device=device).contiguous()
    b = mdgen.md_vector(P, m, seed, mdgen.STREAM_B, device=device).contiguous()
    return A, b


def sources_digest():
    """sha256 over the kernel sources (csrc and the C header): ties counter summaries to a build."""
    import glob
    import hashlib

    csrc = os.path.join(ROOT, "paper_2110_08375_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hpp")) + glob.glob(os.path.join(csrc, "*.hip")) +
                   glob.glob(os.path.join(csrc, "*.cpp")) + [os.path.join(ROOT, "include", "mdls.h")])
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE summary, if it was
    taken on the current kernel sources; else None."""
    import glob

    digest = sources_digest()
    for f in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(f) as fh:
            d = json.load(fh)
        if d.get("kernel") == kernel and d.get("sources_sha256") == digest:
            return d["hbm_bytes_per_launch"], os.path.relpath(f, ROOT)
    return None, None


def measured_fp64():
    """Hardware FP64 instruction counts (per solve and per launch) from the committed
    SQ_INSTS_VALU_*_F64 summary, if it was taken on the current kernel sources; else None."""
    f = os.path.join(ROOT, "profiles", "fp64_insts_ls_n1024.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    return d if d.get("sources_sha256") == sources_digest() else None


def hw_flops_per_launch(hw, kernel):
    """Hardware FP64 flops per launch of `kernel` from measured_fp64()'s summary, or None."""
    pl = hw["per_launch"].get(kernel) if kernel else None
    return None if pl is None else pl["hw_flops"]


def hw_flops_per_solve(hw, prec_name):
    """Hardware FP64 flops of one solve in precision `prec_name` ("dd", "qd", "od"), or None."""
    ps = hw["per_solve"].get(prec_name)
    return None if ps is None else ps["hw_flops"]


def cpu_baseline(sample, threads):
    """The CPU oracle (unchanged) on a bounded sample of square least-squares solves with the
    benchmark's input recipe; Table-1 double ops per second, blended and per precision."""
    import mdgen
    import oracle
    from paper_2110_08375_amd import opcount

    total_ops, total_s = 0.0, 0.0
    per = {}
    for P, n in sample:
        A, _ = mdgen.ls_problem(P, n, n, 3)
        b = mdgen.md_vector(P, n, 3, mdgen.STREAM_B)
        t0 = time.perf_counter()
        oracle.lstsq(A, b, nthreads=threads)
        dt = time.perf_counter() - t0
        ops = opcount.ls_double_ops(P, n, n)
        total_s += dt
        total_ops += ops
        per[PNAME[P]] = {"n": n, "s": round(dt, 3), "tflops": ops / dt / 1e12}
        log("cpu oracle %s n=%d, %d thread(s): %.2f s" % (PNAME[P], n, threads, dt))
    return total_ops / total_s / 1e12, total_s, per


def batched_run(M, P, count, seed, dev, reps, per_problem):
    """The batched workload: count problems, m uniform in [32, 512], n uniform in [16, m], entries as
    the n = 1024 problem; one persistent launch (autotuned variant) against the plain solver called
    once per problem."""
    import numpy as np
    import torch

    import mdgen
    from paper_2110_08375_amd import opcount

    shapes = mdgen.batch_shapes(count, seed)
    descs, a_len, b_len, x_len = M.batch_descs(P, shapes)
    A = np.empty(a_len)
    b = np.empty(b_len)
    for k, (m, n) in enumerate(shapes):
        A[descs[k].a_off:descs[k].a_off + P * m * n] = mdgen.md_uniform(P, m, n, seed + k, mdgen.STREAM_A).ravel()
        b[descs[k].b_off:descs[k].b_off + P * m] = mdgen.md_vector(P, m, seed + k, mdgen.STREAM_B).ravel()
    A0 = torch.from_numpy(A).to(dev)
    b0 = torch.from_numpy(b).to(dev)
    Aw, bw = torch.empty_like(A0), torch.empty_like(b0)
    x = torch.zeros(x_len, dtype=torch.float64, device=dev)
    info = torch.zeros(count, dtype=torch.int32, device=dev)
    times = torch.zeros(2 * count, dtype=torch.int64, device=dev)
    ws = M.batch_workspace(P, count, dev)
    M.batch_plan(P, descs, ws)
    best, tune_ms = M.batch_autotune(P, count, A0, b0, Aw, bw, x, ws, info)
    ms = []
    for _ in range(reps):
        Aw.copy_(A0)
        bw.copy_(b0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        M.solve_batched(P, count, Aw, bw, x, best, ws, info, times)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    if int((info != 0).sum().item()) != 0:
        raise RuntimeError("batched solve reported a zero pivot")
    t = times.cpu().numpy().reshape(-1, 2)
    lat = (t[:, 1] - t[:, 0]) / M.wall_clock_khz()  # ms
    ops = sum(opcount.ls_double_ops(P, m, n) for m, n in shapes)
    ms_b = float(np.median(ms))
    out = {"variant": best, "autotune_ms": [round(v, 3) for v in tune_ms], "ms": round(ms_b, 3),
           "solves_per_s": round(count / (ms_b * 1e-3), 1), "tflops": round(ops / (ms_b * 1e-3) / 1e12, 4),
           "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
           "max_ms": round(float(lat.max()), 4)}
    log("batched %s: variant %d, %.3f ms for %d problems (%.1f solves/s), p50 %.3f ms p99 %.3f ms"
        % (PNAME[P], best, ms_b, count, out["solves_per_s"], out["p50_ms"], out["p99_ms"]))
    if per_problem:
        # the plain solver, one call (several launches) per problem, tile = largest divisor of n <= 128
        xs = [torch.empty((P, n), dtype=torch.float64, device=dev) for _, n in shapes]
        wss = {}
        Aw.copy_(A0)
        bw.copy_(b0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, (m, n) in enumerate(shapes):
            tile = max(t for t in range(1, min(n, 128) + 1) if n % t == 0)
            Ak = Aw[descs[k].a_off:descs[k].a_off + P * m * n].view(P, n, m)
            bk = bw[descs[k].b_off:descs[k].b_off + P * m].view(P, m)
            key = (m, n, tile)
            if key not in wss:
                wss[key] = M.workspace(P, m, n, tile, dev)
            M.solve(P, Ak, bk, tile, x=xs[k], ws=wss[key], info=info[k:k + 1])
        torch.cuda.synchronize()
        ms_p = (time.perf_counter() - t0) * 1e3
        out["per_problem_launches"] = {"ms": round(ms_p, 3), "solves_per_s": round(count / (ms_p * 1e-3), 1)}
        out["speedup_vs_per_problem"] = round(ms_p / ms_b, 2)
        log("per-problem launches %s: %.3f ms (%.1f solves/s)" % (PNAME[P], ms_p, count / (ms_p * 1e-3)))
    return out


def fwd_err(x, xt):
    """max |x - x_true| / max |x_true| of md vectors (limb axis first), the limb differences
    summed from the bottom (an error estimate, not md arithmetic)"""
    import numpy as np

    d = np.zeros(xt.shape[1])
    for k in range(xt.shape[0] - 1, -1, -1):
        d = d + (x[k] - xt[k])
    return float(np.max(np.abs(d)) / np.max(np.abs(xt[0])))


def precision_run(M, dev, n=2048, tile=128):
    """The precision form: m = n = 2048, kappa = 1e8 (U diag(s) V^T), factor in dd and refine with
    qd / od residuals until the correction norms show convergence, against the plain solver at
    the target precision; b = A x_true exact by construction (mdgen.conditioned_exact), so the
    forward error against x_true is reported for every result."""
    import torch

    import mdgen

    out = {"workload": "least squares m=n=%d, tile %d, kappa 1e8 (U diag(s) V^T, 8 reflectors each, entries on a "
                       "2^-50 grid), b = A x_true exact; factor in dd, refine with qd/od residuals until the "
                       "correction norms converge, vs the plain solver at qd/od; forward error vs x_true" % (n, tile)}
    for P, iters in ((4, 8), (8, 10)):
        A, xt, b = mdgen.conditioned_exact(P, n, n, 77, kappa=1e8)
        Ag = torch.from_numpy(A[:2].copy()).to(dev)
        bg = torch.from_numpy(b).to(dev)
        ws = M.refined_workspace(P, n, n, tile, dev)
        F = torch.empty_like(Ag)
        ms = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            x, info, norms = M.solve_refined(P, Ag, bg, tile, iters, F=F, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        steps = int((norms.cpu().numpy().reshape(-1, 2)[:, 0] >= 0).sum())
        err_r = fwd_err(x.cpu().numpy(), xt)
        Ap = torch.from_numpy(A).to(dev)
        bp = bg.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        xp, infop = M.solve(P, Ap, bp, tile)
        e1.record()
        torch.cuda.synchronize()
        mp = e0.elapsed_time(e1)
        err_p = fwd_err(xp.cpu().numpy(), xt)
        if int(info.item()) != 0 or int(infop.item()) != 0:
            raise RuntimeError("precision form: info %d / %d" % (int(info.item()), int(infop.item())))
        out[PNAME[P]] = {"refined_ms": round(ms[-1], 3), "steps": steps, "max_steps": iters,
                         "refined_fwd_err": err_r, "plain_ms": round(mp, 3), "plain_fwd_err": err_p,
                         "speedup": round(mp / ms[-1], 2)}
        log("precision form %s: refined %.2f ms (%d steps, err %.2e), plain %.2f ms (err %.2e)"
            % (PNAME[P], ms[-1], steps, err_r, mp, err_p))
        del Ap, bp, F, ws, Ag, bg
    return out


def split_run(M, dev):
    """The precision form's split-limb product on the FP64 matrix cores against the same
    double-double product Y^T C on the vector units, at the trailing-update shapes of the first
    panel of the n = 1024 and n = 2048 double-double factorisations (w = 16 Householder vectors);
    kernel times from the in-library HIP-event timing."""
    import torch

    import mdgen

    out = {"workload": "double-double S = Y^T C at trailing-update shapes (h rows, w = 16, c columns): "
                       "k_split_tn (exact slicing, v_mfma_f64_16x16x4f64) vs k_dense_tn2 (vector units)"}
    for (h, c) in ((1024, 1008), (2048, 2032)):
        Y = torch.from_numpy(mdgen.md_uniform(2, h, 16, 5100 + h, mdgen.STREAM_A)).to(dev)
        C = torch.from_numpy(mdgen.md_uniform(2, h, c, 5100 + h, mdgen.STREAM_B)).to(dev)
        res = {}
        for method, kname in ((0, "k_dense_tn2"), (1, "k_split_tn")):
            S = M.dd_gemm_tn(method, Y, C)
            torch.cuda.synchronize()
            M.timing_reset()
            M.timing_enable(True)
            for _ in range(5):
                M.dd_gemm_tn(method, Y, C, S=S)
            torch.cuda.synchronize()
            M.timing_enable(False)
            ms, cnt, work = M.timing_query(kname, 2)
            res[kname + "_us"] = round(1e3 * ms / max(cnt, 1), 2)
            if method == 1:
                # 28 slice products of 16 x 16 x 4 per 16 x 16 tile and 4-row step: FP64 matrix flops
                mf = 2.0 * 28 * 16 * 16 * 4 * ((c + 15) // 16) * ((h + 3) // 4)
                res["k_split_tn_mfma_tflops"] = round(mf / (1e-3 * ms / max(cnt, 1)) / 1e12, 3)
        out["h%d_c%d" % (h, c)] = res
        log("split product h=%d c=%d: %s" % (h, c, res))
    return out


def scale_run(M, dev, tile=128):
    """The other plain-method workloads: the tall 2048 x 1024 least squares in dd/qd/od, and the
    back substitution at scale (upper-triangular qd, n = 17 920, tile 256, off-diagonals uniform
    in [-1, 1), diagonal uniform in [1, 2]: the paper's timing input), device-resident and with
    R, b in and x out over PCIe from pinned host memory (the paper's wall clock)."""
    import torch

    import mdgen
    from paper_2110_08375_amd import opcount

    def ev_time(fn, reset, reps=2):
        out = []
        for _ in range(reps + 1):
            reset()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return min(out[1:])

    res = {"tall": {"workload": "least squares m=2048, n=1024, tile 128"}}
    m, n = 2048, 1024
    for P in (2, 4, 8):
        A0, b0 = make_problem(P, m, n, 7100 + P, dev)
        A, b = torch.empty_like(A0), torch.empty_like(b0)
        x = torch.empty((P, n), dtype=torch.float64, device=dev)
        ws = M.workspace(P, m, n, tile, dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)

        def reset():
            A.copy_(A0)
            b.copy_(b0)

        ms = ev_time(lambda: M.solve(P, A, b, tile, x=x, ws=ws, info=info), reset)
        tf = opcount.ls_double_ops(P, m, n) / (ms * 1e-3) / 1e12
        res["tall"][PNAME[P]] = {"ms": round(ms, 3), "tflops": round(tf, 4)}
        log("tall %s: %.3f ms, %.3f TFLOP/s" % (PNAME[P], ms, tf))
        del A0, b0, A, b, x, ws

    P, n, tile_bs = 4, 17920, 256
    R = mdgen.upper_triangular(P, n, 21, device=dev).contiguous()
    y0 = mdgen.md_vector(P, n, 21, mdgen.STREAM_B, device=dev).contiguous()
    x = torch.empty_like(y0)
    ws = M.workspace(P, n, n, tile_bs, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    ms = ev_time(lambda: M.backsub(P, R, x, tile_bs, ws=ws, info=info), lambda: x.copy_(y0))
    ops = opcount.backsub_double_ops(P, n)
    rec = {"workload": "back substitution, upper-triangular qd, n=17920, tile 256", "ms": round(ms, 3),
           "tflops": round(ops / (ms * 1e-3) / 1e12, 4), "paper_v100_kernel_ms": 237.1,
           "paper_v100_wall_ms": 2150.0}
    Rh = torch.empty(R.shape, dtype=torch.float64, pin_memory=True)
    yh = torch.empty(y0.shape, dtype=torch.float64, pin_memory=True)
    xh = torch.empty(y0.shape, dtype=torch.float64, pin_memory=True)
    Rh.copy_(R)
    yh.copy_(y0)
    torch.cuda.synchronize()
    walls = []
    for _ in range(2):
        t0 = time.perf_counter()
        R.copy_(Rh, non_blocking=True)
        x.copy_(yh, non_blocking=True)
        M.backsub(P, R, x, tile_bs, ws=ws, info=info)
        xh.copy_(x, non_blocking=True)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    w = min(walls)
    rec["wall_ms_incl_pcie"] = round(w * 1e3, 3)
    rec["wall_tflops_incl_pcie"] = round(ops / w / 1e12, 4)
    if int(info.item()) != 0:
        raise RuntimeError("back substitution reported info=%d" % int(info.item()))
    log("backsub qd n=17920: %.3f ms resident, %.1f ms with transfers" % (ms, w * 1e3))
    res["backsub_at_scale"] = rec
    del R, Rh, ws
    torch.cuda.empty_cache()
    return res


# Paper, Table 5 (V100, complex double double QR of a 512 x 512 matrix): kernel time in ms
# for the tiles 16 x 32, 8 x 64, 4 x 128 and 2 x 256
PAPER_TABLE5_COMPLEX_KERNEL_MS = {32: 97.4, 64: 227.4, 128: 238.5, 256: 420.8}


def complex_run(M, dev, n=512):
    """The paper's complex workload (Table 5): QR of a complex 512 x 512 matrix in double double
    for the four tile sizes, plus the complex least-squares solve at tile 128 and the qd/od QR
    at tile 128; each timed as the median of 3 eager calls on resident inputs."""
    import torch

    import mdgen
    from paper_2110_08375_amd import opcount

    def timed(fn, reset, reps=3):
        ms = []
        for _ in range(reps + 1):
            reset()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return sorted(ms[1:])[len(ms[1:]) // 2]

    out = {"workload": "complex QR (and least squares) of a square %d x %d matrix, entries with uniform "
                       "real and imaginary parts as the n = 1024 problem" % (n, n),
           "unit": "ms",
           "flops": "Table-1 double operations of the complex QR = 4 x the real QR count"}
    for P, tiles in ((2, (32, 64, 128, 256)), (4, (128,)), (8, (128,))):
        A0 = mdgen.cmd_uniform(P, n, n, 5000 + P, mdgen.STREAM_A, device=dev).contiguous()
        b0 = mdgen.cmd_vector(P, n, 5000 + P, mdgen.STREAM_B, device=dev).contiguous()
        A, b = A0.clone(), b0.clone()
        rec = {}
        for tile in tiles:
            ws = M.cworkspace(P, n, n, tile, dev)
            T = torch.zeros((2, P, n, tile), dtype=torch.float64, device=dev)
            ms = timed(lambda: M.cqr(P, A, tile, T=T, ws=ws), lambda: A.copy_(A0))
            r = {"qr_ms": round(ms, 3),
                 "qr_tflops": round(opcount.cqr_double_ops(P, n, n) / (ms * 1e-3) / 1e12, 4)}
            if P == 2:
                r["paper_v100_kernel_ms"] = PAPER_TABLE5_COMPLEX_KERNEL_MS[tile]
            if tile == 128:
                x = torch.empty((2, P, n), dtype=torch.float64, device=dev)
                info = torch.zeros(1, dtype=torch.int32, device=dev)

                def reset():
                    A.copy_(A0)
                    b.copy_(b0)

                r["solve_ms"] = round(timed(lambda: M.csolve(P, A, b, tile, x=x, ws=ws, info=info), reset), 3)
            rec["tile%d" % tile] = r
            log("complex %s n=%d tile %d: QR %.3f ms" % (PNAME[P], n, tile, ms))
        out[PNAME[P]] = rec
        del A0, b0, A, b
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=1024)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--tile", type=int, default=128)
    ap.add_argument("--precisions", default="2,4,8", help="limb counts, e.g. 2,4,8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-solves measurement")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of a captured graph")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--no-precision", action="store_true", help="skip the refined (precision-form) measurement")
    ap.add_argument("--no-complex", action="store_true", help="skip the complex (Table 5) measurement")
    ap.add_argument("--no-scale", action="store_true",
                    help="skip the tall 2048 x 1024 solves and the n = 17920 back substitution")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2110_08375_amd as M
    from paper_2110_08375_amd import opcount

    M.lib()
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    M.init()  # the look-ahead side stream of this thread
    m, n, tile = args.m, args.n, args.tile
    precs = [int(p) for p in args.precisions.split(",")]
    log("device %s, m=%d n=%d tile=%d precisions=%s" % (torch.cuda.get_device_name(0), m, n, tile, precs))

    prob = {}
    for P in precs:
        A0, b0 = make_problem(P, m, n, 7000 + P, dev)
        prob[P] = dict(A0=A0, b0=b0, A=torch.empty_like(A0), b=torch.empty_like(b0),
                       x=torch.empty((P, n), dtype=torch.float64, device=dev),
                       ws=M.workspace(P, m, n, tile, dev),
                       info=torch.zeros(1, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()

    def step(events=None):
        for P in precs:
            d = prob[P]
            d["A"].copy_(d["A0"])
            d["b"].copy_(d["b0"])
            if events is not None:
                events[P][0].record()
            M.solve(P, d["A"], d["b"], tile, x=d["x"], ws=d["ws"], info=d["info"])
            if events is not None:
                events[P][1].record()

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup step %d done" % (w + 1))
    for P in precs:
        if int(prob[P]["info"].item()) != 0:
            raise RuntimeError("solve reported info=%d for %s" % (int(prob[P]["info"].item()), PNAME[P]))

    # per-precision solve times (eager launches, events around each solve)
    per_ms = {P: 0.0 for P in precs}
    for s in range(args.steps):
        ev = {P: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for P in precs}
        step(ev)
        torch.cuda.synchronize()
        for P in precs:
            per_ms[P] += ev[P][0].elapsed_time(ev[P][1])
    graph = None
    if not args.no_graph:
        # the whole step (input restores and the three solves) captured once and replayed
        graph = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            step()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cs):
            step()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
        torch.cuda.synchronize()
        log("timed step %d done" % (s + 1))
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    for P in precs:
        if int(prob[P]["info"].item()) != 0:
            raise RuntimeError("solve reported info=%d for %s" % (int(prob[P]["info"].item()), PNAME[P]))
    ops_step = sum(opcount.ls_double_ops(P, m, n) for P in precs)
    value = ops_step / (ms_per_step * 1e-3) / 1e12
    peak = opcount.FP64_PEAK_TFLOPS

    per_prec = {}
    for P in precs:
        ms = per_ms[P] / args.steps
        tf = opcount.ls_double_ops(P, m, n) / (ms * 1e-3) / 1e12
        per_prec[PNAME[P]] = {"ms": round(ms, 4), "tflops": round(tf, 4), "frac_fp64_peak": round(tf / peak, 5),
                              "solves_per_s": round(1e3 / ms, 3)}
        log("%s: %.3f ms per solve, %.3f TFLOP/s" % (PNAME[P], ms, tf))

    roof = None
    if not args.no_kernel_timing:
        M.timing_reset()
        M.timing_enable(True)
        step()
        torch.cuda.synchronize()
        M.timing_enable(False)
        best = None
        kernels = {}
        executed = {P: 0.0 for P in precs}
        for name in M.timing_kernels():
            for P in precs:
                ms, cnt, work = M.timing_query(name, P)
                if cnt == 0:
                    continue
                executed[P] += work
                kernels["%s<%s>" % (name, PNAME[P])] = {"ms": round(ms, 4), "launches": cnt,
                                                        "avg_us": round(ms * 1e3 / cnt, 3)}
                if best is None or ms > best[1]:
                    best = (name, ms, cnt, work, P)
        # the trailing-update kernels with the most device time (throughput-bound, for context)
        thr = None
        for name in ("k_apply_s", "k_apply_u"):
            for P in precs:
                ms_, cnt_, work_ = M.timing_query(name, P)
                if cnt_ and (thr is None or ms_ > thr[1]):
                    thr = (name, ms_, cnt_, work_, P)
        M.timing_reset()
        name, ms, cnt, work, P = best
        label = "%s<%s>" % (name, PNAME[P])
        achieved = work * opcount.md_fma_double_ops(P) / (ms * 1e-3) / 1e12
        traffic, tsrc = measured_traffic(label)
        roof = {"bound": "alu", "kernel": label, "achieved": round(achieved, 4),
                "peak": round(peak, 2), "unit": "TFLOP/s", "frac": round(achieved / peak, 5), "traffic": traffic,
                "traffic_unit": "bytes per launch", "traffic_source": tsrc,
                "launches": cnt, "avg_launch_us": round(ms * 1e3 / cnt, 3),
                "per_kernel": kernels}
        if thr is not None:
            tn, tms, tcnt, twork, tP = thr
            tach = twork * opcount.md_fma_double_ops(tP) / (tms * 1e-3) / 1e12
            roof["throughput_kernel"] = {"kernel": "%s<%s>" % (tn, PNAME[tP]), "achieved": round(tach, 4),
                                         "frac": round(tach / peak, 5), "avg_launch_us": round(tms * 1e3 / tcnt, 3)}
        # the hardware view: FP64 VALU instructions counted by rocprofv3 (FMA = 2 flops), the
        # convention of the peak; Table-1 operations above can exceed it
        hw = measured_fp64()
        if hw is not None:
            for lab, key in ((label, None), (roof.get("throughput_kernel", {}).get("kernel"), "throughput_kernel")):
                fl = hw_flops_per_launch(hw, lab)
                if fl is None:
                    continue
                tgt = roof if key is None else roof[key]
                us = tgt["avg_launch_us"]
                tgt["hw_achieved"] = round(fl / (us * 1e-6) / 1e12, 4)
                tgt["hw_frac"] = round(tgt["hw_achieved"] / peak, 5)
            roof["hw_source"] = "profiles/fp64_insts_ls_n1024.json"
        log("dominant kernel %s: %.3f ms over %d launches, %.3f TFLOP/s" % (label, ms, cnt, achieved))

    if not args.no_kernel_timing:
        # executed work: the md multiply-adds every launch of one step recorded (the compact-WY
        # factors, tile inversions and look-ahead updates included), weighted like the
        # algorithmic count
        for P in precs:
            ex = opcount.md_fma_double_ops(P) * executed[P] + 3.0 * n * opcount.weights(P)[2]
            per_prec[PNAME[P]]["executed_double_ops"] = round(ex, 1)
            per_prec[PNAME[P]]["executed_tflops"] = round(ex / (per_prec[PNAME[P]]["ms"] * 1e-3) / 1e12, 4)

    hw = measured_fp64()
    if hw is not None:
        for P in precs:
            fl = hw_flops_per_solve(hw, PNAME[P])
            if fl is not None:
                t = fl / (per_prec[PNAME[P]]["ms"] * 1e-3) / 1e12
                per_prec[PNAME[P]]["hardware_tflops"] = round(t, 4)
                per_prec[PNAME[P]]["hardware_frac"] = round(t / peak, 5)

    # PCIe-inclusive wall time (the paper's wall clock, Section 4: host buffers in and out):
    # A and b copied from pinned host memory, the solve, x copied back; not the headline
    for P in precs:
        d = prob[P]
        Ah = torch.empty(d["A0"].shape, dtype=torch.float64, pin_memory=True)
        bh = torch.empty(d["b0"].shape, dtype=torch.float64, pin_memory=True)
        xh = torch.empty(d["x"].shape, dtype=torch.float64, pin_memory=True)
        Ah.copy_(d["A0"])
        bh.copy_(d["b0"])
        torch.cuda.synchronize()
        walls = []
        for _ in range(2):
            t0 = time.perf_counter()
            d["A"].copy_(Ah, non_blocking=True)
            d["b"].copy_(bh, non_blocking=True)
            M.solve(P, d["A"], d["b"], tile, x=d["x"], ws=d["ws"], info=d["info"])
            xh.copy_(d["x"], non_blocking=True)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        w = min(walls)
        per_prec[PNAME[P]]["wall_ms_incl_pcie"] = round(w * 1e3, 4)
        per_prec[PNAME[P]]["wall_tflops_incl_pcie"] = round(opcount.ls_double_ops(P, m, n) / w / 1e12, 4)
        log("%s: %.3f ms with host transfers" % (PNAME[P], w * 1e3))
        del Ah, bh, xh

    batched = None
    if not args.no_batched:
        batched = {"workload": "%d independent least-squares problems, m uniform in [32, 512], n uniform in "
                               "[16, m], entries as the n = 1024 problem, one persistent launch (autotuned "
                               "variant) vs the plain solver called per problem" % args.batch}
        for P in (2, 4):
            batched[PNAME[P]] = batched_run(M, P, args.batch, 4000 + P, dev, 3, True)

    precision = None if args.no_precision else precision_run(M, dev)
    if precision is not None:
        precision["split_product"] = split_run(M, dev)
    cplx = None if args.no_complex else complex_run(M, dev)
    scale = None if args.no_scale else scale_run(M, dev)

    cpu = None
    if not args.no_cpu_baseline:
        # all host cores the process may use (the box sets OMP_NUM_THREADS), and one thread
        threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
        sample = [(2, 1024), (4, 512), (8, 256)]
        v, secs, per = cpu_baseline(sample, threads)
        sample1 = [(2, 256), (4, 128), (8, 128)]
        v1, secs1, per1 = cpu_baseline(sample1, 1)
        cpu = {"value": v, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
               "sample": "oracle least squares (unblocked Householder QR + Q^T b + back substitution) on square "
                         "dd n=1024, qd n=512, od n=256 with the same input recipe, %d threads; %.1f s"
                         % (threads, secs),
               "nproc": os.cpu_count(), "per_precision": per,
               "single_thread": {"value": v1, "cores": 1, "per_precision": per1,
                                 "sample": "the same solve on square dd n=256, qd n=128, od n=128, one "
                                           "thread; %.1f s" % secs1}}

    out = {
        "metric": METRIC,
        "value": round(value, 5),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "least squares, square m=n=%d, tile %d, one solve each in %s" %
                                (n, tile, "/".join(PNAME[P] for P in precs)),
                   "m": m, "n": n, "tile": tile, "precisions": [PNAME[P] for P in precs],
                   "launch": "graph replay" if graph is not None else "eager"},
        "per_precision": per_prec,
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched": batched,
        "precision_form": precision,
        "complex": cplx,
        "scale": scale,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
