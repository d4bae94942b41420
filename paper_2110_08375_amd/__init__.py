"""Multiple-double least squares on AMD MI355X (gfx950).

The compute path is the HIP library ``libmdls.so`` (built from ``csrc/`` by ``build.py``) behind
the C ABI of ``include/mdls.h``; :mod:`paper_2110_08375_amd.mdls` is a thin ctypes binding with
the same names that only marshals arguments.  PyTorch supplies device memory and streams.
"""
from .mdls import (  # noqa: F401
    MDLS_DD,
    MDLS_F64,
    MDLS_OD,
    MDLS_QD,
    BatchDesc,
    apply_q,
    apply_qt,
    backsub,
    batch_autotune,
    batch_descs,
    batch_plan,
    batch_variants,
    batch_workspace,
    capply_qh,
    cbacksub,
    cqr,
    csolve,
    cworkspace,
    cworkspace_bytes,
    form_q,
    form_w,
    lib,
    max_rows,
    qr,
    refined_workspace,
    solve,
    solve_refined,
    solve_batched,
    status_string,
    timing_enable,
    timing_kernels,
    timing_query,
    timing_reset,
    wall_clock_khz,
    workspace,
    workspace_bytes,
)
