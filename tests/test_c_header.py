"""include/mdls.h is usable from C: a C11 program includes it, links against libmdls.so and
calls the host-side entry points (workspace sizing, argument validation, status text); no GPU
is needed for these."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "mdls.h"

int main(void)
{
    size_t ws = mdls_workspace_bytes(MDLS_QD, 256, 128, 32);
    size_t cws = mdls_cworkspace_bytes(MDLS_DD, 256, 128, 32);
    if (ws == 0 || cws == 0) return 1;
    if (mdls_workspace_bytes(3, 256, 128, 32) != 0) return 2;
    /* invalid precision: -1, checked before anything touches a device */
    if (mdls_solve(3, 256, 128, 32, NULL, 256, NULL, NULL, NULL, ws, NULL, NULL) != -1) return 3;
    if (mdls_csolve(MDLS_DD, 256, 128, 33, NULL, 256, NULL, NULL, NULL, cws, NULL, NULL) != -4) return 4;
    if (strlen(mdls_status_string(MDLS_EHIP)) == 0) return 5;
    printf("ok %zu %zu\n", ws, cws);
    return 0;
}
"""


def test_header_compiles_links_and_runs_as_c(tmp_path):
    from paper_2110_08375_amd import build, mdls

    cc = shutil.which("gcc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("gcc or the ROCm headers are not available")
    if not os.path.exists(mdls._LIB_PATH):
        build.build_library()
    src = tmp_path / "use_mdls.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_mdls"
    libdir = os.path.dirname(mdls._LIB_PATH)
    subprocess.run([cc, "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L" + libdir, "-lmdls",
                    "-Wl,-rpath," + libdir], check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.startswith("ok ")
