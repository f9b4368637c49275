"""The C-ABI library loads and exports every function include/mcx.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os

import pytest

from paper_2506_00263_amd import mcx


def test_library_exports_header_functions():
    if not os.path.exists(mcx.LIB_PATH):
        pytest.skip("libmcx.so not built")
    L = mcx.lib()
    names = mcx.header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    if not os.path.exists(mcx.LIB_PATH):
        pytest.skip("libmcx.so not built")
    L = mcx.lib()
    assert L.mcx_status_str(0) == b"ok"
    assert L.mcx_status_str(4) == b"scheduler capacity exhausted"
    assert L.mcx_last_error(None) == b"null handle"


def test_struct_sizes_match_header():
    # the ctypes mirrors must have the C layout: compare against the header's
    # field order by compiling a tiny probe with the host compiler
    import subprocess
    import tempfile
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "mcx.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mcx_problem_desc), sizeof(mcx_run_opts),
         sizeof(mcx_counters_t), sizeof(mcx_digest), offsetof(mcx_problem_desc, max_steps),
         offsetof(mcx_run_opts, time_kernels), offsetof(mcx_problem_desc, speed_coef), sizeof(mcx_eigen_opts),
         offsetof(mcx_counters_t, sites));
  return 0;
}
'''
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "p.c")
        open(c, "w").write(src)
        exe = os.path.join(td, "p")
        subprocess.check_call(["gcc", "-I", inc, c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    sizes = [int(v) for v in out]
    assert sizes[0] == ctypes.sizeof(mcx.ProblemDesc)
    assert sizes[1] == ctypes.sizeof(mcx.RunOpts)
    assert sizes[2] == ctypes.sizeof(mcx.Counters)
    assert sizes[3] == mcx.DIGEST_DTYPE.itemsize
    assert sizes[4] == mcx.ProblemDesc.max_steps.offset
    assert sizes[5] == mcx.RunOpts.time_kernels.offset
    assert sizes[6] == mcx.ProblemDesc.speed_coef.offset
    assert sizes[7] == ctypes.sizeof(mcx.EigenOpts)
    assert sizes[8] == mcx.Counters.sites.offset
