"""The C ABI from a plain C program (no Python, no torch): compiled with gcc
as C against include/mcx.h and linked against libmcx.so.  On the CPU it must
compile and link; on the GPU its tally must equal the oracle's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "helpers", "c_client.c")
PKG = os.path.join(ROOT, "paper_2506_00263_amd")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(PKG, "libmcx.so")):
        pytest.skip("HIP library not built")
    exe = str(tmp_path_factory.mktemp("cclient") / "c_client")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), SRC, "-o", exe,
                    "-L", PKG, "-lmcx", f"-Wl,-rpath,{PKG}"], check=True)
    return exe


def test_c_client_builds(client):
    assert os.path.exists(client)


def _problem():
    # the same problem the C program describes
    return inputs.box_slabs_mg(size=(10.0, 10.0, 10.0), planes_x=[0.0, 4.0, 10.0], slab_mat=[0, 1],
                               sigma_t=[[1.0, 1.5], [0.6, 0.9]], sigma_s=[[0.7, 1.2], [0.3, 0.5]],
                               cdf=[[[0.6, 1.0], [0.0, 1.0]], [[0.5, 1.0], [0.0, 1.0]]],
                               mesh_n=(5, 5, 5), n_histories=50_000, seed=12345, problem_id=0)


@pytest.mark.gpu
def test_c_client_matches_oracle(client, oracle, tmp_path):
    out = str(tmp_path / "tally.bin")
    r = subprocess.run([client, out], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    got = np.fromfile(out, dtype=np.int64)
    ref = oracle.run(_problem())
    assert got.size == ref["tally"].size
    assert np.array_equal(got, ref["tally"])
