"""Host model of the asynchronous scheduler's work-link protocol.

tests/helpers/arena_model.cpp replays, on host threads with std::atomic,
the stash / global-arena protocol of the asynchronous scheduler: spills of
ready links, refills, lock-free (head, tail) queues claimed by atomic
exchange, donation of sparse drained stashes and the last-wavefront exit
rule.  Every particle must finish exactly once and the arena must end empty,
with and without donation and with forced spills.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "helpers", "arena_model.cpp")


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    exe = str(tmp_path_factory.mktemp("arena") / "arena_model")
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", SRC, "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("workers,particles,links,force,consolidate,seed", [
    (8, 20000, 3, 0, 0, 1),
    (8, 20000, 3, 1, 0, 2),
    (16, 20000, 4, 2, 0, 3),
    (8, 20000, 3, 0, 1, 4),
    (8, 20000, 3, 1, 1, 5),
    (16, 30000, 2, 3, 1, 6),
])
def test_every_particle_once(model, workers, particles, links, force, consolidate, seed):
    r = subprocess.run([model, str(workers), str(particles), str(links), str(force), str(consolidate), str(seed)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    out = dict(kv.split("=") for kv in r.stdout.split())
    assert out["missing"] == "0" and out["twice"] == "0" and out["err"] == "0"
    assert out["spills"] == out["refills"] and out["fill"] == "0"
    if force > 0:
        assert int(out["spills"]) > 0
