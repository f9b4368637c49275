"""Host model of the asynchronous scheduler's work-link protocol.

tests/helpers/arena_model.cpp replays, on host threads with std::atomic,
the stash / global-arena protocol of the asynchronous scheduler: spills of
ready links, refills, lock-free (head, tail) queues claimed by atomic
exchange, donation of sparse drained stashes and the last-wavefront exit
rule.  Every particle must finish exactly once and the arena must end empty,
with and without donation and with forced spills.  An arena too small for
the forced spills must fail fast: the first failed wait ends after its
wall-clock budget and publishes the failure, which ends every other wait at
once.  Each case also runs in a ThreadSanitizer build, which must report no
data race.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "helpers", "arena_model.cpp")


def _build(tmp_path_factory, name, extra):
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    exe = str(tmp_path_factory.mktemp("arena") / name)
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", *extra, SRC, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        if extra:
            pytest.skip(f"host compiler cannot build {extra}: {r.stderr[-300:]}")
        raise AssertionError(r.stderr)
    return exe


@pytest.fixture(scope="module", params=["plain", "tsan"])
def model(request, tmp_path_factory):
    extra = ["-fsanitize=thread"] if request.param == "tsan" else []
    return request.param, _build(tmp_path_factory, "arena_model_" + request.param, extra)


def _run(exe, *args):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=300, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.returncode in (0, 1), (r.returncode, r.stdout, r.stderr[-2000:])
    return r.returncode, dict(kv.split("=") for kv in r.stdout.split())


@pytest.mark.parametrize("workers,particles,links,force,consolidate,seed", [
    (8, 20000, 3, 0, 0, 1),
    (8, 20000, 3, 1, 0, 2),
    (16, 20000, 4, 2, 0, 3),
    (8, 20000, 3, 0, 1, 4),
    (8, 20000, 3, 1, 1, 5),
    (16, 30000, 2, 3, 1, 6),
])
def test_every_particle_once(model, workers, particles, links, force, consolidate, seed):
    _, exe = model
    rc, out = _run(exe, workers, particles, links, force, consolidate, seed)
    assert rc == 0, out
    assert out["missing"] == "0" and out["twice"] == "0" and out["err"] == "0"
    assert out["spills"] == out["refills"] and out["fill"] == "0"
    if force > 0:
        assert int(out["spills"]) > 0


@pytest.mark.parametrize("consolidate", [0, 1])
@pytest.mark.parametrize("arena", [1, 4, 16])
def test_exhausted_arena_fails_fast(model, consolidate, arena):
    # every filled link is spilled into an arena of a few links: the run must
    # report the failure (no particle finished twice) within about one wait
    # budget (20 ms), not after a long spin
    _, exe = model
    rc, out = _run(exe, 8, 20000, 3, 1, consolidate, 11 + arena, arena, 20)
    assert rc == 1 and out["failed"] == "1" and int(out["err"]) > 0
    assert out["twice"] == "0"
    assert float(out["ms"]) < 1000.0, out
