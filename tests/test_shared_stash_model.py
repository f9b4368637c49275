"""Host model of the block-shared stash (tests/helpers/shared_stash_model.cpp).

The wavefronts of a block, as host threads, share one pool of work links
through the lock-free transactions of the GPU kernel: claimed mask bits,
tagged compare-and-swap reservations on the partial link of each event,
written-slot counts that publish full links, closing of partial links by
drained wavefronts, spills to and refills from the global arena, and the
block's exit rule.  Every particle must finish exactly once, the pools and
the arena must end empty; a too small arena must fail fast.  Each case also
runs in a ThreadSanitizer build, which must report no data race.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "helpers", "shared_stash_model.cpp")


@pytest.fixture(scope="module", params=["plain", "tsan"])
def model(request, tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    extra = ["-fsanitize=thread"] if request.param == "tsan" else []
    exe = str(tmp_path_factory.mktemp("shared") / f"shared_stash_{request.param}")
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", *extra, SRC, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        if extra:
            pytest.skip(f"host compiler cannot build {extra}")
        raise AssertionError(r.stderr)
    return exe


def _run(exe, *args):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=300, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.returncode in (0, 1), (r.returncode, r.stdout, r.stderr[-2000:])
    return r.returncode, dict(kv.split("=") for kv in r.stdout.split())


@pytest.mark.parametrize("blocks,wpb,links,particles,force", [
    (2, 4, 8, 20000, 0),      # default-sized pool: events + wavefronts + 2
    (2, 4, 8, 20000, 1),      # every full link through the arena
    (4, 4, 7, 30000, 2),
    (1, 8, 12, 20000, 0),
    (3, 2, 5, 20000, 3),
    (2, 4, 4, 20000, 0),      # a pool smaller than the wavefronts: spills keep it going
    (3, 2, 3, 20000, 0),      # one link more than the events
    (8, 4, 8, 50000, 1),
])
def test_every_particle_once(model, blocks, wpb, links, particles, force):
    rc, out = _run(model, blocks, wpb, links, particles, force)
    assert rc == 0, out
    assert out["missing"] == "0" and out["twice"] == "0" and out["err"] == "0"
    assert out["leftover"] == "0" and out["fill"] == "0" and out["spills"] == out["refills"]
    if force:
        assert int(out["spills"]) > 0


def test_exhausted_arena_fails_fast(model):
    rc, out = _run(model, 4, 4, 5, 20000, 1, 40)
    assert rc == 1 and out["failed"] == "1" and out["twice"] == "0"
    assert float(out["ms"]) < 2000.0
