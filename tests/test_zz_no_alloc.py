"""GPU: mcx_run_noalloc, the entry point that allocates nothing (its scheduler
state and tally replicas live in the library's fixed device array), called
through the C ABI and compared with mcx_run bit for bit, on two calls in a
row with the second on a smaller input."""
import ctypes as C

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

COUNTS = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
          "cutoffs", "killed", "pieces", "qsum", "overflow", "cdf_scans"]


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


def _noalloc(mcx, P, **kw):
    o = mcx.run_opts(**kw)
    st = mcx.lib().mcx_run_noalloc(P.h, C.byref(o))
    assert st == 0, (st, mcx.lib().mcx_last_error(P.h))
    return P.tallies(), P.counters()


def _run(mcx, P, **kw):
    o = mcx.run_opts(**kw)
    st = mcx.lib().mcx_run(P.h, C.byref(o))
    assert st == 0, (st, mcx.lib().mcx_last_error(P.h))
    return P.tallies(), P.counters()


def _same(a, b):
    ta, ca = a
    tb, cb = b
    assert np.array_equal(ta, tb)
    for k in COUNTS:
        assert ca[k] == cb[k], (k, ca[k], cb[k])


# The stack scheme's banks scale with its capacity and resident wavefronts
# (by default far beyond the fixed array): it runs there with both set.
STACK_FIT = {"stack_capacity": 262_144, "stack_threshold": 4096, "waves_per_cu": 1}
CASES = [("naive", "fused", {}), ("async", "fused", {}), ("async", "split", {}), ("stack", "fused", STACK_FIT)]


@pytest.mark.parametrize("sched,decomp,knobs", CASES)
def test_noalloc_equals_run_lattice(mcx, sched, decomp, knobs):
    d = inputs.cfg2_lattice(30_000)
    P = mcx.Problem(d)
    # first call: all histories; second: a smaller range
    for kw in ({}, {"first": 1000, "n": 9000}):
        got = _noalloc(mcx, P, sched=sched, decomp=decomp, **knobs, **kw)
        ref = _run(mcx, P, sched=sched, decomp=decomp, **kw)
        _same(got, ref)
        assert got[1]["sourced"] == (30_000 if not kw else 9000)


def test_noalloc_replicas_and_lds_paths(mcx):
    # an energy tally in 16 replicas (behind the scheduler state in the fixed
    # array), then a smaller problem whose tally is summed in LDS
    for d, path in ((inputs.pincell_ce(n_ebins=10_000, n_histories=4000), "replicas"),
                    (inputs.pincell_ce(n_ebins=100, n_histories=1500), "auto")):
        P = mcx.Problem(d)
        for sched, decomp, knobs in (("async", "fused", {}), ("async", "split", {}), ("stack", "fused", STACK_FIT),
                                     ("naive", "fused", {})):
            got = _noalloc(mcx, P, sched=sched, decomp=decomp, tally_path=path, lookup="hash", **knobs)
            ref = _run(mcx, P, sched=sched, decomp=decomp, tally_path=path, lookup="hash")
            _same(got, ref)


def test_noalloc_batch(mcx):
    probs = inputs.cfg5_batch(n_problems=12, hist_scale=0.05)
    B = mcx.Problem(probs)
    for sched, knobs in (("async", {}), ("stack", STACK_FIT)):
        _noalloc(mcx, B, sched=sched, **knobs)
        got = [B.tallies(k) for k in range(len(probs))]
        _run(mcx, B, sched=sched)
        ref = [B.tallies(k) for k in range(len(probs))]
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), sched


def test_noalloc_refuses_what_does_not_fit(mcx):
    d = inputs.cfg2_lattice(300_000)
    P = mcx.Problem(d)
    need = P.workspace_size(sched="stack")
    assert need > (128 << 20)            # MCX_NOALLOC_SCRATCH_BYTES
    o = mcx.run_opts(sched="stack")
    assert mcx.lib().mcx_run_noalloc(P.h, C.byref(o)) == 1
    assert b"device scratch" in mcx.lib().mcx_last_error(P.h)
    with pytest.raises(mcx.McxError):
        P.tallies()                          # nothing ran
    # with its capacity and wavefronts set it fits, and gives the same integers
    got = _noalloc(mcx, P, sched="stack", **STACK_FIT)
    ref = _run(mcx, P, sched="stack")
    _same(got, ref)
    # async at 1e6 histories fits (its link arena does not grow with N)
    Q = mcx.Problem(inputs.cfg2_lattice(1_000_000))
    assert Q.workspace_size(sched="async", decomp="split") < (128 << 20)
    # options the entry point does not take
    o = mcx.run_opts(sched="async", n=1000, time_kernels=True)
    assert mcx.lib().mcx_run_noalloc(P.h, C.byref(o)) == 1
