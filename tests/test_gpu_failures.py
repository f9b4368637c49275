"""GPU: failure paths end every kernel normally and report through the ABI.

* stack capacity exhausted (a tiny stack capacity under a large make_work
  threshold): MCX_E_CAPACITY, then MCX_E_STATE on reading the tallies, then
  a normal run on the same handle matches the oracle;
* async link arena exhausted (a few arena links, every filled link sent
  through the arena): MCX_E_CAPACITY within well under a second (the first
  failed wait publishes the failure and every other wait ends), then a
  normal run matches the oracle;
* a history range past the problem's histories (including one whose end
  wraps around 2^64) and meshes or energy edges that do not contain the
  geometry are refused before anything runs.
"""
import ctypes as C
import time

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

E_INVALID_ARG, E_CAPACITY, E_STATE = 1, 4, 6


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


@pytest.fixture(scope="module")
def lattice(oracle):
    d = inputs.cfg2_lattice(20_000)
    return d, oracle.run(d)


def _status(mcx, P, fn, **kw):
    o = mcx.run_opts(**kw)
    return getattr(mcx.lib(), fn)(P.h, C.byref(o))


def _tally_status(mcx, P, n):
    out = np.zeros(n, np.int64)
    return mcx.lib().mcx_tallies(P.h, 0, out.ctypes.data_as(C.c_void_p), n, 0)


@pytest.mark.parametrize("decomp", ["fused", "split"])
def test_stack_capacity_exhausted(mcx, lattice, decomp):
    d, ref = lattice
    P = mcx.Problem(d)
    t0 = time.perf_counter()
    st = _status(mcx, P, "mcx_run", sched="stack", decomp=decomp, stack_capacity=64, stack_threshold=1 << 20)
    assert st == E_CAPACITY, (st, mcx.lib().mcx_last_error(P.h))
    assert time.perf_counter() - t0 < 5.0
    assert _tally_status(mcx, P, inputs.n_bins(d)) == E_STATE
    P.run(sched="stack", decomp=decomp)
    assert np.array_equal(P.tallies(), ref["tally"])


@pytest.fixture(scope="module")
def lattice_1e6(oracle):
    d = inputs.cfg2_lattice(1_000_000)
    return d, oracle.run(d)


@pytest.mark.parametrize("decomp", ["fused", "split"])
@pytest.mark.parametrize("arena", [1, 8])
def test_async_arena_exhausted(mcx, lattice_1e6, decomp, arena):
    # with 1e6 histories every wavefront still holds source ids when the few
    # arena links are full, so none refills: every spill's wait ends on its
    # budget or on the published failure
    d, ref = lattice_1e6
    P = mcx.Problem(d)
    t0 = time.perf_counter()
    st = _status(mcx, P, "mcx_run", sched="async", decomp=decomp, arena_links=arena, force_spill=1)
    dt = time.perf_counter() - t0
    assert st == E_CAPACITY, (st, mcx.lib().mcx_last_error(P.h))
    assert dt < 1.0, dt
    assert _tally_status(mcx, P, inputs.n_bins(d)) == E_STATE
    # the same handle runs normally afterwards (forcing every link through
    # the default arena is itself too much at this size for split events:
    # all wavefronts keep sourcing until every particle has been spilled)
    P.run(sched="async", decomp=decomp)
    assert np.array_equal(P.tallies(), ref["tally"])


def test_history_range_refused(mcx, lattice):
    d, _ = lattice
    P = mcx.Problem(d)
    n = d["n_histories"]
    for first, count in ((0, n + 1), (n, 1), (5, 2 ** 64 - 1), (n + 1, 0)):
        assert _status(mcx, P, "mcx_run", sched="async", first=first, n=count) == E_INVALID_ARG, (first, count)
        ws = C.c_size_t(0)
        o = mcx.run_opts(sched="stack", first=first, n=count)
        assert mcx.lib().mcx_workspace_size(P.h, C.byref(o), C.byref(ws)) == E_INVALID_ARG
    assert _tally_status(mcx, P, inputs.n_bins(d)) == E_STATE   # nothing ran


def test_tally_must_cover_geometry(mcx):
    d = inputs.cfg1_box(100)
    d["mesh_x"] = np.linspace(1.0, 10.0, d["mesh_n"][0] + 1)     # misses x in [0, 1)
    with pytest.raises(mcx.McxError) as e:
        mcx.Problem(d)
    assert e.value.status == E_INVALID_ARG
    c = inputs.pincell_ce(n_ebins=10, n_histories=10)
    c["e_edges"] = np.geomspace(1e-5, 1e7, 11)                   # below the 1.4e7 source energy
    with pytest.raises(mcx.McxError) as e:
        mcx.Problem(c)
    assert e.value.status == E_INVALID_ARG
