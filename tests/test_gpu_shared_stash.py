"""GPU parity of the asynchronous scheduler with a block-shared stash
(mcx_run_opts.async_shared_stash = 1: the wavefronts of a block share one
pool of work links through lock-free LDS transactions).  Tallies, counters
and per-history digests must equal the oracle's bit for bit: with tiny pools,
forced spills through the global arena, one to four wavefronts per block,
continuous energy, batches, the backward replays, time bins with weights and
the full-size lattice."""
import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

INVARIANT = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
             "cutoffs", "killed", "pieces", "qsum", "overflow", "cdf_scans", "roulettes"]


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
    return d, oracle.run(d, digest=True)


def _check(P, ref):
    c = P.counters()
    for k in INVARIANT:
        assert c[k] == ref["counts"][k], (k, c[k], ref["counts"][k])


def _digest(n):
    import torch
    return torch.zeros(n * 24, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("decomp", ["fused", "split"])
@pytest.mark.parametrize("knobs", [{}, {"async_block_waves": 1}, {"async_block_waves": 2},
                                   {"stash_links": 0, "force_spill": 1}, {"force_spill": 3},
                                   {"stash_links": 2}, {"stash_links": 5, "force_spill": 2},
                                   {"async_drain_events": 1}])
def test_lattice_shared(mcx, lattice, decomp, knobs):
    d, ref = lattice
    kw = dict(knobs)
    if decomp == "split" and kw.get("stash_links") == 2:
        kw["stash_links"] = 5           # one more than the events
    P = mcx.Problem(d)
    dg = _digest(d["n_histories"])
    P.run(sched="async", decomp=decomp, async_shared_stash=1, digest=dg, **kw)
    assert np.array_equal(P.tallies(), ref["tally"]), (decomp, kw)
    _check(P, ref)
    assert np.array_equal(dg.cpu().numpy().view(mcx.DIGEST_DTYPE), ref["digest"])
    if kw.get("force_spill"):
        assert P.counters()["spills"] > 0


@pytest.mark.parametrize("n_ebins", [100, 10000])
def test_ce_shared(mcx, oracle, n_ebins):
    d = inputs.pincell_ce(n_ebins=n_ebins, n_histories=1500)
    ref = oracle.run(d)
    P = mcx.Problem(d)
    for decomp in ("fused", "split"):
        for lookup in ("binary", "hash"):
            P.run(sched="async", decomp=decomp, lookup=lookup, async_shared_stash=1)
            assert np.array_equal(P.tallies(), ref["tally"]), (decomp, lookup)
            _check(P, ref)


def test_batch_shared(mcx, oracle):
    probs = inputs.cfg5_batch(n_problems=40, hist_scale=0.03)
    refs = [oracle.run(d) for d in probs]
    P = mcx.Problem(probs)
    for decomp in ("fused", "split"):
        for fs in (0, 2):
            P.run(sched="async", decomp=decomp, async_shared_stash=1, force_spill=fs)
            for k, ref in enumerate(refs):
                assert np.array_equal(P.tallies(k), ref["tally"]), (decomp, fs, k)


def test_backward_shared(mcx, oracle, lattice):
    d, _ = lattice
    P = mcx.Problem(d)
    w = np.random.default_rng(9).normal(size=inputs.n_bins(d))
    rb = oracle.backward(d, w)
    for decomp in ("fused", "split"):
        P.run(sched="async", decomp=decomp, async_shared_stash=1)
        gt, gs = P.backward(w, sched="async", decomp=decomp, async_shared_stash=1)
        assert np.array_equal(gt, rb["grad_sigma_t"]) and np.array_equal(gs, rb["grad_sigma_s"]), decomp


def test_time_weights_shared(mcx, oracle):
    d = inputs.with_implicit_capture(inputs.with_time_bins(inputs.cfg2_lattice(6000), 8, 60.0), 0.25, 0.5)
    ref = oracle.run(d)
    P = mcx.Problem(d)
    for decomp in ("fused", "split"):
        P.run(sched="async", decomp=decomp, async_shared_stash=1, force_spill=4)
        assert np.array_equal(P.tallies(), ref["tally"]), decomp
        _check(P, ref)


def test_lattice_1e6_shared(mcx, oracle):
    d = inputs.cfg2_lattice(1_000_000)
    ref = oracle.run(d)
    P = mcx.Problem(d)
    shapes = {}
    for decomp in ("fused", "split"):
        for mode in (1, 2, 0):
            P.run(sched="async", decomp=decomp, async_shared_stash=mode)
            assert np.array_equal(P.tallies(), ref["tally"]), (decomp, mode)
            _check(P, ref)
            c = P.counters()
            shapes[(decomp, mode)] = (c["block_threads"], c["lds_bytes"])
    # the default: the shared pool for split events at this size, one stash
    # per wavefront for fused events
    assert shapes[("split", 0)] == shapes[("split", 1)] != shapes[("split", 2)]
    assert shapes[("fused", 0)] == shapes[("fused", 2)]
