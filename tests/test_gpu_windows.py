"""GPU parity with weight windows: the closeout (an event of its own in the
split decomposition) splits heavy particles into copies run as later
generations, ordered by (parent, copy), and plays roulette with light ones.
Tallies, counters, the number of generations and generation 0's digests must
equal the oracle's on every scheduler and decomposition."""
import ctypes as C

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

INVARIANT = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
             "cutoffs", "killed", "pieces", "qsum", "overflow", "cdf_scans", "roulettes", "splits"]
SCHEDS = [("naive", "fused"), ("stack", "fused"), ("stack", "split"), ("async", "fused"), ("async", "split")]


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


def _check(P, ref):
    c = P.counters()
    for k in INVARIANT:
        assert c[k] == ref["counts"][k], (k, c[k], ref["counts"][k])
    assert c["generations"] == len(ref["generations"])


def _box():
    return inputs.with_weight_windows(inputs.with_implicit_capture(inputs.cfg1_box(5000), 0.25, 0.5),
                                      n=(4, 4, 4), lo_range=(0.05, 0.5))


def _lattice():
    return inputs.with_weight_windows(inputs.cfg2_lattice(3000), n=(5, 5, 2), lo_range=(0.1, 0.4))


def _pincell():
    d = inputs.with_implicit_capture(inputs.pincell_ce(n_ebins=200, n_histories=500, grid_len=4000), 0.2, 0.4)
    d["box_lo"] = np.array([-0.63, -0.63, -100.0])
    d["box_hi"] = np.array([0.63, 0.63, 100.0])
    return inputs.with_weight_windows(d, n=(3, 3, 2), lo_range=(0.1, 0.2))


@pytest.mark.parametrize("make", [_box, _lattice, _pincell], ids=["box", "lattice", "pincell"])
def test_windows_parity(mcx, oracle, make):
    d = make()
    ref = oracle.run(d, digest=True)
    assert len(ref["generations"]) > 2 and ref["counts"]["splits"] > 0 and ref["counts"]["roulettes"] > 0
    P = mcx.Problem(d)
    import torch
    for sched, decomp in SCHEDS:
        for lookup in (("binary", "hash") if d["energy_mode"] == 1 else ("binary",)):
            dg = torch.zeros(d["n_histories"] * 24, dtype=torch.uint8, device="cuda")
            P.run(sched=sched, decomp=decomp, lookup=lookup, digest=dg)
            assert np.array_equal(P.tallies(), ref["tally"]), (sched, decomp, lookup)
            _check(P, ref)
            assert np.array_equal(dg.cpu().numpy().view(mcx.DIGEST_DTYPE), ref["digest"]), (sched, decomp)


def test_windows_with_time_bins_and_ranges(mcx, oracle):
    d = inputs.with_time_bins(_box(), 6, 25.0)
    P = mcx.Problem(d)
    for h0, h1 in ((0, d["n_histories"]), (700, 2900)):
        ref = oracle.run_ww(d, h0, h1)
        for sched, decomp in (("async", "split"), ("stack", "fused"), ("naive", "fused")):
            P.run(sched=sched, decomp=decomp, first=h0, n=h1 - h0)
            assert np.array_equal(P.tallies(), ref["tally"]), (h0, sched, decomp)
            _check(P, ref)


def test_windows_forced_spills_and_shared_stash(mcx, oracle):
    d = _lattice()
    ref = oracle.run(d)
    P = mcx.Problem(d)
    for kw in ({"force_spill": 1}, {"async_shared_stash": 1, "force_spill": 2}, {"async_shared_stash": 1}):
        for decomp in ("fused", "split"):
            P.run(sched="async", decomp=decomp, **kw)
            assert np.array_equal(P.tallies(), ref["tally"]), (kw, decomp)
            _check(P, ref)


def test_windows_refused_where_not_supported(mcx):
    d = _box()
    P = mcx.Problem(d)
    P.run(sched="async")
    with pytest.raises(mcx.McxError) as e:
        P.backward(np.ones(inputs.n_bins(d)), sched="async")
    assert e.value.status == 1
    o = mcx.run_opts(sched="async")
    assert mcx.lib().mcx_run_noalloc(P.h, C.byref(o)) == 1
    with pytest.raises(mcx.McxError) as e:
        mcx.Problem([d, d])
    assert e.value.status == 1
    bad = dict(d)
    bad["ww_surv"] = 5.0                  # survival above the upper bound
    with pytest.raises(mcx.McxError):
        mcx.Problem(bad)
