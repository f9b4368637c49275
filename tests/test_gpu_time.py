"""GPU parity of time-binned tallies (the temporal tally resolution of
Sec. 4 of the paper) against the CPU oracle.

Time bins change the histories themselves: a flight that would reach t_max
stops there and its history ends, so the tallies, every invariant counter
and the per-history digests must all match bit for bit, on every scheduler
and event decomposition, through both tally paths (per-block LDS sums for
small tallies, global atomics or replicas for large ones), with tables in
LDS and in global memory, in batches, and in the score-function backward.
"""
import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

INVARIANT = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
             "cutoffs", "killed", "pieces", "qsum", "overflow", "cdf_scans"]
SCHEDS = [("naive", "fused"), ("stack", "fused"), ("stack", "split"), ("async", "fused"), ("async", "split")]
CE_SPEED = 1.383e6   # cm/s per sqrt(eV): a neutron's speed


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


def _digest(n):
    import torch
    return torch.zeros(n * 24, dtype=torch.uint8, device="cuda")


def _check(mcx, P, dg, ref, what):
    assert np.array_equal(P.tallies(), ref["tally"]), what
    got = P.counters()
    for k in INVARIANT:
        assert got[k] == ref["counts"][k], (what, k, got[k], ref["counts"][k])
    if dg is not None:
        assert np.array_equal(dg.cpu().numpy().view(mcx.DIGEST_DTYPE), ref["digest"]), what


@pytest.fixture(scope="module")
def lattice_t(oracle):
    # 8 time bins over the 51 x 51 x 20 x 7 mesh (2.9 M bins: global atomics);
    # group speeds 10^(-g/2), t_max = 100: about half the histories are cut
    d = inputs.with_time_bins(inputs.cfg2_lattice(12_000), 8, 100.0)
    ref = oracle.run(d, digest=True)
    c = ref["counts"]
    assert 0 < c["cutoffs"] < d["n_histories"] and c["absorbs"] > 0
    return d, ref


@pytest.mark.parametrize("sched,decomp", SCHEDS)
def test_lattice_time_bins(mcx, lattice_t, sched, decomp):
    d, ref = lattice_t
    P = mcx.Problem(d)
    dg = _digest(d["n_histories"])
    P.run(sched=sched, decomp=decomp, digest=dg)
    _check(mcx, P, dg, ref, (sched, decomp))


@pytest.mark.parametrize("n_tbins,t_max", [(2, 10.0), (16, 10.0), (1, 1e30)])
def test_box_time_bins_lds_and_global(mcx, oracle, n_tbins, t_max):
    # 2000 bins x 2 time bins fit the per-block LDS sums; x 16 do not
    d = inputs.with_time_bins(inputs.cfg1_box(8000), n_tbins, t_max)
    ref = oracle.run(d, digest=True)
    P = mcx.Problem(d)
    for sched, decomp in SCHEDS:
        dg = _digest(d["n_histories"])
        P.run(sched=sched, decomp=decomp, digest=dg)
        _check(mcx, P, dg, ref, (sched, decomp))


@pytest.mark.parametrize("n_ebins,n_tbins", [(100, 8), (1000, 8), (100, 128)])
def test_ce_time_bins(mcx, oracle, n_ebins, n_tbins):
    # 100 x 8 bins in LDS, 1000 x 8 and 100 x 128 in replicas; t_max = 2e-7 s
    # cuts most histories while they slow down, the rest are absorbed
    d = inputs.with_time_bins(inputs.pincell_ce(n_ebins=n_ebins, n_histories=600), n_tbins, 2e-7,
                              speed_coef=CE_SPEED)
    ref = oracle.run(d, digest=True)
    assert 0 < ref["counts"]["cutoffs"] < d["n_histories"]
    P = mcx.Problem(d)
    for sched, decomp in SCHEDS:
        for lookup in ("binary", "hash"):
            dg = _digest(d["n_histories"])
            P.run(sched=sched, decomp=decomp, lookup=lookup, digest=dg)
            _check(mcx, P, dg, ref, (sched, decomp, lookup))


def test_batch_time_bins(mcx, oracle):
    # per-problem time bins, widths and group speeds; tables read from global memory
    probs = inputs.cfg5_batch(n_problems=16, hist_scale=0.03)
    probs = [inputs.with_time_bins(d, 1 + (k % 4) * 3, 20.0 + 15.0 * k) for k, d in enumerate(probs)]
    refs = [oracle.run(d) for d in probs]
    assert sum(r["counts"]["cutoffs"] for r in refs) > 0
    P = mcx.Problem(probs)
    for sched, decomp in SCHEDS:
        P.run(sched=sched, decomp=decomp)
        for k, ref in enumerate(refs):
            assert np.array_equal(P.tallies(k), ref["tally"]), (sched, decomp, k)
        c = P.counters()
        for key in ("flights", "cutoffs", "pieces"):
            assert c[key] == sum(r["counts"][key] for r in refs), (sched, decomp, key)


def test_time_bins_tables_in_global_memory(mcx, oracle):
    # a single problem whose packed tables (transfer CDF of 8 x 40 x 40
    # doubles, 40 group speeds) exceed the LDS copy
    rng = np.random.default_rng(1007)
    n_mat, n_grp = 8, 40
    st, ss = inputs._mg_tables(rng, n_mat, n_grp, 0.3, 0.95)
    cdf = inputs._transfer_cdf(rng, n_mat, n_grp)
    d = inputs.box_slabs_mg(planes_x=np.linspace(0.0, 10.0, n_mat + 1), sigma_t=st, sigma_s=ss, cdf=cdf,
                            mesh_n=(6, 6, 6), n_histories=3000)
    d = inputs.with_time_bins(d, 4, 10.0, speed=np.linspace(1.0, 0.1, n_grp))
    ref = oracle.run(d)
    P = mcx.Problem(d)
    for sched, decomp in SCHEDS:
        P.run(sched=sched, decomp=decomp)
        _check(mcx, P, None, ref, (sched, decomp))


def test_time_bins_async_spills(mcx, lattice_t):
    # the time field travels with the particle through the global link arena
    d, ref = lattice_t
    P = mcx.Problem(d)
    for decomp in ("fused", "split"):
        P.run(sched="async", decomp=decomp, force_spill=3, stash_links=6)
        _check(mcx, P, None, ref, decomp)
        assert P.counters()["spills"] > 0


@pytest.mark.parametrize("sched", ["naive", "stack", "async"])
def test_time_bins_backward(mcx, oracle, sched):
    # the replays see the same cut flights: pass A weights pieces by the
    # time-binned dL/dT, pass B sums the cut track lengths
    d = inputs.with_time_bins(inputs.lattice_mg(n_histories=4000), 4, 150.0)
    nb = inputs.n_bins(d)
    w = np.random.default_rng(11).normal(size=nb)
    ref = oracle.backward(d, w)
    P = mcx.Problem(d)
    P.run(sched=sched)
    for decomp in (("fused", "split") if sched != "naive" else ("fused",)):
        gt, gs = P.backward(w, sched=sched, decomp=decomp)
        assert np.array_equal(gt, ref["grad_sigma_t"]), decomp
        assert np.array_equal(gs, ref["grad_sigma_s"]), decomp


def test_time_bins_invalid(mcx):
    base = inputs.cfg1_box(64)
    tb = inputs.with_time_bins(base, 4, 10.0)
    bad = [
        dict(tb, n_tbins=-1),
        dict(tb, t_max=0.0),
        dict(tb, t_max=float("inf")),
        dict(tb, speed=np.array([1.0, -1.0])),
        dict(tb, speed=np.array([1.0, 0.0])),
        dict(tb, speed=np.array([1.0, np.nan])),
    ]
    for d in bad:
        with pytest.raises(mcx.McxError) as e:
            mcx.Problem(d)
        assert e.value.status == 1
    ce = inputs.with_time_bins(inputs.pincell_ce(n_ebins=10, n_histories=8), 4, 1e-6, speed_coef=0.0)
    with pytest.raises(mcx.McxError):
        mcx.Problem(ce)
    # one speed per group, checked before the descriptor is built
    with pytest.raises(ValueError):
        mcx.Problem(dict(tb, speed=np.array([1.0])))
