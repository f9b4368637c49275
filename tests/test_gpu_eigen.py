"""GPU parity of k-eigenvalue power iteration (the paper's multigroup
workload, Sec. 4) against the CPU oracle.

Every cycle's histories, the fission bank (ordered by history), the
splitting-roulette copies and hence the next cycle's source are determined
by the random-number keys, so the active-cycle tally, k and the source size
of every cycle and the counters must match the oracle exactly on every
scheduler and event decomposition.
"""
import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

INVARIANT = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
             "cutoffs", "killed", "pieces", "qsum", "overflow", "cdf_scans", "fissions", "sites"]
SCHEDS = [("naive", "fused"), ("stack", "fused"), ("stack", "split"), ("async", "fused"), ("async", "split")]


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


def _check(P, got, ref, what):
    assert np.array_equal(P.tallies(), ref["tally"]), what
    assert np.array_equal(got["n_source"], ref["n_source"]), (what, got["n_source"], ref["n_source"])
    assert np.array_equal(got["k"], ref["k"]), (what, got["k"], ref["k"])
    c = P.counters()
    for k in INVARIANT:
        assert c[k] == ref["counts"][k], (what, k, c[k], ref["counts"][k])


@pytest.fixture(scope="module")
def lattice_k(oracle):
    d = inputs.with_fission(inputs.cfg2_lattice(1))
    return d, oracle.eigen(d, 20_000, 5, 2)


@pytest.mark.parametrize("sched,decomp", SCHEDS)
def test_lattice_eigen(mcx, lattice_k, sched, decomp):
    d, ref = lattice_k
    P = mcx.Problem(d)
    got = P.run_eigen(20_000, 5, 2, sched=sched, decomp=decomp)
    _check(P, got, ref, (sched, decomp))
    if sched == "async":
        got = P.run_eigen(20_000, 5, 2, sched=sched, decomp=decomp, async_block_waves=4)
        _check(P, got, ref, (sched, decomp, "4 waves per block"))


def test_slab_eigen_leakage_and_tally_paths(mcx, oracle):
    # vacuum x faces, only the middle slab fissile; a small mesh tally (LDS sums,
    # replicas or direct adds) and a ragged particle count
    st = np.array([[1.0], [0.8], [1.2]])
    ss = np.array([[0.7], [0.4], [0.9]])
    d = inputs.box_slabs_mg(planes_x=[0.0, 4.0, 6.0, 10.0], sigma_t=st, sigma_s=ss,
                            bc=[inputs.BC_VACUUM, inputs.BC_VACUUM] + [inputs.BC_REFLECT] * 4,
                            mesh_n=(10, 1, 1), n_histories=1)
    d = inputs.with_fission(d, fissile=[1], nu=np.full((3, 1), 2.5), chi=np.ones((3, 1)))
    ref = oracle.eigen(d, 7_777, 6, 2)
    P = mcx.Problem(d)
    for sched, decomp in SCHEDS:
        for path in ("lds", "replicas", "direct"):
            got = P.run_eigen(7_777, 6, 2, sched=sched, decomp=decomp, tally_path=path)
            _check(P, got, ref, (sched, decomp, path))


def test_cycle_zero_equals_fixed_source_run(mcx):
    d = inputs.with_fission(inputs.cfg2_lattice(6_000))
    P = mcx.Problem(d)
    P.run(sched="async")
    t0 = P.tallies()
    got = P.run_eigen(6_000, 1, 0, sched="stack")
    assert np.array_equal(P.tallies(), t0)
    assert got["n_source"][0] == 6_000
    # and again after an eigenvalue run: the handle's fixed-source state is intact
    P.run(sched="naive")
    assert np.array_equal(P.tallies(), t0)


def test_eigen_runs_back_to_back(mcx, lattice_k):
    d, ref = lattice_k
    P = mcx.Problem(d)
    a = P.run_eigen(20_000, 5, 2, sched="async")
    small = P.run_eigen(3_000, 3, 1, sched="stack")
    assert small["n_source"][0] == 3_000
    b = P.run_eigen(20_000, 5, 2, sched="naive")
    _check(P, b, ref, "third run")
    assert np.array_equal(a["k"], b["k"])


def test_eigen_invalid(mcx):
    base = inputs.cfg2_lattice(64)
    with pytest.raises(mcx.McxError) as e:
        mcx.Problem(base).run_eigen(100, 3, 1)            # no fission data
    assert e.value.status == 1
    d = inputs.with_fission(base)
    P = mcx.Problem(d)
    for n, c, i in ((0, 3, 1), (100, 0, 0), (100, 3, 4), (100, 3, -1)):
        with pytest.raises(mcx.McxError) as e:
            P.run_eigen(n, c, i)
        assert e.value.status == 1
    bad = dict(d, sigma_f=np.asarray(d["sigma_f"]) + 10.0)   # Sigma_f above Sigma_a
    with pytest.raises(mcx.McxError):
        mcx.Problem(bad)
    chi = np.asarray(d["chi"]).copy()
    chi[6] = 0.9                                            # a row ending below 1
    with pytest.raises(mcx.McxError):
        mcx.Problem(dict(d, chi=chi))
    with pytest.raises(mcx.McxError):
        mcx.Problem(inputs.with_time_bins(d, 4, 10.0)).run_eigen(100, 2, 1)
    with pytest.raises(mcx.McxError):
        mcx.Problem([d, d]).run_eigen(100, 2, 1)
