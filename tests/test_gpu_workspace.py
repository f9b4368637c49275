"""GPU: runs on a caller-owned workspace (mcx_run_opts.workspace, ws_bytes).

Device memory for the scheduler state and tally replicas comes from a torch
allocation sized by mcx_workspace_size; tallies, counters and gradients must
equal the oracle's (and the library-workspace run's) bit for bit, and a
workspace that is too small is refused before anything runs.
"""
import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

INVARIANT = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
             "cutoffs", "killed", "pieces", "qsum", "overflow", "cdf_scans"]
SCHEDS = [("naive", "fused"), ("stack", "fused"), ("stack", "split"), ("async", "fused"), ("async", "split")]


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


def _ws(nbytes):
    import torch
    return torch.full((max(nbytes, 1),), 0xA5, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("sched,decomp", SCHEDS)
def test_run_on_caller_workspace(mcx, lattice, sched, decomp):
    d, ref = lattice
    P = mcx.Problem(d)
    need = P.workspace_size(sched=sched, decomp=decomp)
    ws = _ws(need)
    for _ in range(2):                   # the second run reuses the dirty workspace
        P.run(sched=sched, decomp=decomp, workspace=ws)
        assert np.array_equal(P.tallies(), ref["tally"])
        c = P.counters()
        for k in INVARIANT:
            assert c[k] == ref["counts"][k], (k, c[k], ref["counts"][k])


@pytest.mark.parametrize("sched", ["stack", "async"])
def test_backward_on_caller_workspace(mcx, lattice, oracle, sched):
    d, _ = lattice
    P = mcx.Problem(d)
    ws = _ws(P.workspace_size(sched=sched))
    w = np.random.default_rng(5).normal(size=inputs.n_bins(d))
    P.run(sched=sched, workspace=ws)
    gt, gs = P.backward(w, sched=sched, workspace=ws)
    rb = oracle.backward(d, w)
    assert np.array_equal(gt, rb["grad_sigma_t"]) and np.array_equal(gs, rb["grad_sigma_s"])


def test_replica_tally_in_caller_workspace(mcx, oracle):
    # an energy tally above the LDS limit: its 16 replicas live in the
    # workspace behind the scheduler state
    d = inputs.pincell_ce(n_ebins=10_000, n_histories=3000)
    ref = oracle.run(d)
    P = mcx.Problem(d)
    for sched in ("naive", "async", "stack"):
        need = P.workspace_size(sched=sched, tally_path="replicas")
        assert need >= 16 * 10_000 * 8
        P.run(sched=sched, tally_path="replicas", workspace=_ws(need))
        assert np.array_equal(P.tallies(), ref["tally"]), sched


def test_workspace_too_small_is_refused(mcx, lattice):
    d, ref = lattice
    P = mcx.Problem(d)
    need = P.workspace_size(sched="async")
    # (the size covers the backward's larger replay particle as well, so
    # half of it is too small for the forward's link arena)
    small = _ws(need // 2)
    with pytest.raises(mcx.McxError) as e:
        P.run(sched="async", workspace=small)
    assert e.value.status == 1
    with pytest.raises(mcx.McxError):
        P.tallies()                      # nothing ran: no valid tallies
    # misaligned pointers are refused as well
    import torch
    big = _ws(need + 512)
    o = mcx.run_opts(sched="async")
    o.workspace = big.data_ptr() + 8
    o.ws_bytes = need
    st = mcx.lib().mcx_run(P.h, mcx.C.byref(o))
    assert st == 1
    # and the exact size is enough
    P.run(sched="async", workspace=_ws(need))
    assert np.array_equal(P.tallies(), ref["tally"])
