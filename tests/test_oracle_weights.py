"""Oracle pins for non-analog weights: implicit capture and the closeout's
weight roulette (the "weights and weight windows" part of the paper's
decomposed transport loop, Sec. 4).

With implicit capture a collision never absorbs: the particle scatters and
its weight is multiplied by the scattering probability; below w_cutoff a
roulette keeps it with probability w / w_survival at weight w_survival.
Tallies score length times weight.
"""
import math

import numpy as np

from paper_2506_00263_amd import inputs

SCALE = 2.0 ** -32


def _infinite(st, ss, n, w_cutoff, w_survival, seed=inputs.TRANSPORT_SEED_BASE):
    d = inputs.box_slabs_mg(sigma_t=[[st]], sigma_s=[[ss]], bc=[inputs.BC_REFLECT] * 6, mesh_n=(1, 1, 1),
                            n_histories=n, seed=seed)
    return inputs.with_implicit_capture(d, w_cutoff, w_survival)


def test_roulette_happens_at_predictable_collisions(oracle):
    # Sigma_s / Sigma_t = 1/2: the weight halves exactly at every collision.
    # From 1 it first drops below 0.1 at collision 4 (0.0625); a survivor
    # restarts at 0.5 and drops below again 3 collisions later.  Each roulette
    # is survived with probability 0.0625 / 0.5 = 1/8.
    n = 40_000
    r = oracle.run(_infinite(1.0, 0.5, n, 0.1, 0.5), digest=True)
    dg = r["digest"]
    col = dg["collisions"].astype(np.int64)
    assert np.all(dg["fate"] == 4)
    assert np.all((col >= 4) & ((col - 4) % 3 == 0))
    c = r["counts"]
    assert c["roulettes"] == n and c["absorbs"] == 0 and c["scatters"] == c["collisions"]
    p4 = np.mean(col == 4)
    assert abs(p4 - 0.875) < 5 * math.sqrt(0.875 * 0.125 / n), p4
    # roulettes survived: geometric with mean (1/8) / (7/8)
    surv = (col - 4) // 3
    assert abs(surv.mean() - 1.0 / 7.0) < 5 * math.sqrt((1.0 / 8.0) / (7.0 / 8.0) ** 2 / n)


def test_implicit_capture_is_unbiased_in_an_infinite_medium(oracle):
    # the expected track length per source particle is 1 / Sigma_a whatever
    # the weighting; compare the mean weighted track with its standard error
    st, ss, n = 1.0, 0.8, 100_000
    r = oracle.run(_infinite(st, ss, n, 0.25, 0.5), digest=True)
    per = r["digest"]["qsum"].astype(np.float64) * SCALE
    se = per.std(ddof=1) / math.sqrt(n)
    assert abs(per.mean() - 1.0 / (st - ss)) < 5 * se, (per.mean(), se)
    # and the analog estimate of the same quantity has the larger spread
    a = oracle.run(dict(_infinite(st, ss, n, 0.25, 0.5), implicit_capture=0), digest=True)
    pa = a["digest"]["qsum"].astype(np.float64) * SCALE
    assert per.std() < pa.std()


def test_no_cutoff_ends_histories_only_by_leaking(oracle):
    # vacuum box, no roulette (cutoff 0): a weighted particle never dies in a collision
    d = inputs.with_implicit_capture(inputs.cfg1_box(3000), 0.0, 1.0)
    r = oracle.run(d, digest=True)
    c = r["counts"]
    assert c["leaks"] == 3000 and c["absorbs"] == 0 and c["roulettes"] == 0
    assert np.all(r["digest"]["fate"] == 0)


def test_weighted_tallies_agree_with_analog_ones(oracle):
    # the lattice: mesh-tally totals from weighted and analog histories estimate
    # the same expectation (independent streams: two-sample test on the totals
    # of 20 batches each)
    def batches(d, seeds):
        out = []
        for s in seeds:
            out.append(oracle.run(dict(d, seed=s))["tally"].astype(np.float64).sum() * SCALE / d["n_histories"])
        return np.array(out)
    d = inputs.cfg2_lattice(2000)
    a = batches(d, range(100, 120))
    w = batches(inputs.with_implicit_capture(d, 0.25, 0.5), range(200, 220))
    se = math.sqrt(a.var(ddof=1) / a.size + w.var(ddof=1) / w.size)
    assert abs(a.mean() - w.mean()) < 5 * se, (a.mean(), w.mean(), se)


def test_continuous_energy_weights(oracle):
    # implicit capture with species selection: the weight takes the chosen
    # species' scattering probability; the slowing-down track totals agree
    # with analog histories (batches, two-sample test)
    def batches(d, seeds):
        return np.array([oracle.run(dict(d, seed=s))["tally"].astype(np.float64).sum() / d["n_histories"]
                         for s in seeds])
    d = inputs.pincell_ce(n_ebins=50, n_histories=150, grid_len=2000)
    a = batches(d, range(300, 316))
    w = batches(inputs.with_implicit_capture(d, 0.1, 0.4), range(400, 416))
    se = math.sqrt(a.var(ddof=1) / a.size + w.var(ddof=1) / w.size)
    assert abs(a.mean() - w.mean()) < 5 * se, (a.mean(), w.mean(), se)
    r = oracle.run(inputs.with_implicit_capture(d, 0.1, 0.4))
    assert r["counts"]["absorbs"] == 0 and r["counts"]["roulettes"] + r["counts"]["cutoffs"] == d["n_histories"]


def test_analog_runs_are_unchanged_by_the_weight_fields(oracle):
    d = inputs.cfg2_lattice(2000)
    a = oracle.run(d, digest=True)
    b = oracle.run(dict(d, w_cutoff=0.3, w_survival=0.9), digest=True)   # implicit capture off
    assert np.array_equal(a["tally"], b["tally"]) and np.array_equal(a["digest"], b["digest"])


# ------------------------------------------------------------ weight windows

def _ww_infinite(st, ss, n, lo, implicit=True, ratio=4.0, surv=2.0, max_split=8, grid=(2, 2, 2)):
    d = inputs.box_slabs_mg(sigma_t=[[st]], sigma_s=[[ss]], bc=[inputs.BC_REFLECT] * 6, mesh_n=(1, 1, 1),
                            src_kind=inputs.SRC_BOX, src_lo=[0.0, 0.0, 0.0], src_hi=[10.0, 10.0, 10.0],
                            n_histories=n)
    if implicit:
        d = inputs.with_implicit_capture(d, 0.0, 1.0)
    return inputs.with_weight_windows(d, n=grid, lo=lo, ratio=ratio, surv=surv, max_split=max_split)


def test_windows_unbiased_one_group(oracle):
    # infinite medium, one group, implicit capture with windows that split in
    # some cells and roulette in others: track length per source particle is
    # still 1 / Sigma_a
    st, ss = 1.0, 0.8
    lo = np.array([0.02, 0.3, 0.05, 0.2, 0.1, 0.4, 0.03, 0.25])
    d = _ww_infinite(st, ss, 20000, lo)
    batches = 10
    per = d["n_histories"] // batches
    est = []
    splits = rou = 0
    for b in range(batches):
        r = oracle.run(d, b * per, (b + 1) * per)
        est.append(r["tally"].sum() * SCALE / per)
        splits += r["counts"]["splits"]
        rou += r["counts"]["roulettes"]
        assert len(r["generations"]) > 1
    est = np.array(est)
    mean, se = est.mean(), est.std(ddof=1) / math.sqrt(batches)
    assert splits > 1000 and rou > 1000
    assert abs(mean - 1.0 / (st - ss)) < 4 * se, (mean, se)


def test_windows_unbiased_multigroup(oracle):
    # multigroup infinite medium: per-group track lengths solve
    # (diag Sigma_t - M^T) phi = e_0, windows or not
    rng = np.random.default_rng(41)
    G = 3
    st = rng.uniform(0.6, 1.4, G)
    ss = st * rng.uniform(0.5, 0.85, G)
    P = np.zeros((G, G))
    for g in range(G):
        w = rng.uniform(0.1, 1.0, G) * (np.arange(G) >= g)
        P[g] = w / w.sum()
    cdf = np.cumsum(P, axis=1)
    cdf[:, -1] = 1.0
    d = inputs.box_slabs_mg(sigma_t=st[None], sigma_s=ss[None], cdf=cdf[None], bc=[inputs.BC_REFLECT] * 6,
                            mesh_n=(1, 1, 1), src_kind=inputs.SRC_BOX, src_lo=[0.0, 0.0, 0.0],
                            src_hi=[10.0, 10.0, 10.0], n_histories=30000)
    d = inputs.with_weight_windows(inputs.with_implicit_capture(d, 0.0, 1.0), n=(3, 3, 3), lo_range=(0.03, 0.4))
    phi = np.linalg.solve(np.diag(st) - (ss[:, None] * P).T, np.eye(G)[0])
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * SCALE / per for b in range(batches)])
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / math.sqrt(batches)
    assert np.all(np.abs(mean - phi) < 4 * se + 1e-12), (mean, phi, se)


def test_split_copies_conserve_weight(oracle):
    # a window whose upper bound is below the starting weight 1: the first
    # closeout splits weight 1 into n = floor(1 / (surv lo)) copies of exactly
    # 1 / n (clamped to max_split); analog collisions keep the weight, so
    # every banked copy of generation 1 carries 1 / n
    lo = 0.05                             # upper 0.2, survival 0.1: n = 10 -> 8
    d = _ww_infinite(1.0, 0.9, 400, np.full(8, lo), implicit=False)
    r = oracle.run_ww(d)
    gens = r["generations"]
    # a source particle that reaches a closeout (not absorbed first) splits
    # once into 8 and its copies stay at 1/8 inside the windows
    assert len(gens) == 2 and gens[1] % 7 == 0 and gens[1] > 7 * 300
    P = oracle.Problem(d)
    L = oracle.lib()
    bank = (oracle.OrcSite * 8000)()
    n = oracle.C.c_uint64(0)
    t = np.zeros(P.n_bins, np.int64)
    cnt = oracle.OrcCounts()
    assert L.orc_run_gen(oracle.C.byref(P.s), 0, None, 0, 400, t.ctypes.data_as(oracle.C.c_void_p), None,
                         oracle.C.byref(cnt), oracle.C.cast(bank, oracle.C.c_void_p), 8000, oracle.C.byref(n)) == 0
    w = np.array([bank[i].w for i in range(n.value)])
    assert n.value == gens[1] and np.all(w == 1.0 / 8.0)
    # copies of one split share the parent's state; 7 per parent, in order
    k = n.value // 7
    pos = np.array([[bank[i].pos[a] for a in range(3)] for i in range(n.value)])
    assert np.all(pos.reshape(k, 7, 3) == pos.reshape(k, 7, 3)[:, :1, :])
    assert cnt.splits == n.value


def test_windows_that_never_act(oracle):
    # lower bounds of 0 (no window anywhere): the closeout does nothing and
    # the run equals implicit capture without roulette, bit for bit
    # (a vacuum box: without roulette only leakage ends a history)
    d0 = inputs.with_implicit_capture(inputs.cfg1_box(3000), 0.0, 1.0)
    d1 = inputs.with_weight_windows(d0, n=(2, 3, 1), lo=np.zeros(6))
    a = oracle.run(d0)
    b = oracle.run(d1)
    assert np.array_equal(a["tally"], b["tally"]) and b["generations"] == [3000]
    assert b["counts"]["splits"] == 0 and b["counts"]["roulettes"] == 0
