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
