"""Pins of the oracle's score-function (likelihood-ratio) backward.

For a linear loss L = sum_b w_b T_b with T_b the normalised track-length
tally, the gradient with respect to Sigma_t[m,g] and Sigma_s[m,g] is checked
against
* closed forms: one-group infinite medium, E[track] = 1/(Sigma_t - Sigma_s);
  multigroup infinite medium, d phi/d theta = -A^-1 (dA/d theta) phi with
  A = diag(Sigma_t) - M^T, M[g,g'] = Sigma_s,g P[g,g'];
* central finite differences with common random numbers (relative step
  1e-4), a different estimator of the same derivative (statistical z-test
  over independent seeds).

Implicit capture (weights Sigma_s / Sigma_t per collision, roulette below
the cutoff) has its own estimator: the same closed forms, the analog
estimator of the same derivative on a heterogeneous problem, and central
finite differences of the weighted forward with common random numbers.
"""
import math

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

SCALE = 2.0 ** -32


def _inf_medium(st, ss, cdf=None, n=4000, seed=99):
    return inputs.box_slabs_mg(size=(1.0, 1.0, 1.0), planes_x=[0.0, 1.0], slab_mat=[0],
                               bc=[inputs.BC_REFLECT] * 6, sigma_t=np.atleast_2d(st), sigma_s=np.atleast_2d(ss),
                               cdf=cdf, src_pos=[0.5, 0.5, 0.5], mesh_n=(1, 1, 1), n_histories=n, seed=seed)


def test_pass_a_is_weighted_track_length(oracle):
    d = inputs.cfg1_box(3000)
    fw = oracle.run(d, digest=True)
    G, U = oracle.replay_a(d, np.ones(2000))
    q = fw["digest"]["qsum"] * SCALE
    assert np.all(np.abs(G - q) <= 1e-6)
    # weights pick out bins: G with one-hot w equals that history's share of the bin
    w = np.zeros(2000)
    w[int(np.argmax(fw["tally"]))] = 1.0
    G1, _ = oracle.replay_a(d, w)
    assert abs(G1.sum() - fw["tally"].max() * SCALE) < 1e-5
    assert U >= 1 and oracle.grad_scale(U) < 62


def test_fixed_point_sums_fit(oracle):
    d = inputs.cfg1_box(3000)
    w = np.random.default_rng(3).normal(size=2000)
    out = oracle.backward(d, w)
    for k in ("SL", "SA", "SS"):
        assert np.all(np.abs(out[k].astype(np.float64)) < 2.0 ** 63)
    # the scale is chosen so the largest sum uses most of the 62 bits
    assert max(np.abs(out["SL"]).max(), np.abs(out["SS"]).max()) > 2.0 ** 50


def _replicates(oracle, d, w, seeds):
    gts, gss = [], []
    for s in seeds:
        d = dict(d, seed=int(s))
        out = oracle.backward(d, w)
        gts.append(out["grad_sigma_t"])
        gss.append(out["grad_sigma_s"])
    return np.array(gts), np.array(gss)


def test_grad_one_group_closed_form(oracle):
    st, ss = 1.2, 0.6
    d = _inf_medium([[st]], [[ss]], n=4000)
    gts, gss = _replicates(oracle, d, np.ones(1), range(1, 13))
    sa = st - ss
    for est, ref in ((gts[:, 0], -1.0 / sa ** 2), (gss[:, 0], 1.0 / sa ** 2)):
        se = est.std(ddof=1) / math.sqrt(est.size)
        assert abs(est.mean() - ref) < 4 * se, (est.mean(), ref, se)


def test_grad_multigroup_closed_form(oracle):
    rng = np.random.default_rng(51)
    G = 3
    st = rng.uniform(0.6, 1.4, G)
    ss = st * rng.uniform(0.4, 0.7, G)
    P = np.triu(rng.uniform(0.2, 1.0, (G, G)))
    P /= P.sum(axis=1, keepdims=True)
    cdf = np.cumsum(P, axis=1)
    cdf[:, -1] = 1.0
    d = _inf_medium(st[None, :], ss[None, :], cdf=cdf[None], n=4000)
    w = rng.uniform(0.5, 2.0, G)
    A = np.diag(st) - (ss[:, None] * P).T
    phi = np.linalg.solve(A, np.eye(G)[0])
    ref_t = np.empty(G)
    ref_s = np.empty(G)
    for g in range(G):
        dA = np.zeros((G, G))
        dA[g, g] = 1.0
        ref_t[g] = w @ (-np.linalg.solve(A, dA @ phi))
        dA = np.zeros((G, G))
        dA[:, g] = -P[g, :]
        ref_s[g] = w @ (-np.linalg.solve(A, dA @ phi))
    gts, gss = _replicates(oracle, d, w, range(1, 13))
    for est, ref in ((gts, ref_t), (gss, ref_s)):
        se = est.std(axis=0, ddof=1) / math.sqrt(est.shape[0])
        assert np.all(np.abs(est.mean(axis=0) - ref) < 4 * se), (est.mean(axis=0), ref, se)


def test_grad_matches_central_fd(oracle):
    d0 = inputs.cfg1_box(20000)
    nb = 2000
    w = np.random.default_rng(61).uniform(-1.0, 1.0, nb)
    h = 1e-4
    n = d0["n_histories"]
    diffs_t, diffs_s = [], []
    for seed in range(1, 9):
        d = dict(d0, seed=seed)
        sf = oracle.backward(d, w)
        fd_t = np.empty(4)
        fd_s = np.empty(4)
        for p in range(4):
            for key, out in (("sigma_t", fd_t), ("sigma_s", fd_s)):
                vals = []
                for sgn in (1.0, -1.0):
                    dd = dict(d)
                    arr = np.array(d[key], dtype=np.float64)
                    step = h * arr[p]
                    arr[p] = arr[p] + sgn * step
                    dd[key] = arr
                    t = oracle.run(dd)["tally"] * SCALE / n
                    vals.append(float(w @ t))
                out[p] = (vals[0] - vals[1]) / (2 * step)
        diffs_t.append(sf["grad_sigma_t"] - fd_t)
        diffs_s.append(sf["grad_sigma_s"] - fd_s)
    for diffs in (np.array(diffs_t), np.array(diffs_s)):
        mean = diffs.mean(axis=0)
        se = diffs.std(axis=0, ddof=1) / math.sqrt(diffs.shape[0])
        assert np.all(np.abs(mean) < 4 * se + 1e-9), (mean, se)


# ------------------------------------------------------------ implicit capture

def _implicit(d, cut=0.25, surv=0.5):
    return inputs.with_implicit_capture(d, cut, surv)


def _z_ok(est, ref, k=4.0):
    est = np.atleast_2d(np.asarray(est).T).T
    se = est.std(axis=0, ddof=1) / math.sqrt(est.shape[0])
    return np.all(np.abs(est.mean(axis=0) - ref) < k * se), (est.mean(axis=0), ref, se)


def test_weighted_pass_a_is_weighted_track_length(oracle):
    d = _implicit(inputs.cfg1_box(3000))
    fw = oracle.run(d, digest=True)
    G, U = oracle.replay_a(d, np.ones(2000))
    q = fw["digest"]["qsum"] * SCALE
    assert np.all(np.abs(G - q) <= 1e-6)
    assert fw["counts"]["roulettes"] > 0 and fw["counts"]["absorbs"] == 0


def test_weighted_fixed_point_sums_fit(oracle):
    d = _implicit(inputs.cfg1_box(3000))
    w = np.random.default_rng(3).normal(size=2000)
    out = oracle.backward(d, w)
    top = max(np.abs(out[k].astype(np.float64)).max() for k in ("SL", "SA", "SS"))
    assert top < 2.0 ** 62 and top > 2.0 ** 48


def test_weighted_pass_b_needs_weights(oracle):
    d = _implicit(inputs.cfg1_box(100))
    G, U = oracle.replay_a(d, np.ones(2000))
    with pytest.raises(ValueError):
        oracle.replay_b(d, G, oracle.grad_scale(U))


@pytest.mark.parametrize("cut,surv", [(0.25, 0.5), (0.05, 0.2)])
def test_weighted_grad_one_group_closed_form(oracle, cut, surv):
    # E[weighted track length] = 1 / (Sigma_t - Sigma_s) as in the analog game
    st, ss = 1.2, 0.9
    d = _implicit(_inf_medium([[st]], [[ss]], n=4000), cut, surv)
    gts, gss = _replicates(oracle, d, np.ones(1), range(1, 13))
    sa = st - ss
    for est, ref in ((gts[:, 0], -1.0 / sa ** 2), (gss[:, 0], 1.0 / sa ** 2)):
        ok, info = _z_ok(est, ref)
        assert ok, info


def test_weighted_grad_multigroup_closed_form(oracle):
    rng = np.random.default_rng(52)
    G = 3
    st = rng.uniform(0.6, 1.4, G)
    ss = st * rng.uniform(0.5, 0.8, G)
    P = rng.uniform(0.2, 1.0, (G, G))
    P /= P.sum(axis=1, keepdims=True)
    cdf = np.cumsum(P, axis=1)
    cdf[:, -1] = 1.0
    d = _implicit(_inf_medium(st[None, :], ss[None, :], cdf=cdf[None], n=4000))
    w = rng.uniform(-1.0, 2.0, G)
    A = np.diag(st) - (ss[:, None] * P).T
    phi = np.linalg.solve(A, np.eye(G)[0])
    lam = np.linalg.solve(A.T, w)
    ref_t = -lam * phi                       # dA/dSigma_t,g = e_g e_g^T
    ref_s = phi * (P @ lam)                  # dA/dSigma_s,g = -P[g, :] in column g
    gts, gss = _replicates(oracle, d, w, range(1, 13))
    for est, ref in ((gts, ref_t), (gss, ref_s)):
        ok, info = _z_ok(est, ref)
        assert ok, info


def test_weighted_grad_matches_analog(oracle):
    # two estimators of one derivative on a heterogeneous box: the analog
    # game and the weighted one, on independent seeds
    d0 = inputs.cfg1_box(6000)
    w = np.random.default_rng(62).uniform(-0.5, 1.0, 2000)
    ga = _replicates(oracle, d0, w, range(1, 11))
    gw = _replicates(oracle, _implicit(d0), w, range(101, 111))
    for a, b in zip(ga, gw):
        diff = a.mean(axis=0) - b.mean(axis=0)
        se = np.sqrt(a.var(axis=0, ddof=1) / a.shape[0] + b.var(axis=0, ddof=1) / b.shape[0])
        assert np.all(np.abs(diff) < 4.5 * se + 1e-12), (diff, se)


def test_weighted_grad_matches_central_fd(oracle):
    d0 = _implicit(inputs.cfg1_box(8000))
    nb = 2000
    w = np.random.default_rng(63).uniform(-1.0, 1.0, nb)
    h = 1e-3
    n = d0["n_histories"]
    mg = np.asarray(d0["sigma_t"]).size
    diffs_t, diffs_s = [], []
    for seed in range(1, 9):
        d = dict(d0, seed=seed)
        sf = oracle.backward(d, w)
        fd = {}
        for key in ("sigma_t", "sigma_s"):
            fd[key] = np.empty(mg)
            for p in range(mg):
                vals = []
                for sgn in (1.0, -1.0):
                    arr = np.array(d[key], dtype=np.float64)
                    step = h * arr.flat[p]
                    arr.flat[p] = arr.flat[p] + sgn * step
                    t = oracle.run(dict(d, **{key: arr}))["tally"] * SCALE / n
                    vals.append(float(w @ t))
                fd[key][p] = (vals[0] - vals[1]) / (2 * step)
        diffs_t.append(sf["grad_sigma_t"] - fd["sigma_t"])
        diffs_s.append(sf["grad_sigma_s"] - fd["sigma_s"])
    for diffs in (np.array(diffs_t), np.array(diffs_s)):
        ok, info = _z_ok(diffs, 0.0, 4.5)
        assert ok, info
