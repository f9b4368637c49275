"""Pins of the oracle's whole-history transport against closed forms.

* uncollided transmission of a beam through a slab: exp(-Sigma_t x)
* one-group infinite medium: track length per source particle 1/Sigma_a,
  collisions 1/(1-c), scatters c/(1-c)
* multigroup infinite medium: per-group track length solves
  (diag Sigma_t - M^T) phi = e_0 with M[g,g'] = Sigma_s,g P[g,g']
* elastic slowing down in an infinite non-absorbing medium: track length per
  unit lethargy 1/(xi Sigma_s), xi = 1 + (A-1)^2/(2A) ln((A-1)/(A+1))
* elastic kinematics: E'/E mean (A^2+1)/(A+1)^2, mean lab cosine 2/(3A),
  cos(angle(old, new)) = mu_L, unit direction
* integer bookkeeping: sum of bins = total of contributions, range splits and
  thread counts give identical integers

Statistical checks use |z| < 4 with fixed seeds.
"""
import math

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

SCALE = 2.0 ** -32


def _inf_medium(sigma_t, sigma_s, cdf=None, n=20000, seed=777):
    st = np.atleast_2d(np.asarray(sigma_t, float))
    ss = np.atleast_2d(np.asarray(sigma_s, float))
    return inputs.box_slabs_mg(size=(1.0, 1.0, 1.0), planes_x=[0.0, 1.0], slab_mat=[0],
                               bc=[inputs.BC_REFLECT] * 6, sigma_t=st, sigma_s=ss, cdf=cdf,
                               src_pos=[0.5, 0.5, 0.5], mesh_n=(1, 1, 1), n_histories=n, seed=seed)


def _z(mean, ref, se):
    return abs(mean - ref) / se


def test_uncollided_slab_transmission(oracle):
    thick, st = 2.0, 0.8
    d = inputs.box_slabs_mg(size=(thick, 1e6, 1e6), planes_x=[0.0, thick], slab_mat=[0],
                            sigma_t=[[st]], sigma_s=[[0.5 * st]], src_pos=[0.0, 5e5, 5e5], src_isotropic=0,
                            src_dir=[1.0, 0.0, 0.0], mesh_n=(1, 1, 1), n_histories=40000)
    r = oracle.run(d, digest=True)
    dg = r["digest"]
    through = np.count_nonzero((dg["collisions"] == 0) & (dg["fate"] == 0))
    n = dg.size
    p = math.exp(-st * thick)
    se = math.sqrt(p * (1 - p) / n)
    assert _z(through / n, p, se) < 4
    # and every uncollided history is exactly one flight of length `thick`
    unc = dg[(dg["collisions"] == 0)]
    assert np.all(unc["flights"] == 1)
    assert np.all(np.abs(unc["qsum"] * SCALE - thick) < 1e-9)


@pytest.mark.parametrize("st,c", [(1.0, 0.5), (0.4, 0.9), (2.0, 0.3)])
def test_infinite_medium_one_group(oracle, st, c):
    d = _inf_medium([[st]], [[c * st]])
    r = oracle.run(d, digest=True)
    dg = r["digest"]
    n = dg.size
    track = dg["qsum"] * SCALE
    assert _z(track.mean(), 1.0 / (st * (1 - c)), track.std() / math.sqrt(n)) < 4
    coll = dg["collisions"].astype(float)
    assert _z(coll.mean(), 1.0 / (1 - c), coll.std() / math.sqrt(n)) < 4
    sc = coll - 1.0                      # every history ends in one absorption
    assert np.all(dg["fate"] == 1)
    assert _z(sc.mean(), c / (1 - c), sc.std() / math.sqrt(n)) < 4
    assert r["counts"]["scatters"] == int(sc.sum())


def test_infinite_medium_multigroup(oracle):
    rng = np.random.default_rng(21)
    G = 4
    st = rng.uniform(0.5, 1.5, G)
    ss = st * rng.uniform(0.4, 0.8, G)
    P = np.zeros((G, G))
    for g in range(G):
        w = rng.uniform(0.1, 1.0, G) * (np.arange(G) >= g - 1)
        P[g] = w / w.sum()
    cdf = np.cumsum(P, axis=1)
    cdf[:, -1] = 1.0
    d = _inf_medium(st[None, :], ss[None, :], cdf=cdf[None], n=40000)
    d["mesh_n"] = np.array([1, 1, 1], np.int32)
    M = ss[:, None] * P
    phi = np.linalg.solve(np.diag(st) - M.T, np.eye(G)[0])
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * SCALE / per for b in range(batches)])
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / math.sqrt(batches)
    assert np.all(np.abs(mean - phi) < 4 * se + 1e-12), (mean, phi, se)


def test_cdf_scans_in_group_scatter(oracle):
    """Transfer rows that keep every scatter in its group (the CDF jumps to 1
    at the incoming group): finding group g reads entries 0..g, so each
    scatter from source group g0 reads exactly g0 + 1 entries."""
    G, g0 = 5, 3
    st = np.linspace(0.6, 1.4, G)
    ss = 0.7 * st
    cdf = np.zeros((G, G))
    for g in range(G):
        cdf[g, g:] = 1.0
    d = _inf_medium(st[None, :], ss[None, :], cdf=cdf[None], n=3000)
    d["src_group"] = g0
    c = oracle.run(d)["counts"]
    assert c["scatters"] > 1000
    assert c["cdf_scans"] == (g0 + 1) * c["scatters"]
    # one group: one entry per scatter
    c1 = oracle.run(_inf_medium([[1.0]], [[0.8]], n=2000))["counts"]
    assert c1["cdf_scans"] == c1["scatters"] > 0


def test_cdf_scans_multigroup_mean(oracle):
    """Expected entries read per history in a multigroup infinite medium:
    sum over g of (scatters out of g) times sum_k (k+1) P[g,k], with the
    scatters out of g equal to Sigma_s,g phi_g and phi from the linear solve
    (diag Sigma_t - M^T) phi = e_0."""
    rng = np.random.default_rng(33)
    G = 5
    st = rng.uniform(0.5, 1.5, G)
    ss = st * rng.uniform(0.5, 0.85, G)
    P = np.zeros((G, G))
    for g in range(G):
        w = rng.uniform(0.1, 1.0, G)
        P[g] = w / w.sum()
    cdf = np.cumsum(P, axis=1)
    cdf[:, -1] = 1.0
    d = _inf_medium(st[None, :], ss[None, :], cdf=cdf[None], n=40000)
    M = ss[:, None] * P
    phi = np.linalg.solve(np.diag(st) - M.T, np.eye(G)[0])
    expect = float(np.sum(ss * phi * (P @ (np.arange(G) + 1.0))))
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["counts"]["cdf_scans"] / per for b in range(batches)])
    assert _z(est.mean(), expect, est.std(ddof=1) / math.sqrt(batches)) < 4, (est.mean(), expect)


def test_sum_of_bins_equals_total(oracle):
    d = inputs.cfg1_box(5000)
    r = oracle.run(d, digest=True)
    assert int(r["tally"].sum()) == r["counts"]["qsum"] == int(r["digest"]["qsum"].sum())
    assert int(r["digest"]["flights"].sum()) == r["counts"]["flights"]
    assert int(r["digest"]["collisions"].sum()) == r["counts"]["collisions"]
    c = r["counts"]
    assert c["collisions"] == c["scatters"] + c["absorbs"]
    assert c["flights"] == c["collisions"] + c["crossings"]
    assert c["sourced"] == 5000 == c["leaks"] + c["absorbs"] + c["cutoffs"] + c["killed"]


def test_threads_and_ranges_are_exact(oracle):
    d = inputs.cfg2_lattice(3000)
    a = oracle.run(d, threads=1)
    b = oracle.run(d, threads=7)
    c1 = oracle.run(d, 0, 1234, threads=3)
    c2 = oracle.run(d, 1234, 3000, threads=2)
    assert np.array_equal(a["tally"], b["tally"])
    assert np.array_equal(a["tally"], c1["tally"] + c2["tally"])
    assert a["counts"] == b["counts"]


def test_max_steps_kills(oracle):
    d = inputs.cfg2_lattice(500)
    d["max_steps"] = 3
    r = oracle.run(d, digest=True)
    dg = r["digest"]
    killed = dg["fate"] == 3
    assert killed.sum() == r["counts"]["killed"] > 0
    assert np.all(dg["flights"][killed] == 3)
    assert np.all(dg["flights"] <= 3)


def test_overflow_flag(oracle):
    d = inputs.cfg1_box(200)
    d["tally_scale_log2"] = 62
    r = oracle.run(d)
    assert r["counts"]["overflow"] == 1
    d["tally_scale_log2"] = 32
    assert oracle.run(d)["counts"]["overflow"] == 0


# ---------------------------------------------------------------- elastic

def _xi(A):
    if A == 1.0:
        return 1.0
    return 1.0 + (A - 1) ** 2 / (2 * A) * math.log((A - 1) / (A + 1))


@pytest.mark.parametrize("A", [1.0, 1.5, 12.0, 238.0])
def test_elastic_kinematics(oracle, A):
    n = 4000
    xs = (np.arange(n) + 0.5) / n
    ratios, mus = [], []
    rng = np.random.default_rng(31)
    for k, xm in enumerate(xs):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        e, v = oracle.elastic(A, 1.0, xm, rng.random(), tuple(u))
        v = np.array(v)
        muc = 2 * xm - 1
        D = A * A + 2 * A * muc + 1
        mul = (1 + A * muc) / math.sqrt(D)
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        assert abs(float(np.dot(u, v)) - mul) < 1e-12
        ratios.append(e)
        mus.append(mul)
    # midpoint rule is exact for the linear E'/E; smooth mu_L converges fast
    assert abs(np.mean(ratios) - (A * A + 1) / (A + 1) ** 2) < 1e-12
    assert abs(np.mean(mus) - 2.0 / (3.0 * A)) < 1e-5


def test_elastic_along_axis_and_azimuth(oracle):
    # direction along z takes the special branch; azimuth must be uniform
    for w in (1.0, -1.0):
        _, v = oracle.elastic(12.0, 1.0, 0.3, 0.1, (0.0, 0.0, w))
        assert abs(np.linalg.norm(v) - 1) < 1e-12
    u = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    acc = np.zeros(3)
    n = 2000
    for k in range(n):
        _, v = oracle.elastic(5.0, 1.0, 0.7, (k + 0.5) / n, tuple(u))
        v = np.array(v)
        acc += v - np.dot(u, v) * u
    assert np.linalg.norm(acc / n) < 1e-6


def _ce_homogeneous(A, n_hist, n_bins=24, e0=1e6, e_min=1e-3):
    d = inputs.pincell_ce(n_ebins=10, n_histories=n_hist, grid_len=64, n_peaks=1)
    grid = np.geomspace(1e-6, 1e8, 64)
    d.update(n_species=1, grid_len=64, e_grid=grid, sig_a=np.zeros(64), sig_s=np.ones(64),
             awr=np.array([A]), density=np.array([1.0, 1.0]), e_min=e_min, e_source=e0,
             n_ebins=n_bins, e_edges=np.geomspace(e_min, e0, n_bins + 1))
    return d


@pytest.mark.parametrize("A", [1.0, 12.0])
def test_slowing_down_spectrum(oracle, A):
    d = _ce_homogeneous(A, n_hist=3000)
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * 2.0 ** -20 / per for b in range(batches)])
    du = math.log(d["e_edges"][1] / d["e_edges"][0])
    ref = du / (_xi(A) * 1.0)
    # bins well below the source (asymptotic region)
    far = slice(0, d["n_ebins"] - 6)
    mean = est.mean(axis=0)[far]
    se = est.std(axis=0, ddof=1)[far] / math.sqrt(batches)
    assert np.all(np.abs(mean - ref) < 4 * se), (mean, ref, se)
    r = oracle.run(d, 0, 200)
    assert r["counts"]["cutoffs"] == 200      # no absorption: all end at the cutoff


def test_ce_lookup_interpolation(oracle):
    d = inputs.pincell_ce(n_histories=1, grid_len=2000, n_peaks=20, jitter_grid=True)
    P = oracle.Problem(d)
    S, n = d["n_species"], d["grid_len"]
    grid = d["e_grid"].reshape(S, n)
    sa = d["sig_a"].reshape(S, n)
    ss = d["sig_s"].reshape(S, n)
    dens = d["density"].reshape(2, S)
    rng = np.random.default_rng(41)
    for e in np.concatenate([np.exp(rng.uniform(np.log(1e-6), np.log(3e7), 300)), grid[0, :5], grid[1, -5:]]):
        for m in (0, 1):
            st, a, s = oracle.ce_xs(P, m, e)
            tot = 0.0
            for k in range(S):
                ec = min(max(e, grid[k, 0]), grid[k, -1])
                ra = np.interp(ec, grid[k], sa[k])
                rs = np.interp(ec, grid[k], ss[k])
                assert abs(a[k] - ra) <= 1e-12 * max(abs(ra), 1e-300)
                assert abs(s[k] - rs) <= 1e-12 * max(abs(rs), 1e-300)
                tot += dens[m, k] * (ra + rs)
            assert abs(st - tot) <= 1e-12 * tot


def test_ce_run_counts(oracle):
    d = inputs.cfg3_pincell(n_ebins=1000, n_histories=300)
    r = oracle.run(d, digest=True)
    c = r["counts"]
    assert c["sourced"] == 300 == c["absorbs"] + c["cutoffs"] + c["killed"] + c["leaks"]
    assert c["leaks"] == 0                         # reflective everywhere
    assert int(r["tally"].sum()) == c["qsum"]


# ---------------------------------------------------------------- sources

def _cell_integral(edges, f, sub=24):
    """Midpoint-rule integral of f over every cell of a 3-D mesh."""
    nx, ny, nz = (len(e) - 1 for e in edges)
    out = np.zeros((nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                xs = [np.linspace(edges[a][c], edges[a][c + 1], sub + 1) for a, c in ((0, i), (1, j), (2, k))]
                mids = [(x[1:] + x[:-1]) / 2 for x in xs]
                X, Y, Z = np.meshgrid(*mids, indexing="ij")
                vol = np.prod([x[1] - x[0] for x in xs])
                out[k, j, i] = f(X, Y, Z).sum() * vol
    return out


def test_isotropic_point_source_uncollided(oracle):
    # near-void cube: every history flies straight out; the expected track
    # length in a cell is (1/4 pi) * integral over the cell of 1/r^2
    d = inputs.box_slabs_mg(size=(2.0, 2.0, 2.0), planes_x=[0.0, 2.0], slab_mat=[0], sigma_t=[[1e-9]],
                            sigma_s=[[0.0]], src_pos=[1.0, 1.0, 1.0], mesh_n=(4, 4, 4), n_histories=40000)
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * SCALE / per for b in range(batches)])
    edges = [d["mesh_x"], d["mesh_y"], d["mesh_z"]]
    ref = _cell_integral(edges, lambda X, Y, Z: 1.0 / (4 * math.pi * ((X - 1) ** 2 + (Y - 1) ** 2 + (Z - 1) ** 2)),
                         sub=40).ravel()
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / math.sqrt(batches)
    # the midpoint rule is poor in the 8 cells touching the source corner
    far = ref < 0.9 * ref.max()
    assert np.all(np.abs(mean[far] - ref[far]) < 4 * se[far] + 2e-3 * ref[far])


def test_box_source_uniform(oracle):
    # dense pure absorber: each history scores a short track at its birth
    # point, so the mesh tally follows the source density (uniform)
    d = inputs.box_slabs_mg(size=(2.0, 1.0, 1.0), planes_x=[0.0, 2.0], slab_mat=[0], sigma_t=[[200.0]],
                            sigma_s=[[0.0]], src_kind=inputs.SRC_BOX, src_lo=[0.0, 0.0, 0.0],
                            src_hi=[2.0, 1.0, 1.0], mesh_n=(4, 2, 2), n_histories=40000)
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * SCALE / per for b in range(batches)])
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / math.sqrt(batches)
    ref = (1.0 / 200.0) / 16 * np.ones(16)
    # a mean free path of 0.005 leaks a little across faces of 0.5 cells;
    # faces at the box walls lose a little to leakage
    assert np.all(np.abs(mean - ref) < 4 * se + 0.02 * ref)


def test_disc_source_uniform(oracle):
    d = inputs.lattice_mg(n_pins=1, pitch=2.0, radius=0.9, height=1.0, n_mat_pins=1, n_grp=1,
                          mesh_n=(4, 4, 1), n_histories=40000)
    d.update(sigma_t=np.array([500.0, 500.0]), sigma_s=np.array([0.0, 0.0]), src_kind=inputs.SRC_DISC,
             src_pos=np.array([1.0, 1.0, 0.5]), src_radius=0.9)
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * SCALE / per for b in range(batches)])
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / math.sqrt(batches)
    # independent: fraction of a uniform disc in each mesh cell
    rng = np.random.default_rng(5)
    r = 0.9 * np.sqrt(rng.random(2_000_000))
    ph = 2 * np.pi * rng.random(2_000_000)
    x, y = 1.0 + r * np.cos(ph), 1.0 + r * np.sin(ph)
    h, _, _ = np.histogram2d(y, x, bins=[d["mesh_y"], d["mesh_x"]])
    ref = (h / h.sum()).ravel() / 500.0
    assert np.all(np.abs(mean - ref) < 4 * se + 0.02 * ref + 1e-7)


def test_slowing_down_three_species(oracle):
    # species chosen in proportion to their macroscopic cross section:
    # flux per unit lethargy 1/sum_s(Sigma_s,s xi_s)
    d = _ce_homogeneous(1.0, n_hist=3000)
    grid = d["e_grid"][:64]
    d.update(n_species=3, e_grid=np.concatenate([grid, grid, grid]), sig_a=np.zeros(192),
             sig_s=np.concatenate([np.full(64, 0.2), np.full(64, 0.3), np.full(64, 0.5)]),
             awr=np.array([1.0, 12.0, 50.0]), density=np.ones(6))
    batches = 10
    per = d["n_histories"] // batches
    est = np.array([oracle.run(d, b * per, (b + 1) * per)["tally"] * 2.0 ** -20 / per for b in range(batches)])
    du = math.log(d["e_edges"][1] / d["e_edges"][0])
    ref = du / (0.2 * _xi(1.0) + 0.3 * _xi(12.0) + 0.5 * _xi(50.0))
    far = slice(0, d["n_ebins"] - 6)
    mean = est.mean(axis=0)[far]
    se = est.std(axis=0, ddof=1)[far] / math.sqrt(batches)
    assert np.all(np.abs(mean - ref) < 4 * se), (mean, ref, se)
