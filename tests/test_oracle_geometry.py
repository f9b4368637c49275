"""Pins of the oracle's geometry and mesh walk.

Hand-computed distances, Cauchy's mean-chord theorem (mean chord of a convex
body under cosine-law surface incidence = 4V/S) for a cube and a finite
cylinder, an independent quadratic for the cylinder, and brute-force
segment/cell clipping for the track-length mesh walk.
"""
import math

import numpy as np
import pytest

from paper_2506_00263_amd import inputs


def _box(planes=(0.0, 10.0), size=(10.0, 10.0, 10.0), mesh_n=(10, 10, 10)):
    ns = len(planes) - 1
    return inputs.box_slabs_mg(size=size, planes_x=list(planes), slab_mat=list(range(ns)),
                               sigma_t=np.ones((ns, 1)), sigma_s=np.zeros((ns, 1)), mesh_n=mesh_n)


def _pin(radius=1.0, height=3.0, pitch=None):
    pitch = pitch if pitch is not None else 2 * radius + 1.0
    d = inputs.lattice_mg(n_pins=1, pitch=pitch, radius=radius, height=height, n_mat_pins=1, n_grp=1,
                          mesh_n=(1, 1, 1))
    # centre the single pin at the origin
    h = pitch / 2
    d.update(xplanes=np.array([-h, h]), yplanes=np.array([-h, h]), cx=np.array([0.0]), cy=np.array([0.0]),
             box_lo=np.array([-h, -h, 0.0]), box_hi=np.array([h, h, height]),
             mesh_x=np.array([-h, h]), mesh_y=np.array([-h, h]), mesh_z=np.array([0.0, height]))
    return d


def test_box_hand_distances(oracle):
    P = oracle.Problem(_box(planes=(0.0, 5.0, 10.0)))
    c = oracle.locate(P, (5.0, 5.0, 5.0), (1.0, 0.0, 0.0))
    assert c[0] == 1
    assert oracle.distance(P, (5.0, 5.0, 5.0), (1.0, 0.0, 0.0), c) == (5.0, 0)
    c = oracle.locate(P, (5.0, 5.0, 5.0), (-1.0, 0.0, 0.0))
    assert c[0] == 0                                  # on the interface moving -x
    assert oracle.distance(P, (5.0, 5.0, 5.0), (-1.0, 0.0, 0.0), c) == (5.0, 0)
    assert oracle.distance(P, (2.0, 5.0, 5.0), (1.0, 0.0, 0.0), (0, 0, 0)) == (3.0, 0)
    assert oracle.distance(P, (2.0, 5.0, 5.0), (0.0, 1.0, 0.0), (0, 0, 0)) == (5.0, 1)
    assert oracle.distance(P, (2.0, 5.0, 4.0), (0.0, 0.0, -1.0), (0, 0, 0)) == (4.0, 2)
    s = 1 / math.sqrt(2)
    d, surf = oracle.distance(P, (7.0, 7.0, 5.0), (s, s, 0.0), (1, 0, 0))
    assert surf == 0 and abs(d - 3 * math.sqrt(2)) < 1e-14     # tie x/y: x wins


def test_lattice_hand_distances(oracle):
    d = inputs.lattice_mg(n_histories=1)
    P = oracle.Problem(d)
    cx, cy, r = d["cx"][3], d["cy"][5], d["radius"]
    cell = oracle.locate(P, (cx, cy, 10.0), (1.0, 0.0, 0.0))
    assert cell == (3, 5, 1)
    dist, surf = oracle.distance(P, (cx, cy, 10.0), (1.0, 0.0, 0.0), cell)
    assert surf == 3 and abs(dist - r) < 1e-15
    # outside, aimed at the pin along -x from 0.6 right of the centre
    cell = oracle.locate(P, (cx + 0.6, cy, 10.0), (-1.0, 0.0, 0.0))
    assert cell == (3, 5, 0)
    dist, surf = oracle.distance(P, (cx + 0.6, cy, 10.0), (-1.0, 0.0, 0.0), cell)
    assert surf == 3 and abs(dist - 0.06) < 1e-14
    # outside, moving away: the cell plane
    dist, surf = oracle.distance(P, (cx + 0.6, cy, 10.0), (1.0, 0.0, 0.0), cell)
    assert surf == 0 and abs(dist - (d["xplanes"][4] - cx - 0.6)) < 1e-14
    # up the axis inside a pin: the top face
    cell = oracle.locate(P, (cx, cy, 10.0), (0.0, 0.0, 1.0))
    assert oracle.distance(P, (cx, cy, 10.0), (0.0, 0.0, 1.0), cell) == (10.0, 2)


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def test_cylinder_distance_against_quadratic(oracle):
    rng = np.random.default_rng(11)
    d = _pin(radius=1.0, height=1e6, pitch=10.0)
    d["box_lo"][2], d["box_hi"][2] = -1e6, 1e6
    d["mesh_z"] = np.array([-1e6, 1e6])
    P = oracle.Problem(d)
    dirs = _unit(rng, 4000)
    pts = rng.uniform(-4.5, 4.5, size=(4000, 3))
    pts[:, 2] = 0.0
    checked = 0
    for p, u in zip(pts, dirs):
        cell = oracle.locate(P, p, u)
        dist, surf = oracle.distance(P, p, u, cell)
        # independent: solve |p + t u|_xy = r in extended precision
        x, y = np.longdouble(p[0]), np.longdouble(p[1])
        a = np.longdouble(u[0]) ** 2 + np.longdouble(u[1]) ** 2
        b = 2 * (x * np.longdouble(u[0]) + y * np.longdouble(u[1]))
        c = x * x + y * y - 1
        disc = b * b - 4 * a * c
        tc = np.inf
        if disc >= 0 and a > 0:
            r1 = (-b - np.sqrt(disc)) / (2 * a)
            r2 = (-b + np.sqrt(disc)) / (2 * a)
            cand = [t for t in (r1, r2) if t > 0]
            if cell[2] == 1:
                tc = float(r2)
            elif cand:
                tc = float(min(cand))
        planes = []
        if cell[2] == 0:
            for k in range(2):
                if u[k] > 0:
                    planes.append((5.0 - p[k]) / u[k])
                elif u[k] < 0:
                    planes.append((-5.0 - p[k]) / u[k])
        tp = min(planes) if planes else np.inf
        ref = min(tc, tp)
        if abs(tc - tp) < 1e-9:
            continue
        assert abs(dist - ref) <= 1e-12 * max(1.0, ref), (p, u, cell, dist, ref)
        assert (surf == 3) == (tc < tp)
        checked += 1
    assert checked > 3500


def _cosine_dir(rng, normal, t1, t2):
    mu = math.sqrt(rng.random())
    phi = 2 * math.pi * rng.random()
    st = math.sqrt(1 - mu * mu)
    return mu * normal + st * (math.cos(phi) * t1 + math.sin(phi) * t2)


def test_mean_chord_cube(oracle):
    rng = np.random.default_rng(12)
    a = 3.0
    P = oracle.Problem(_box(planes=(0.0, a), size=(a, a, a), mesh_n=(1, 1, 1)))
    n = 20000
    chords = np.empty(n)
    eye = np.eye(3)
    for k in range(n):
        face = rng.integers(0, 6)
        ax, side = face >> 1, face & 1
        pos = rng.uniform(0, a, 3)
        pos[ax] = a * side
        normal = eye[ax] * (1.0 if side == 0 else -1.0)
        t1, t2 = eye[(ax + 1) % 3], eye[(ax + 2) % 3]
        u = _cosine_dir(rng, normal, t1, t2)
        chords[k] = oracle.distance(P, pos, u, (0, 0, 0))[0]
    mean, se = chords.mean(), chords.std() / math.sqrt(n)
    assert abs(mean - 2 * a / 3) < 4 * se, (mean, 2 * a / 3, se)


def test_mean_chord_finite_cylinder(oracle):
    rng = np.random.default_rng(13)
    R, H = 1.0, 3.0
    P = oracle.Problem(_pin(radius=R, height=H))
    n = 20000
    chords = np.empty(n)
    lat, cap = 2 * math.pi * R * H, 2 * math.pi * R * R
    for k in range(n):
        if rng.random() < lat / (lat + cap):
            phi = 2 * math.pi * rng.random()
            pos = np.array([R * math.cos(phi), R * math.sin(phi), H * rng.random()])
            normal = np.array([-math.cos(phi), -math.sin(phi), 0.0])
            t1 = np.array([0.0, 0.0, 1.0])
            t2 = np.cross(normal, t1)
        else:
            rr, phi = R * math.sqrt(rng.random()), 2 * math.pi * rng.random()
            top = rng.random() < 0.5
            pos = np.array([rr * math.cos(phi), rr * math.sin(phi), H if top else 0.0])
            normal = np.array([0.0, 0.0, -1.0 if top else 1.0])
            t1, t2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
        u = _cosine_dir(rng, normal, t1, t2)
        chords[k] = oracle.distance(P, pos, u, (0, 0, 1))[0]
    mean, se = chords.mean(), chords.std() / math.sqrt(n)
    ref = 2 * R * H / (R + H)
    assert abs(mean - ref) < 4 * se, (mean, ref, se)


def _clip_lengths(edges, x0, u, d, n, g, n_grp):
    """Brute force: length of the segment inside every mesh cell by slab
    clipping (independent of the walk's incremental crossing logic)."""
    out = np.zeros(n_grp * n[0] * n[1] * n[2])
    spans = []
    for ax in range(3):
        s = []
        for i in range(n[ax]):
            lo_e, hi_e = edges[ax][i], edges[ax][i + 1]
            if u[ax] != 0.0:
                ta, tb = (lo_e - x0[ax]) / u[ax], (hi_e - x0[ax]) / u[ax]
                s.append((min(ta, tb), max(ta, tb)))
            else:
                s.append((-np.inf, np.inf) if lo_e <= x0[ax] < hi_e else (1.0, 0.0))
        spans.append(s)
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                lo = max(0.0, spans[0][i][0], spans[1][j][0], spans[2][k][0])
                hi = min(d, spans[0][i][1], spans[1][j][1], spans[2][k][1])
                if hi > lo:
                    out[((g * n[2] + k) * n[1] + j) * n[0] + i] = hi - lo
    return out


def test_mesh_walk_brute_force(oracle):
    rng = np.random.default_rng(14)
    d = _box(planes=(0.0, 4.0), size=(4.0, 3.0, 2.0), mesh_n=(5, 4, 3))
    d["n_grp"] = 2
    d["sigma_t"] = np.ones(2)
    d["sigma_s"] = np.zeros(2)
    d["cdf"] = np.ones(4)
    P = oracle.Problem(d)
    edges = [d["mesh_x"], d["mesh_y"], d["mesh_z"]]
    n = [5, 4, 3]
    for trial in range(500):
        x0 = rng.uniform([0, 0, 0], [4, 3, 2])
        u = _unit(rng, 1)[0]
        if trial % 10 == 0:
            u[rng.integers(0, 3)] = 0.0     # axis-parallel cases
            u /= np.linalg.norm(u)
        # length up to the box boundary at most
        tmax = min([((4, 3, 2)[a] - x0[a]) / u[a] if u[a] > 0 else (-x0[a] / u[a] if u[a] < 0 else np.inf)
                    for a in range(3)])
        dist = tmax * rng.uniform(0.05, 1.0)
        g = int(rng.integers(0, 2))
        got = oracle.tally_segment(P, x0, u, dist, g)
        ref = _clip_lengths(edges, x0, u, dist, n, g, 2)
        assert np.allclose(got, ref, rtol=0, atol=1e-12), (x0, u, dist)
        assert abs(got.sum() - dist) < 1e-12


@pytest.mark.parametrize("start_on_edge", [True, False])
def test_mesh_walk_starting_on_edges(oracle, start_on_edge):
    d = _box(planes=(0.0, 10.0), mesh_n=(10, 10, 10))
    P = oracle.Problem(d)
    x0 = (5.0, 5.0, 5.0) if start_on_edge else (5.5, 5.5, 5.5)
    for u in [(-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.0, 0.0, 1.0)]:
        got = oracle.tally_segment(P, x0, u, 2.5)
        ref = _clip_lengths([d["mesh_x"], d["mesh_y"], d["mesh_z"]], x0, u, 2.5, [10, 10, 10], 0, 1)
        if start_on_edge:
            # on a vertex the brute force owns the zero-width touching cells
            # differently; the walk assigns by the direction of travel
            assert abs(got.sum() - 2.5) < 1e-15 and np.count_nonzero(got) == 3
        else:
            assert np.allclose(got, ref, atol=1e-14)
