"""Seeded synthetic problem generators.

This module produces plain problem descriptions (numpy arrays and scalars)
for the five workloads the transport hot path is exercised on.  It holds
data only: geometry planes, cross-section tables, transfer CDFs, mesh and
energy-bin edges, source definitions and seeds.  None of the transport
arithmetic lives here; both the CPU oracle and the GPU binding read the
same dictionaries and marshal them into their own structures.

The paper (Sec. 4) runs the 3-D C5G7 benchmark and a continuous-energy
infinite pin cell; neither data set is available, so ``lattice_mg`` and
``pincell_ce`` are synthetic stand-ins with the same structure (a 17x17
pin lattice with 7 groups; a single reflected fuel pin with pointwise
continuous-energy tables).

All draws use ``numpy.random.Generator(Philox(seed))`` so every problem is
reproducible from its integer data seed.
"""
from __future__ import annotations

import numpy as np

# geometry kinds
GEOM_BOX = 0        # box cut into x-slabs
GEOM_LATTICE = 1    # rectangular pin lattice (a 1x1 lattice is a pin cell)
# energy treatment
ENERGY_MG = 0
ENERGY_CE = 1
# boundary conditions per face, order x-, x+, y-, y+, z-, z+
BC_VACUUM = 0
BC_REFLECT = 1
# source kinds
SRC_POINT = 0       # fixed point
SRC_BOX = 1         # uniform in an axis-aligned box
SRC_DISC = 2        # uniform in a disc (cylinder cross-section) at fixed z
# tally kinds
TALLY_MESH = 0
TALLY_ENERGY = 1

DATA_SEED_BASE = 1000
TRANSPORT_SEED_BASE = 20250427
DEFAULT_MAX_STEPS = 1_000_000


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _transfer_cdf(rng, n_mat: int, n_grp: int, downscatter_only_2g: bool = False) -> np.ndarray:
    """Row-stochastic group-transfer matrices as cumulative rows.

    Rows are the *from* group.  Mass concentrates on g' >= g (downscatter):
    Dirichlet weights alpha=1 for g' >= g and 0.05 for g' < g.  The last
    entry of each row is set to exactly 1.0.
    """
    cdf = np.zeros((n_mat, n_grp, n_grp))
    for m in range(n_mat):
        for g in range(n_grp):
            if downscatter_only_2g:
                p = rng.dirichlet([1.0, 1.0]) if g == 0 else np.array([0.0, 1.0])
            else:
                alpha = np.where(np.arange(n_grp) >= g, 1.0, 0.05)
                p = rng.dirichlet(alpha)
            c = np.cumsum(p)
            c = np.minimum(c, 1.0)
            c[-1] = 1.0
            cdf[m, g] = c
    return cdf


def _mg_tables(rng, n_mat: int, n_grp: int, c_lo: float, c_hi: float):
    sigma_t = rng.uniform(0.2, 2.0, size=(n_mat, n_grp))
    c = rng.uniform(c_lo, c_hi, size=(n_mat, n_grp))
    sigma_s = sigma_t * c
    return sigma_t, sigma_s


def _base(n_histories: int, seed: int, problem_id: int) -> dict:
    return dict(
        n_histories=int(n_histories),
        seed=int(seed),
        problem_id=int(problem_id),
        max_steps=DEFAULT_MAX_STEPS,
        # unused-by-default fields, filled so every description has them
        n_slabs=0, slab_planes=_f64([0.0]), slab_mat=_i32([0]),
        nx=0, ny=0, xplanes=_f64([0.0]), yplanes=_f64([0.0]), cx=_f64([0.0]), cy=_f64([0.0]),
        radius=0.0, pin_mat=_i32([0]), mod_mat=0,
        n_mat=0, n_grp=0, sigma_t=_f64([0.0]), sigma_s=_f64([0.0]), cdf=_f64([0.0]),
        n_species=0, grid_len=0, e_grid=_f64([0.0]), sig_a=_f64([0.0]), sig_s=_f64([0.0]),
        awr=_f64([0.0]), density=_f64([0.0]), e_min=0.0, e_source=0.0,
        src_kind=SRC_POINT, src_pos=_f64([0, 0, 0]), src_lo=_f64([0, 0, 0]), src_hi=_f64([0, 0, 0]),
        src_radius=0.0, src_isotropic=1, src_dir=_f64([0, 0, 1]), src_group=0,
        tally_kind=TALLY_MESH, mesh_n=_i32([1, 1, 1]), mesh_x=_f64([0, 1]), mesh_y=_f64([0, 1]),
        mesh_z=_f64([0, 1]), n_ebins=0, e_edges=_f64([0.0, 1.0]), tally_scale_log2=32,
        n_tbins=0, t_max=0.0, speed=_f64([1.0]), speed_coef=0.0,
        implicit_capture=0, w_cutoff=0.0, w_survival=0.0,
    )


def box_slabs_mg(*, size=(10.0, 10.0, 10.0), planes_x=None, slab_mat=None, bc=None,
                 sigma_t=None, sigma_s=None, cdf=None, src_kind=SRC_POINT, src_pos=None,
                 src_lo=None, src_hi=None, src_isotropic=1, src_dir=(1.0, 0.0, 0.0),
                 src_group=0, mesh_n=(10, 10, 10), n_histories=10_000, seed=TRANSPORT_SEED_BASE,
                 problem_id=0, tally_scale_log2=32) -> dict:
    """A box [0,Lx]x[0,Ly]x[0,Lz] cut into x-slabs, multigroup.

    Explicit cross-section arrays let tests build closed-form cases
    (one material, one group, reflective faces, a beam source ...)."""
    lx, ly, lz = size
    if planes_x is None:
        planes_x = [0.0, lx]
    planes_x = _f64(planes_x)
    ns = len(planes_x) - 1
    if slab_mat is None:
        slab_mat = list(range(ns))
    sigma_t = _f64(sigma_t)
    sigma_s = _f64(sigma_s)
    n_mat, n_grp = sigma_t.shape
    if cdf is None:
        assert n_grp == 1
        cdf = np.ones((n_mat, 1, 1))
    d = _base(n_histories, seed, problem_id)
    d.update(
        geometry=GEOM_BOX, box_lo=_f64([0.0, 0.0, 0.0]), box_hi=_f64([lx, ly, lz]),
        bc=_i32(bc if bc is not None else [BC_VACUUM] * 6),
        n_slabs=ns, slab_planes=planes_x, slab_mat=_i32(slab_mat),
        energy_mode=ENERGY_MG, n_mat=n_mat, n_grp=n_grp,
        sigma_t=_f64(sigma_t.ravel()), sigma_s=_f64(sigma_s.ravel()), cdf=_f64(np.asarray(cdf).ravel()),
        src_kind=src_kind, src_pos=_f64(src_pos if src_pos is not None else [lx / 2, ly / 2, lz / 2]),
        src_lo=_f64(src_lo if src_lo is not None else [0, 0, 0]),
        src_hi=_f64(src_hi if src_hi is not None else [lx, ly, lz]),
        src_isotropic=int(src_isotropic), src_dir=_f64(src_dir), src_group=int(src_group),
        tally_kind=TALLY_MESH, mesh_n=_i32(mesh_n),
        mesh_x=_f64(np.linspace(0.0, lx, mesh_n[0] + 1)),
        mesh_y=_f64(np.linspace(0.0, ly, mesh_n[1] + 1)),
        mesh_z=_f64(np.linspace(0.0, lz, mesh_n[2] + 1)),
        tally_scale_log2=int(tally_scale_log2),
    )
    return d


def cfg1_box(n_histories: int = 10_000) -> dict:
    """Plain multigroup fixed source: 10 cm vacuum box, two materials split at
    x = 5, two groups with downscatter-only transfer, isotropic point source at
    the centre in the fast group, 10x10x10 mesh track-length tally."""
    rng = _rng(DATA_SEED_BASE + 1)
    st, ss = _mg_tables(rng, 2, 2, 0.3, 0.9)
    cdf = _transfer_cdf(rng, 2, 2, downscatter_only_2g=True)
    return box_slabs_mg(size=(10.0, 10.0, 10.0), planes_x=[0.0, 5.0, 10.0], slab_mat=[0, 1],
                        sigma_t=st, sigma_s=ss, cdf=cdf, src_pos=[5.0, 5.0, 5.0],
                        mesh_n=(10, 10, 10), n_histories=n_histories,
                        seed=TRANSPORT_SEED_BASE + 1)


def lattice_mg(*, n_pins: int = 17, pitch: float = 1.26, radius: float = 0.54, height: float = 20.0,
               n_mat_pins: int = 6, n_grp: int = 7, mesh_n=(51, 51, 20), n_histories: int = 1_000_000,
               data_seed: int = DATA_SEED_BASE + 2, seed: int = TRANSPORT_SEED_BASE + 2) -> dict:
    """Multigroup pin lattice: n_pins x n_pins cylinders (full height) in a
    reflective box, pin materials 0..n_mat_pins-1 drawn per pin, moderator is
    material n_mat_pins, uniform volumetric source in group 0."""
    rng = _rng(data_seed)
    n_mat = n_mat_pins + 1
    st, ss = _mg_tables(rng, n_mat, n_grp, 0.3, 0.95)
    cdf = _transfer_cdf(rng, n_mat, n_grp)
    pin_mat = rng.integers(0, n_mat_pins, size=n_pins * n_pins)
    side = n_pins * pitch
    planes = np.arange(n_pins + 1) * pitch
    centres = (np.arange(n_pins) + 0.5) * pitch
    d = _base(n_histories, seed, 0)
    d.update(
        geometry=GEOM_LATTICE, box_lo=_f64([0.0, 0.0, 0.0]), box_hi=_f64([planes[-1], planes[-1], height]),
        bc=_i32([BC_REFLECT] * 6),
        nx=n_pins, ny=n_pins, xplanes=_f64(planes), yplanes=_f64(planes), cx=_f64(centres), cy=_f64(centres),
        radius=float(radius), pin_mat=_i32(pin_mat), mod_mat=n_mat_pins,
        energy_mode=ENERGY_MG, n_mat=n_mat, n_grp=n_grp,
        sigma_t=_f64(st.ravel()), sigma_s=_f64(ss.ravel()), cdf=_f64(cdf.ravel()),
        src_kind=SRC_BOX, src_lo=_f64([0.0, 0.0, 0.0]), src_hi=_f64([planes[-1], planes[-1], height]),
        src_group=0,
        tally_kind=TALLY_MESH, mesh_n=_i32(mesh_n),
        mesh_x=_f64(np.linspace(0.0, planes[-1], mesh_n[0] + 1)),
        mesh_y=_f64(np.linspace(0.0, planes[-1], mesh_n[1] + 1)),
        mesh_z=_f64(np.linspace(0.0, height, mesh_n[2] + 1)),
        tally_scale_log2=32,
    )
    del side
    return d


def cfg2_lattice(n_histories: int = 1_000_000) -> dict:
    return lattice_mg(n_histories=n_histories)


def _ce_species(rng, n_species: int, grid_len: int, e_lo: float, e_hi: float, n_peaks: int):
    """Pointwise tables: 1/v absorption plus Breit-Wigner-shaped peaks;
    constant elastic scattering; target mass ratio A ~ U[1, 240]."""
    grid = np.geomspace(e_lo, e_hi, grid_len)
    e_grid = np.empty((n_species, grid_len))
    sig_a = np.empty((n_species, grid_len))
    sig_s = np.empty((n_species, grid_len))
    awr = rng.uniform(1.0, 240.0, size=n_species)
    for s in range(n_species):
        a_s = rng.uniform(0.1, 1.0)
        b_s = rng.uniform(2.0, 20.0)
        ek = np.exp(rng.uniform(np.log(1.0), np.log(1e5), size=n_peaks))
        gk = ek * 10.0 ** rng.uniform(-4.0, -2.0, size=n_peaks)
        hk = np.exp(rng.uniform(np.log(10.0), np.log(1e4), size=n_peaks))
        sa = a_s / np.sqrt(grid)
        for k in range(n_peaks):
            half = gk[k] / 2.0
            sa = sa + hk[k] * half * half / ((grid - ek[k]) ** 2 + half * half)
        e_grid[s] = grid
        sig_a[s] = sa
        sig_s[s] = b_s
    return e_grid, sig_a, sig_s, awr


def pincell_ce(*, n_ebins: int = 100, n_histories: int = 1_000_000, grid_len: int = 100_000,
               n_peaks: int = 200, jitter_grid: bool = False, data_seed: int = DATA_SEED_BASE + 3,
               seed: int = TRANSPORT_SEED_BASE + 3) -> dict:
    """Continuous-energy pin cell: a 1x1 lattice (fuel cylinder r=0.54 in a
    1.26 cm reflective square, infinite in z), three species, energy-binned
    track-length tally; uniform source in the fuel at 1.4e7."""
    rng = _rng(data_seed)
    n_species = 3
    e_lo, e_hi = 1e-5, 2e7
    e_grid, sig_a, sig_s, awr = _ce_species(rng, n_species, grid_len, e_lo, e_hi, n_peaks)
    if jitter_grid:
        # arbitrary sorted grids: perturb interior points per species
        for s in range(n_species):
            g = np.log(e_grid[s])
            step = (g[-1] - g[0]) / (grid_len - 1)
            g[1:-1] += rng.uniform(-0.45, 0.45, size=grid_len - 2) * step
            e_grid[s] = np.exp(g)
            e_grid[s, 0], e_grid[s, -1] = e_lo, e_hi
    light = int(np.argmin(awr))
    density = np.zeros((2, n_species))      # material 0 fuel, 1 moderator
    for s in range(n_species):
        if s == light:
            density[1, s] = rng.uniform(0.02, 0.07)
        else:
            density[0, s] = rng.uniform(0.01, 0.05)
    half = 0.63
    d = _base(n_histories, seed, 0)
    d.update(
        geometry=GEOM_LATTICE, box_lo=_f64([-half, -half, -np.inf]), box_hi=_f64([half, half, np.inf]),
        bc=_i32([BC_REFLECT] * 6),
        nx=1, ny=1, xplanes=_f64([-half, half]), yplanes=_f64([-half, half]), cx=_f64([0.0]), cy=_f64([0.0]),
        radius=0.54, pin_mat=_i32([0]), mod_mat=1,
        energy_mode=ENERGY_CE, n_mat=2, n_grp=1,
        n_species=n_species, grid_len=grid_len, e_grid=_f64(e_grid.ravel()), sig_a=_f64(sig_a.ravel()),
        sig_s=_f64(sig_s.ravel()), awr=_f64(awr), density=_f64(density.ravel()),
        e_min=1e-5, e_source=1.4e7,
        src_kind=SRC_DISC, src_pos=_f64([0.0, 0.0, 0.0]), src_radius=0.54,
        tally_kind=TALLY_ENERGY, n_ebins=int(n_ebins), e_edges=_f64(np.geomspace(e_lo, e_hi, n_ebins + 1)),
        tally_scale_log2=20,
    )
    return d


def cfg3_pincell(n_ebins: int = 100, n_histories: int = 1_000_000) -> dict:
    return pincell_ce(n_ebins=n_ebins, n_histories=n_histories)


def target_tally(t_hat: np.ndarray, data_seed: int = DATA_SEED_BASE + 4) -> np.ndarray:
    """Seeded target for the differentiable lattice run:
    tau_b = T_b * (0.9 + 0.2 * xi_b)."""
    rng = _rng(data_seed)
    return t_hat * (0.9 + 0.2 * rng.random(t_hat.shape))


def cfg4_lattice_grad(n_histories: int = 1_000_000) -> dict:
    return lattice_mg(n_histories=n_histories)


def cfg5_batch(n_problems: int = 256, hist_scale: float = 1.0, data_seed: int = DATA_SEED_BASE + 5,
               seed: int = TRANSPORT_SEED_BASE + 5) -> list:
    """Independent fixed-source box or slab problems of uneven size.

    Histories ~ round(10**(3 + 2 xi)) (times ``hist_scale``), 1-8 materials as
    equal-width x-slabs, 1-16 groups, mesh n^3 with n in 8..32.  "Box" has
    vacuum faces everywhere; "slab" has vacuum x faces and reflective y/z."""
    rng = _rng(data_seed)
    probs = []
    for i in range(n_problems):
        n_hist = int(round(10.0 ** (3.0 + 2.0 * rng.random()) * hist_scale))
        n_hist = max(n_hist, 1)
        n_mat = int(rng.integers(1, 9))
        n_grp = int(rng.integers(1, 17))
        n_mesh = int(rng.integers(8, 33))
        side = float(rng.uniform(5.0, 20.0))
        slab = bool(rng.random() < 0.5)
        st, ss = _mg_tables(rng, n_mat, n_grp, 0.3, 0.95)
        cdf = _transfer_cdf(rng, n_mat, n_grp)
        planes = np.linspace(0.0, side, n_mat + 1)
        bc = [BC_VACUUM, BC_VACUUM] + ([BC_REFLECT] * 4 if slab else [BC_VACUUM] * 4)
        probs.append(box_slabs_mg(size=(side, side, side), planes_x=planes, slab_mat=list(range(n_mat)), bc=bc,
                                  sigma_t=st, sigma_s=ss, cdf=cdf, src_pos=[side / 2] * 3,
                                  mesh_n=(n_mesh,) * 3, n_histories=n_hist, seed=seed, problem_id=i))
    return probs


def n_bins(d: dict) -> int:
    """Number of tally bins of a problem description (times the time bins)."""
    if d["tally_kind"] == TALLY_MESH:
        nb = int(np.prod(d["mesh_n"])) * (int(d["n_grp"]) if d["energy_mode"] == ENERGY_MG else 1)
    else:
        nb = int(d["n_ebins"])
    return nb * max(1, int(d.get("n_tbins", 0)))


def with_time_bins(d: dict, n_tbins: int, t_max: float, speed=None, speed_coef: float = 0.0) -> dict:
    """A copy of problem d with a time-binned tally: n_tbins equal bins over
    [0, t_max); a flight that would reach t_max ends there.  Speeds: one per
    group (multigroup, default 10^(-g/2)) or speed_coef * sqrt(E) (continuous
    energy)."""
    d = dict(d)
    d["n_tbins"] = int(n_tbins)
    d["t_max"] = float(t_max)
    if d["energy_mode"] == ENERGY_MG:
        g = np.arange(int(d["n_grp"]), dtype=np.float64)
        d["speed"] = _f64(speed if speed is not None else 10.0 ** (-0.5 * g))
    d["speed_coef"] = float(speed_coef)
    return d


def with_implicit_capture(d: dict, w_cutoff: float = 0.25, w_survival: float = 0.5) -> dict:
    """A copy of problem d with non-analog weights: implicit capture (every
    collision scatters, the weight carries the absorption) and weight roulette
    below w_cutoff to weight w_survival."""
    d = dict(d)
    d["implicit_capture"] = 1
    d["w_cutoff"] = float(w_cutoff)
    d["w_survival"] = float(w_survival)
    return d


def with_weight_windows(d: dict, n=(4, 4, 4), lo=None, lo_range=(0.05, 0.5), ratio: float = 4.0,
                        surv: float = 2.0, max_split: int = 8, data_seed: int = DATA_SEED_BASE + 7) -> dict:
    """A copy of problem d with spatial weight windows: a uniform grid of n
    cells over the box, lower bounds lo (one per cell, [iz][iy][ix]) or drawn
    log-uniform in lo_range; upper bound ratio * lo, survival weight surv * lo,
    at most max_split copies per split.  Data only."""
    d = dict(d)
    n = tuple(int(v) for v in n)
    if lo is None:
        rng = _rng(data_seed)
        lo = np.exp(rng.uniform(np.log(lo_range[0]), np.log(lo_range[1]), size=int(np.prod(n))))
    d["ww_n"] = _i32(n)
    d["ww_lo"] = _f64(np.asarray(lo, np.float64).ravel())
    d["ww_ratio"] = float(ratio)
    d["ww_surv"] = float(surv)
    d["ww_max_split"] = int(max_split)
    return d


def with_fission(d: dict, fissile=None, sigma_f=None, nu=None, chi=None,
                 data_seed: int = DATA_SEED_BASE + 6) -> dict:
    """A copy of multigroup problem d with fission data for k-eigenvalue runs.

    Defaults (a synthetic stand-in for fuel data): the `fissile` materials
    (default: every material but the moderator of a lattice, every material of
    a box) get Sigma_f = f Sigma_a with f ~ U[0.3, 0.7] per (material, group)
    and nu ~ U[2.3, 2.7]; the others none.  chi (the cumulative fission
    spectrum, per material) puts the neutrons into the fastest groups with
    weights proportional to 0.6^g over the first min(3, G) groups."""
    d = dict(d)
    assert d["energy_mode"] == ENERGY_MG
    n_mat, n_grp = int(d["n_mat"]), int(d["n_grp"])
    rng = np.random.default_rng(data_seed)
    st = np.asarray(d["sigma_t"], np.float64).reshape(n_mat, n_grp)
    ss = np.asarray(d["sigma_s"], np.float64).reshape(n_mat, n_grp)
    if fissile is None:
        fissile = [m for m in range(n_mat) if not (d["geometry"] == GEOM_LATTICE and m == d["mod_mat"])]
    if sigma_f is None:
        sigma_f = np.zeros((n_mat, n_grp))
        for m in fissile:
            sigma_f[m] = rng.uniform(0.3, 0.7, n_grp) * (st[m] - ss[m])
    if nu is None:
        nu = np.zeros((n_mat, n_grp))
        for m in fissile:
            nu[m] = rng.uniform(2.3, 2.7, n_grp)
    if chi is None:
        w = np.zeros(n_grp)
        k = min(3, n_grp)
        w[:k] = 0.6 ** np.arange(k)
        c = np.cumsum(w / w.sum())
        c[-1] = 1.0
        chi = np.tile(c, (n_mat, 1))
    d["sigma_f"] = _f64(np.asarray(sigma_f, np.float64).reshape(n_mat * n_grp))
    d["nu"] = _f64(np.asarray(nu, np.float64).reshape(n_mat * n_grp))
    d["chi"] = _f64(np.asarray(chi, np.float64).reshape(n_mat * n_grp))
    return d


def config(k: int, **kw):
    """Workload k in 1..5 (see module docstring)."""
    return {1: cfg1_box, 2: cfg2_lattice, 3: cfg3_pincell, 4: cfg4_lattice_grad, 5: cfg5_batch}[k](**kw)
