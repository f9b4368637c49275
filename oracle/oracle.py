"""ctypes wrapper of the CPU oracle -- TEST INFRASTRUCTURE.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  It marshals a problem description produced by
``paper_2506_00263_amd.inputs`` into the oracle's own C structure and runs
histories on the host.  Independent history ranges can run in parallel
threads (ctypes releases the GIL); their integer tallies are summed, which
is exact, so the thread count never changes a result.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "oracle.h")]
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (contraction off, no fast math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SOURCES[0], "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcProblem(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("bc", C.c_int32 * 6), ("n_slabs", C.c_int32), ("slab_planes", C.c_void_p), ("slab_mat", C.c_void_p),
        ("nx", C.c_int32), ("ny", C.c_int32), ("xplanes", C.c_void_p), ("yplanes", C.c_void_p),
        ("cx", C.c_void_p), ("cy", C.c_void_p), ("radius", C.c_double), ("pin_mat", C.c_void_p),
        ("mod_mat", C.c_int32), ("energy_mode", C.c_int32), ("n_mat", C.c_int32), ("n_grp", C.c_int32),
        ("sigma_t", C.c_void_p), ("sigma_s", C.c_void_p), ("cdf", C.c_void_p),
        ("n_species", C.c_int32), ("grid_len", C.c_int32), ("e_grid", C.c_void_p), ("sig_a", C.c_void_p),
        ("sig_s", C.c_void_p), ("awr", C.c_void_p), ("density", C.c_void_p), ("e_min", C.c_double),
        ("e_source", C.c_double), ("src_kind", C.c_int32), ("src_isotropic", C.c_int32),
        ("src_group", C.c_int32), ("tally_kind", C.c_int32), ("src_pos", C.c_double * 3),
        ("src_lo", C.c_double * 3), ("src_hi", C.c_double * 3), ("src_dir", C.c_double * 3),
        ("src_radius", C.c_double), ("mesh_n", C.c_int32 * 3), ("mesh_x", C.c_void_p),
        ("mesh_y", C.c_void_p), ("mesh_z", C.c_void_p), ("n_ebins", C.c_int32), ("e_edges", C.c_void_p),
        ("tally_scale_log2", C.c_int32), ("problem_id", C.c_uint32), ("seed", C.c_uint64),
        ("max_steps", C.c_int64), ("n_tbins", C.c_int32), ("t_max", C.c_double), ("speed", C.c_void_p),
        ("speed_coef", C.c_double), ("sigma_f", C.c_void_p), ("nu", C.c_void_p), ("chi", C.c_void_p),
        ("implicit_capture", C.c_int32), ("w_cutoff", C.c_double), ("w_survival", C.c_double),
        ("ww_n", C.c_int32 * 3), ("ww_lo", C.c_void_p), ("ww_ratio", C.c_double), ("ww_surv", C.c_double),
        ("ww_max_split", C.c_int32),
    ]


class OrcSite(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("dir", C.c_double * 3), ("e", C.c_double), ("w", C.c_double),
                ("t", C.c_double), ("g", C.c_int32), ("cell", C.c_int32 * 3)]


class OrcDigest(C.Structure):
    _fields_ = [("qsum", C.c_int64), ("flights", C.c_uint32), ("collisions", C.c_uint32),
                ("fate", C.c_uint32), ("pad", C.c_uint32)]


DIGEST_DTYPE = np.dtype([("qsum", "<i8"), ("flights", "<u4"), ("collisions", "<u4"),
                         ("fate", "<u4"), ("pad", "<u4")])
COUNT_NAMES = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks",
               "reflections", "cutoffs", "killed", "pieces", "qsum", "overflow", "fissions", "sites", "roulettes",
               "cdf_scans", "splits"]


class OrcCounts(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in COUNT_NAMES]


_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH) or any(os.path.getmtime(f) > os.path.getmtime(LIB_PATH)
                                                   for f in SOURCES):
                build()
            L = C.CDLL(LIB_PATH)
            P = C.POINTER
            L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
            L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
            L.orc_uniform.restype = C.c_double
            for f in ("orc_nlog", "orc_sqrt"):
                getattr(L, f).argtypes = [C.c_double]
                getattr(L, f).restype = C.c_double
            L.orc_cos_sin_turn.argtypes = [C.c_double, P(C.c_double), P(C.c_double)]
            L.orc_fixed.argtypes = [C.c_double, C.c_int32]
            L.orc_fixed.restype = C.c_int64
            L.orc_locate.argtypes = [P(OrcProblem), P(C.c_double), P(C.c_double), P(C.c_int32)]
            L.orc_distance.argtypes = [P(OrcProblem), P(C.c_double), P(C.c_double), P(C.c_int32), P(C.c_int32)]
            L.orc_distance.restype = C.c_double
            L.orc_ce_index.argtypes = [C.c_void_p, C.c_int32, C.c_double]
            L.orc_ce_index.restype = C.c_int32
            L.orc_ce_index_fast.argtypes = [C.c_void_p, C.c_int32, C.c_double]
            L.orc_ce_index_fast.restype = C.c_int32
            L.orc_edge_index.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32]
            L.orc_run_gen.argtypes = [P(OrcProblem), C.c_int32, C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p,
                                      C.c_void_p, P(OrcCounts), C.c_void_p, C.c_uint64, P(C.c_uint64)]
            L.orc_edge_index.restype = C.c_int32
            L.orc_elastic.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, P(C.c_double)]
            L.orc_elastic.restype = C.c_double
            L.orc_tally_segment.argtypes = [P(OrcProblem), P(C.c_double), P(C.c_double), C.c_double,
                                            C.c_int32, C.c_void_p]
            L.orc_ce_xs_hook.argtypes = [P(OrcProblem), C.c_int32, C.c_double, C.c_void_p, C.c_void_p]
            L.orc_ce_xs_hook.restype = C.c_double
            L.orc_run.argtypes = [P(OrcProblem), C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p, P(OrcCounts)]
            L.orc_replay_a.argtypes = [P(OrcProblem), C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p,
                                       P(C.c_uint64)]
            L.orc_replay_b.argtypes = [P(OrcProblem), C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
            L.orc_eigen.argtypes = [P(OrcProblem), C.c_uint64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, P(OrcCounts), C.c_void_p, C.c_uint64, P(C.c_uint64)]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check_windows(d: dict) -> None:
    """Weight windows need a finite box (their grid spans it)."""
    if int(d.get("ww_n", [0])[0]) > 0:
        if not (np.all(np.isfinite(d["box_lo"])) and np.all(np.isfinite(d["box_hi"]))):
            raise ValueError("weight windows need a finite box")
        if min(int(v) for v in d["ww_n"]) < 1 or len(d["ww_lo"]) != int(np.prod(d["ww_n"])):
            raise ValueError("weight windows: ww_n >= 1 per axis and one lower bound per cell")
        if not (float(d["ww_ratio"]) > float(d["ww_surv"]) > 1.0 and int(d["ww_max_split"]) >= 2):
            raise ValueError("weight windows: need ww_ratio > ww_surv > 1 and ww_max_split >= 2")


def _check_tally_covers(d: dict) -> None:
    """A mesh tally's edges must contain the geometry's box and a
    continuous-energy tally's edges [e_min, e_source]; otherwise track outside
    them would have no bin (the last energy bin holds its upper edge).  Such
    problems are not accepted."""
    if int(d["tally_kind"]) == 0:
        for a, name in enumerate(("mesh_x", "mesh_y", "mesh_z")):
            e = np.asarray(d[name], np.float64)
            if not (e[0] <= d["box_lo"][a] and e[-1] >= d["box_hi"][a]):
                raise ValueError(f"mesh edges {name} do not contain the box")
    elif int(d["energy_mode"]) == 1:
        e = np.asarray(d["e_edges"], np.float64)
        if not (e[0] <= d["e_min"] and d["e_source"] <= e[-1]):
            raise ValueError("energy edges do not contain [e_min, e_source]")


class Problem:
    """A problem description marshalled for the oracle.  Keeps references to
    every array it points into."""

    def __init__(self, d: dict):
        self.d = d
        keep = {}
        _check_tally_covers(d)
        _check_windows(d)

        def arr(name, dtype):
            a = np.ascontiguousarray(np.asarray(d[name], dtype=dtype))
            keep[name] = a
            return _ptr(a)

        s = OrcProblem()
        s.geometry = d["geometry"]
        s.box_lo[:] = list(d["box_lo"])
        s.box_hi[:] = list(d["box_hi"])
        s.bc[:] = [int(b) for b in d["bc"]]
        s.n_slabs = d["n_slabs"]
        s.slab_planes = arr("slab_planes", np.float64)
        s.slab_mat = arr("slab_mat", np.int32)
        s.nx, s.ny = d["nx"], d["ny"]
        s.xplanes = arr("xplanes", np.float64)
        s.yplanes = arr("yplanes", np.float64)
        s.cx = arr("cx", np.float64)
        s.cy = arr("cy", np.float64)
        s.radius = d["radius"]
        s.pin_mat = arr("pin_mat", np.int32)
        s.mod_mat = d["mod_mat"]
        s.energy_mode = d["energy_mode"]
        s.n_mat, s.n_grp = d["n_mat"], d["n_grp"]
        s.sigma_t = arr("sigma_t", np.float64)
        s.sigma_s = arr("sigma_s", np.float64)
        s.cdf = arr("cdf", np.float64)
        s.n_species, s.grid_len = d["n_species"], d["grid_len"]
        s.e_grid = arr("e_grid", np.float64)
        s.sig_a = arr("sig_a", np.float64)
        s.sig_s = arr("sig_s", np.float64)
        s.awr = arr("awr", np.float64)
        s.density = arr("density", np.float64)
        s.e_min, s.e_source = d["e_min"], d["e_source"]
        s.src_kind = d["src_kind"]
        s.src_isotropic = d["src_isotropic"]
        s.src_group = d["src_group"]
        s.tally_kind = d["tally_kind"]
        s.src_pos[:] = list(d["src_pos"])
        s.src_lo[:] = list(d["src_lo"])
        s.src_hi[:] = list(d["src_hi"])
        s.src_dir[:] = list(d["src_dir"])
        s.src_radius = d["src_radius"]
        s.mesh_n[:] = [int(v) for v in d["mesh_n"]]
        s.mesh_x = arr("mesh_x", np.float64)
        s.mesh_y = arr("mesh_y", np.float64)
        s.mesh_z = arr("mesh_z", np.float64)
        s.n_ebins = d["n_ebins"]
        s.e_edges = arr("e_edges", np.float64)
        s.tally_scale_log2 = d["tally_scale_log2"]
        s.problem_id = d["problem_id"]
        s.seed = d["seed"]
        s.max_steps = d["max_steps"]
        s.n_tbins = int(d.get("n_tbins", 0))
        s.t_max = float(d.get("t_max", 0.0))
        if s.n_tbins > 0 and d["energy_mode"] == 0:
            s.speed = arr("speed", np.float64)
        s.speed_coef = float(d.get("speed_coef", 0.0))
        s.implicit_capture = int(d.get("implicit_capture", 0))
        s.w_cutoff = float(d.get("w_cutoff", 0.0))
        s.w_survival = float(d.get("w_survival", 0.0))
        if int(d.get("ww_n", [0])[0]) > 0:
            s.ww_n[:] = [int(v) for v in d["ww_n"]]
            s.ww_lo = arr("ww_lo", np.float64)
            s.ww_ratio = float(d["ww_ratio"])
            s.ww_surv = float(d["ww_surv"])
            s.ww_max_split = int(d["ww_max_split"])
        if d.get("sigma_f") is not None:
            s.sigma_f = arr("sigma_f", np.float64)
            s.nu = arr("nu", np.float64)
            s.chi = arr("chi", np.float64)
        self.s = s
        self._keep = keep

    @property
    def n_bins(self) -> int:
        d = self.d
        if d["tally_kind"] == 0:
            nb = int(np.prod(d["mesh_n"])) * (int(d["n_grp"]) if d["energy_mode"] == 0 else 1)
        else:
            nb = int(d["n_ebins"])
        return nb * max(1, int(d.get("n_tbins", 0)))


def _ranges(h0: int, h1: int, threads: int):
    n = h1 - h0
    threads = max(1, min(threads, n)) if n > 0 else 1
    cuts = [h0 + (n * k) // threads for k in range(threads + 1)]
    return [(cuts[k], cuts[k + 1]) for k in range(threads)]


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def run(d: dict, h0: int = 0, h1: int | None = None, *, digest: bool = False, threads: int | None = None):
    """Forward run of histories [h0, h1).  Returns a dict with the int64
    tally, counters (summed over threads) and, optionally, per-history
    digests.  Problems with weight windows run in generations (run_ww)."""
    if int(d.get("ww_n", [0])[0]) > 0:
        return run_ww(d, h0, h1, digest=digest, threads=threads)
    P = Problem(d)
    L = lib()
    if h1 is None:
        h1 = d["n_histories"]
    threads = default_threads() if threads is None else threads
    parts = _ranges(h0, h1, threads)
    tallies = [np.zeros(P.n_bins, dtype=np.int64) for _ in parts]
    counts = [OrcCounts() for _ in parts]
    dig = np.zeros(h1 - h0, dtype=DIGEST_DTYPE) if digest else None
    rcs = [0] * len(parts)

    def work(k):
        a, b = parts[k]
        dptr = _ptr(dig[a - h0:]) if digest else None
        rcs[k] = L.orc_run(C.byref(P.s), a, b, _ptr(tallies[k]), dptr, C.byref(counts[k]))

    _parallel(work, len(parts))
    tally = np.sum(tallies, axis=0, dtype=np.int64) if tallies else np.zeros(P.n_bins, np.int64)
    tot = {n: 0 for n in COUNT_NAMES}
    for c in counts:
        for n in COUNT_NAMES:
            tot[n] += int(getattr(c, n))
    # the overflow rule is on the total of all contributions, not per part
    tot["overflow"] = int(tot["qsum"] >= 2 ** 63 or any(c.overflow for c in counts))
    out = dict(tally=tally, counts=tot)
    if digest:
        out["digest"] = dig
    return out


MAX_GENERATIONS = 64


def run_ww(d: dict, h0: int = 0, h1: int | None = None, *, digest: bool = False, threads: int | None = None,
           max_generations: int = MAX_GENERATIONS):
    """Forward run with weight windows: generation 0 runs histories [h0, h1)
    from the problem's source; the copies they split off, in history order,
    are the histories of generation 1 (random-number stream 1), and so on
    until a generation splits nothing.  Histories of a generation run in
    threads over contiguous ranges whose banks are joined in range order, so
    every generation's order is the sequential one.  Returns the summed
    tally and counters, the history count of every generation and,
    optionally, generation 0's digests."""
    P = Problem(d)
    L = lib()
    if h1 is None:
        h1 = d["n_histories"]
    threads = default_threads() if threads is None else threads
    tally = np.zeros(P.n_bins, dtype=np.int64)
    tot = {n: 0 for n in COUNT_NAMES}
    gens = []
    dig = np.zeros(h1 - h0, dtype=DIGEST_DTYPE) if digest else None
    src = None
    lo, hi = h0, h1
    any_overflow = False
    for gen in range(max_generations):
        gens.append(hi - lo)
        parts = _ranges(lo, hi, threads)
        tallies = [np.zeros(P.n_bins, dtype=np.int64) for _ in parts]
        counts = [OrcCounts() for _ in parts]
        caps = [max(1024, 4 * (b - a) + 64) for a, b in parts]
        banks = [(OrcSite * c)() for c in caps]
        ns = [C.c_uint64(0) for _ in parts]
        rcs = [0] * len(parts)

        def work(k):
            a, b = parts[k]
            dptr = _ptr(dig[a - h0:]) if (digest and gen == 0) else None
            sp = C.cast(src, C.c_void_p) if src is not None else None
            for _ in range(40):
                rcs[k] = L.orc_run_gen(C.byref(P.s), gen, sp, a, b, _ptr(tallies[k]), dptr, C.byref(counts[k]),
                                       C.cast(banks[k], C.c_void_p), caps[k], C.byref(ns[k]))
                if rcs[k] != 3:
                    return
                # the range split off more copies than its bank holds: run it
                # again from scratch with a larger bank (it is deterministic)
                tallies[k][:] = 0
                caps[k] *= 4
                banks[k] = (OrcSite * caps[k])()

        _parallel(work, len(parts))
        if any(r == 3 for r in rcs):
            raise RuntimeError("oracle: split bank full")
        any_overflow = any_overflow or any(r == 1 for r in rcs)
        for t in tallies:
            tally += t
        for c in counts:
            for n in COUNT_NAMES:
                tot[n] += int(getattr(c, n))
        m = sum(n.value for n in ns)
        if m == 0:
            break
        nxt = (OrcSite * m)()
        o = 0
        for k in range(len(parts)):
            n = ns[k].value
            C.memmove(C.addressof(nxt) + o * C.sizeof(OrcSite), banks[k], n * C.sizeof(OrcSite))
            o += n
        src, lo, hi = nxt, 0, m
    else:
        raise RuntimeError("oracle: more than %d generations of split copies" % max_generations)
    tot["overflow"] = int(tot["qsum"] >= 2 ** 63 or any_overflow)
    out = dict(tally=tally, counts=tot, generations=gens)
    if digest:
        out["digest"] = dig
    return out


def replay_a(d: dict, w: np.ndarray, h0: int = 0, h1: int | None = None, threads: int | None = None):
    """Pass A of the score-function backward: per-history G_h and the
    integer bound U."""
    P = Problem(d)
    L = lib()
    if h1 is None:
        h1 = d["n_histories"]
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert w.size == P.n_bins
    G = np.zeros(h1 - h0, dtype=np.float64)
    threads = default_threads() if threads is None else threads
    parts = _ranges(h0, h1, threads)
    Us = [C.c_uint64(0) for _ in parts]
    rcs = [0] * len(parts)

    def work(k):
        a, b = parts[k]
        rcs[k] = L.orc_replay_a(C.byref(P.s), a, b, _ptr(w), _ptr(G[a - h0:]), C.byref(Us[k]))

    _parallel(work, len(parts))
    U = sum(int(u.value) for u in Us)
    if any(rcs) or U >= 2 ** 64:
        raise OverflowError("score-function bound does not fit 64 bits")
    return G, U


def grad_scale(U: int) -> int:
    """s = 62 - ceil(log2(U + 1)) = 62 - bit_length(U)."""
    return 62 - int(U).bit_length()


def replay_b(d: dict, G: np.ndarray, s: int, h0: int = 0, h1: int | None = None, threads: int | None = None,
             w: np.ndarray | None = None):
    """Pass B: the fixed-point sums SL, SA, SS at scale 2^s.  Weighted
    (implicit-capture) runs need the loss weights w again: SS is then the
    score still to come at each collision."""
    P = Problem(d)
    L = lib()
    if h1 is None:
        h1 = d["n_histories"]
    mg = d["n_mat"] * d["n_grp"]
    G = np.ascontiguousarray(G, dtype=np.float64)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float64)
        assert w.size == P.n_bins
        wp = _ptr(w)
    elif d.get("implicit_capture", 0):
        raise ValueError("pass B of a weighted run needs the loss weights")
    threads = default_threads() if threads is None else threads
    parts = _ranges(h0, h1, threads)
    acc = [[np.zeros(mg, np.int64) for _ in range(3)] for _ in parts]

    def work(k):
        a, b = parts[k]
        L.orc_replay_b(C.byref(P.s), a, b, wp, _ptr(G[a - h0:]), s, *[_ptr(x) for x in acc[k]])

    _parallel(work, len(parts))
    SL = np.sum([a[0] for a in acc], axis=0, dtype=np.int64)
    SA = np.sum([a[1] for a in acc], axis=0, dtype=np.int64)
    SS = np.sum([a[2] for a in acc], axis=0, dtype=np.int64)
    return SL, SA, SS


def grads_from_sums(d: dict, SL, SA, SS, s: int, n: int):
    """Analog runs: grad Sigma_t = (-SL + SA/Sigma_a) 2^-s / N and
    grad Sigma_s = (SS/Sigma_s - SA/Sigma_a) 2^-s / N.  Implicit capture (SA
    over collisions, SS the score still to come at them):
    grad Sigma_t = (-SL + (SA/Sigma_t - SS/Sigma_t)) 2^-s / N and
    grad Sigma_s = (SS/Sigma_s) 2^-s / N.  In float64."""
    st = np.asarray(d["sigma_t"], np.float64).ravel()
    ss = np.asarray(d["sigma_s"], np.float64).ravel()
    sa = st - ss
    sc = 2.0 ** (-s)
    gt = np.empty_like(st)
    gs = np.empty_like(st)
    weighted = bool(d.get("implicit_capture", 0))
    for p in range(st.size):
        if weighted:
            gt[p] = ((-float(SL[p])) + ((float(SA[p]) / st[p]) - (float(SS[p]) / st[p]))) * sc / n
            gs[p] = (float(SS[p]) / ss[p]) * sc / n
        else:
            gt[p] = ((-float(SL[p])) + (float(SA[p]) / sa[p])) * sc / n
            gs[p] = ((float(SS[p]) / ss[p]) - (float(SA[p]) / sa[p])) * sc / n
    return gt, gs


def backward(d: dict, w: np.ndarray, threads: int | None = None):
    """Score-function vector-Jacobian product for the normalised tally
    T = raw * 2^-S / N: returns (grad Sigma_t, grad Sigma_s), each [M*G].

    With implicit capture the tally carries weights that are products of
    Sigma_s / Sigma_t over earlier collisions: the estimator adds their
    derivative along the path (the score still to come after a collision,
    times d log(Sigma_s / Sigma_t)) to the score of the path's density, in
    which a collision is Sigma_t exp(-Sigma_t l) and the roulette's survival
    probability is held at its value (a roulette with a fixed probability
    is unbiased for every Sigma and plays the same game here)."""
    if int(d.get("energy_mode", 0)) != 0:
        raise ValueError("the score-function backward needs a multigroup problem")
    if int(d.get("ww_n", [0])[0]) > 0:
        raise ValueError("the score-function backward takes no weight windows")
    G, U = replay_a(d, w, threads=threads)
    s = grad_scale(U)
    SL, SA, SS = replay_b(d, G, s, threads=threads, w=w)
    gt, gs = grads_from_sums(d, SL, SA, SS, s, d["n_histories"])
    return dict(grad_sigma_t=gt, grad_sigma_s=gs, G=G, U=U, s=s, SL=SL, SA=SA, SS=SS)


def eigen(d: dict, n_particles: int, n_cycles: int, n_inactive: int, bank_cap: int | None = None):
    """k-eigenvalue power iteration (multigroup problem with fission data):
    the int64 tally summed over the active cycles, k and the source size of
    every cycle, counters over all cycles and the source bank that would
    start the next cycle (positions, [n, 3])."""
    P = Problem(d)
    if d.get("sigma_f") is None:
        raise ValueError("k-eigenvalue runs need fission data")
    if d.get("implicit_capture", 0):
        raise ValueError("k-eigenvalue runs are analog (no implicit capture)")
    if int(d.get("ww_n", [0])[0]) > 0:
        raise ValueError("k-eigenvalue runs take no weight windows")
    L = lib()
    tally = np.zeros(P.n_bins, dtype=np.int64)
    k = np.zeros(n_cycles, dtype=np.float64)
    ns = np.zeros(n_cycles, dtype=np.uint64)
    cap = 2 * n_particles + 1024 if bank_cap is None else bank_cap
    bank = np.zeros((cap, 3), dtype=np.float64)
    bn = C.c_uint64(0)
    cnt = OrcCounts()
    rc = L.orc_eigen(C.byref(P.s), n_particles, n_cycles, n_inactive, _ptr(tally), _ptr(k), _ptr(ns),
                     C.byref(cnt), _ptr(bank), cap, C.byref(bn))
    if rc == 2:
        raise RuntimeError("no neutron was banked in a cycle")
    if rc == 3:
        raise RuntimeError("source bank capacity exceeded")
    counts = {n: int(getattr(cnt, n)) for n in COUNT_NAMES}
    return dict(tally=tally, k=k, n_source=ns.astype(np.int64), counts=counts, bank=bank[:bn.value].copy(),
                status=rc)


def _parallel(fn, n):
    if n == 1:
        fn(0)
        return
    ts = [threading.Thread(target=fn, args=(k,)) for k in range(n)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()


# ----------------------------------------------------------- primitive hooks

def philox(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    L.orc_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def uniform(seed, problem_id, particle, step, slot, stream=0):
    return lib().orc_uniform(seed, problem_id, particle, step, slot, stream)


def nlog(x):
    return lib().orc_nlog(float(x))


def sqrt(x):
    return lib().orc_sqrt(float(x))


def cos_sin_turn(t):
    c, s = C.c_double(), C.c_double()
    lib().orc_cos_sin_turn(float(t), C.byref(c), C.byref(s))
    return c.value, s.value


def fixed(x, scale_log2):
    return lib().orc_fixed(float(x), int(scale_log2))


def locate(P: Problem, pos, dir_):
    cell = (C.c_int32 * 3)()
    lib().orc_locate(C.byref(P.s), (C.c_double * 3)(*pos), (C.c_double * 3)(*dir_), cell)
    return tuple(cell)


def distance(P: Problem, pos, dir_, cell):
    surf = C.c_int32()
    d = lib().orc_distance(C.byref(P.s), (C.c_double * 3)(*pos), (C.c_double * 3)(*dir_),
                           (C.c_int32 * 3)(*cell), C.byref(surf))
    return d, surf.value


def ce_index(grid: np.ndarray, e: float, fast: bool = False):
    grid = np.ascontiguousarray(grid, np.float64)
    f = lib().orc_ce_index_fast if fast else lib().orc_ce_index
    return f(_ptr(grid), grid.size, float(e))


def edge_index(edges: np.ndarray, x: float, direction: float, fast: bool):
    edges = np.ascontiguousarray(edges, np.float64)
    return lib().orc_edge_index(_ptr(edges), edges.size - 1, float(x), float(direction), int(fast))


def elastic(A, e, xi_mu, xi_phi, dir_):
    d = (C.c_double * 3)(*dir_)
    enew = lib().orc_elastic(float(A), float(e), float(xi_mu), float(xi_phi), d)
    return enew, tuple(d)


def tally_segment(P: Problem, pos, dir_, d, g=0):
    out = np.zeros(P.n_bins, np.float64)
    lib().orc_tally_segment(C.byref(P.s), (C.c_double * 3)(*pos), (C.c_double * 3)(*dir_), float(d), int(g),
                            _ptr(out))
    return out


def ce_xs(P: Problem, m, e):
    S = P.d["n_species"]
    sa = np.zeros(S)
    ss = np.zeros(S)
    st = lib().orc_ce_xs_hook(C.byref(P.s), int(m), float(e), _ptr(sa), _ptr(ss))
    return st, sa, ss
