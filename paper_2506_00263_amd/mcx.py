"""ctypes binding of libmcx.so (C ABI in include/mcx.h).

Argument marshalling only: every step of the transport runs in the HIP
library.  Problem descriptions are the dictionaries produced by
``paper_2506_00263_amd.inputs``.  Device buffers (digests, dL/dT on the
device) and streams may come from PyTorch; nothing here computes physics.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mcx.h")

SCHED = {"naive": 0, "stack": 1, "async": 2}
DECOMP = {"fused": 0, "split": 1}
LOOKUP = {"binary": 0, "hash": 1}
TALLY_PATH = {"auto": 0, "lds": 1, "replicas": 2, "direct": 3}
STATUS = {0: "MCX_OK", 1: "MCX_E_INVALID_ARG", 2: "MCX_E_OOM", 3: "MCX_E_DEVICE", 4: "MCX_E_CAPACITY",
          5: "MCX_E_OVERFLOW", 6: "MCX_E_STATE"}
HOST, DEVICE = 0, 1


class McxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("bc", C.c_int32 * 6),
        ("n_slabs", C.c_int32), ("slab_planes", C.c_void_p), ("slab_mat", C.c_void_p),
        ("nx", C.c_int32), ("ny", C.c_int32), ("xplanes", C.c_void_p), ("yplanes", C.c_void_p),
        ("cx", C.c_void_p), ("cy", C.c_void_p), ("radius", C.c_double), ("pin_mat", C.c_void_p),
        ("mod_mat", C.c_int32), ("energy_mode", C.c_int32), ("n_mat", C.c_int32), ("n_grp", C.c_int32),
        ("sigma_t", C.c_void_p), ("sigma_s", C.c_void_p), ("transfer_cdf", C.c_void_p),
        ("n_species", C.c_int32), ("grid_len", C.c_int32), ("e_grid", C.c_void_p), ("sig_a", C.c_void_p),
        ("sig_s", C.c_void_p), ("awr", C.c_void_p), ("density", C.c_void_p), ("e_min", C.c_double),
        ("e_source", C.c_double), ("hash_bins", C.c_int32), ("src_kind", C.c_int32), ("src_isotropic", C.c_int32),
        ("src_group", C.c_int32), ("src_pos", C.c_double * 3), ("src_lo", C.c_double * 3),
        ("src_hi", C.c_double * 3), ("src_dir", C.c_double * 3), ("src_radius", C.c_double),
        ("tally_kind", C.c_int32), ("mesh_n", C.c_int32 * 3), ("mesh_x", C.c_void_p), ("mesh_y", C.c_void_p),
        ("mesh_z", C.c_void_p), ("n_ebins", C.c_int32), ("e_edges", C.c_void_p), ("tally_scale_log2", C.c_int32),
        ("problem_id", C.c_uint32), ("seed", C.c_uint64), ("n_histories", C.c_uint64), ("max_steps", C.c_int64),
        ("n_tbins", C.c_int32), ("t_max", C.c_double), ("speed", C.c_void_p), ("speed_coef", C.c_double),
        ("sigma_f", C.c_void_p), ("nu", C.c_void_p), ("chi", C.c_void_p),
        ("implicit_capture", C.c_int32), ("w_cutoff", C.c_double), ("w_survival", C.c_double),
        ("ww_n", C.c_int32 * 3), ("ww_lo", C.c_void_p), ("ww_ratio", C.c_double), ("ww_surv", C.c_double),
        ("ww_max_split", C.c_int32),
    ]


class RunOpts(C.Structure):
    _fields_ = [
        ("sched", C.c_int32), ("decomp", C.c_int32), ("lookup", C.c_int32), ("accumulate", C.c_int32),
        ("first_history", C.c_uint64), ("n_histories", C.c_uint64), ("stack_capacity", C.c_int64),
        ("stack_threshold", C.c_int64), ("stash_links", C.c_int32), ("arena_links", C.c_int32),
        ("waves_per_cu", C.c_int32), ("block_size", C.c_int32), ("hip_stream", C.c_void_p), ("digest", C.c_void_p),
        ("time_kernels", C.c_int32), ("force_spill", C.c_int32), ("consolidate", C.c_int32),
        ("stack_tail_events", C.c_int32), ("stack_min_events", C.c_int32), ("tally_path", C.c_int32),
        ("async_block_waves", C.c_int32), ("async_drain_events", C.c_int32),
        ("async_shared_stash", C.c_int32), ("workspace", C.c_void_p), ("ws_bytes", C.c_size_t),
        ("async_bulk_events", C.c_int32), ("stack_bulk_events", C.c_int32),
    ]


COUNTER_NAMES = ["sourced", "flights", "collisions", "scatters", "absorbs", "crossings", "leaks", "reflections",
                 "cutoffs", "killed", "pieces", "qsum", "overflow", "events", "lane_slots", "dispatches", "spills",
                 "refills", "make_work", "rounds", "launches"]


class Counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in COUNTER_NAMES] + [
        ("kernel_ms", C.c_double), ("grid_blocks", C.c_int32), ("block_threads", C.c_int32),
        ("lds_bytes", C.c_int32), ("pad", C.c_int32), ("fissions", C.c_uint64), ("sites", C.c_uint64),
        ("roulettes", C.c_uint64), ("cdf_scans", C.c_uint64), ("splits", C.c_uint64),
        ("generations", C.c_uint64)]


class EigenOpts(C.Structure):
    _fields_ = [("n_particles", C.c_uint64), ("n_cycles", C.c_int32), ("n_inactive", C.c_int32),
                ("k_cycle", C.c_void_p), ("n_source", C.c_void_p)]


DIGEST_DTYPE = np.dtype([("qsum", "<i8"), ("flights", "<u4"), ("collisions", "<u4"), ("fate", "<u4"),
                         ("pad", "<u4")])

_lib = None


def lib():
    """Load libmcx.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.mcx_create_problem.argtypes = [P(ProblemDesc), C.c_int32, P(C.c_void_p)]
        L.mcx_set_xs.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]
        L.mcx_run.argtypes = [C.c_void_p, P(RunOpts)]
        L.mcx_run_noalloc.argtypes = [C.c_void_p, P(RunOpts)]
        L.mcx_tallies.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int32]
        L.mcx_backward.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, P(RunOpts)]
        L.mcx_counters.argtypes = [C.c_void_p, P(Counters)]
        L.mcx_stack_rounds.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, P(C.c_int32)]
        L.mcx_run_eigen.argtypes = [C.c_void_p, P(RunOpts), P(EigenOpts)]
        L.mcx_workspace_size.argtypes = [C.c_void_p, P(RunOpts), P(C.c_size_t)]
        L.mcx_problem_info.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int32), P(C.c_int32),
                                       P(C.c_uint64)]
        L.mcx_destroy_problem.argtypes = [C.c_void_p]
        L.mcx_destroy_problem.restype = None
        L.mcx_status_str.argtypes = [C.c_int]
        L.mcx_status_str.restype = C.c_char_p
        L.mcx_last_error.argtypes = [C.c_void_p]
        L.mcx_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/mcx.h declares."""
    text = open(HEADER).read()
    pat = r"^(?:mcx_status|void|const char \*)\s*(mcx_[a-z_]+)\s*\("
    return sorted(set(re.findall(pat, text, flags=re.M)))


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _desc(d: dict, keep: list) -> ProblemDesc:
    def arr(name, dtype):
        a = np.ascontiguousarray(np.asarray(d[name], dtype=dtype))
        keep.append(a)
        return _ptr(a)

    s = ProblemDesc()
    s.geometry = d["geometry"]
    s.box_lo[:] = [float(v) for v in d["box_lo"]]
    s.box_hi[:] = [float(v) for v in d["box_hi"]]
    s.bc[:] = [int(v) for v in d["bc"]]
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
    s.transfer_cdf = arr("cdf", np.float64)
    s.n_species, s.grid_len = d["n_species"], d["grid_len"]
    s.e_grid = arr("e_grid", np.float64)
    s.sig_a = arr("sig_a", np.float64)
    s.sig_s = arr("sig_s", np.float64)
    s.awr = arr("awr", np.float64)
    s.density = arr("density", np.float64)
    s.e_min, s.e_source = d["e_min"], d["e_source"]
    s.hash_bins = int(d.get("hash_bins", 0))
    s.src_kind = d["src_kind"]
    s.src_isotropic = d["src_isotropic"]
    s.src_group = d["src_group"]
    s.src_pos[:] = [float(v) for v in d["src_pos"]]
    s.src_lo[:] = [float(v) for v in d["src_lo"]]
    s.src_hi[:] = [float(v) for v in d["src_hi"]]
    s.src_dir[:] = [float(v) for v in d["src_dir"]]
    s.src_radius = d["src_radius"]
    s.tally_kind = d["tally_kind"]
    s.mesh_n[:] = [int(v) for v in d["mesh_n"]]
    s.mesh_x = arr("mesh_x", np.float64)
    s.mesh_y = arr("mesh_y", np.float64)
    s.mesh_z = arr("mesh_z", np.float64)
    s.n_ebins = d["n_ebins"]
    s.e_edges = arr("e_edges", np.float64)
    s.tally_scale_log2 = d["tally_scale_log2"]
    s.problem_id = d["problem_id"]
    s.seed = d["seed"]
    s.n_histories = d["n_histories"]
    s.max_steps = d["max_steps"]
    s.n_tbins = int(d.get("n_tbins", 0))
    s.t_max = float(d.get("t_max", 0.0))
    s.speed = None
    if s.n_tbins > 0 and d["energy_mode"] == 0:
        if np.asarray(d["speed"]).size != d["n_grp"]:
            raise ValueError("time bins need one speed per group")
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
    s.sigma_f = s.nu = s.chi = None
    if d.get("sigma_f") is not None:
        mg = int(d["n_mat"]) * int(d["n_grp"])
        for name in ("sigma_f", "nu", "chi"):
            if np.asarray(d[name]).size != mg:
                raise ValueError(f"{name} needs n_mat * n_grp entries")
        s.sigma_f = arr("sigma_f", np.float64)
        s.nu = arr("nu", np.float64)
        s.chi = arr("chi", np.float64)
    return s


def run_opts(sched="async", decomp="fused", lookup="binary", accumulate=False, first=0, n=0, stack_capacity=0,
             stack_threshold=0, stash_links=0, arena_links=0, waves_per_cu=0, block_size=0, stream=None,
             digest=None, time_kernels=False, force_spill=0, consolidate=0, stack_tail_events=0,
             stack_min_events=0, tally_path="auto", async_block_waves=0,
             async_drain_events=0, workspace=None, async_shared_stash=0, async_bulk_events=0,
             stack_bulk_events=0) -> RunOpts:
    o = RunOpts()
    o.sched = SCHED[sched] if isinstance(sched, str) else int(sched)
    o.decomp = DECOMP[decomp] if isinstance(decomp, str) else int(decomp)
    o.lookup = LOOKUP[lookup] if isinstance(lookup, str) else int(lookup)
    o.accumulate = int(bool(accumulate))
    o.first_history = int(first)
    o.n_histories = int(n)
    o.stack_capacity = int(stack_capacity)
    o.stack_threshold = int(stack_threshold)
    o.stash_links = int(stash_links)
    o.arena_links = int(arena_links)
    o.waves_per_cu = int(waves_per_cu)
    o.block_size = int(block_size)
    o.hip_stream = _stream_handle(stream)
    o.digest = _ptr(digest)
    o.time_kernels = int(bool(time_kernels))
    o.force_spill = int(force_spill)
    o.stack_tail_events = int(stack_tail_events)
    o.stack_min_events = int(stack_min_events)
    o.tally_path = TALLY_PATH[tally_path] if isinstance(tally_path, str) else int(tally_path)
    o.async_block_waves = int(async_block_waves)
    o.async_drain_events = int(async_drain_events)
    o.async_bulk_events = int(async_bulk_events)
    o.stack_bulk_events = int(stack_bulk_events)
    # async stash shared by a block's wavefronts: True/1 on, False/2 off, 0 default
    o.async_shared_stash = {True: 1, False: 2}.get(async_shared_stash, async_shared_stash) \
        if isinstance(async_shared_stash, bool) else int(async_shared_stash)
    # caller-owned device scratch: a device tensor (its bytes) or None
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.ws_bytes = workspace.numel() * workspace.element_size()
    # async stash donation: None/"default" = library default, True/"on", False/"off"
    if isinstance(consolidate, bool):
        o.consolidate = 1 if consolidate else 2
    else:
        o.consolidate = {None: 0, "default": 0, "on": 1, "off": 2}.get(consolidate, consolidate)
    return o


class Problem:
    """A handle over one problem or a batch of problems (mcx_create_problem)."""

    def __init__(self, descs):
        if isinstance(descs, dict):
            descs = [descs]
        self.descs = list(descs)
        # bumped by every call that replaces what mcx_backward would replay
        # (a forward run, new cross sections): autograd checks it
        self.generation = 0
        self._keep = []
        arr = (ProblemDesc * len(self.descs))(*[_desc(d, self._keep) for d in self.descs])
        h = C.c_void_p()
        L = lib()
        st = L.mcx_create_problem(arr, len(self.descs), C.byref(h))
        if st != 0:
            raise McxError(st, "mcx_create_problem failed (invalid descriptor?)")
        self.h = h
        self._keep = None   # the library deep-copied every array

    def _check(self, st):
        if st != 0:
            raise McxError(st, lib().mcx_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().mcx_destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_problems(self) -> int:
        return len(self.descs)

    def info(self, problem: int = 0) -> dict:
        nb, nm, ng, nh = C.c_int64(), C.c_int32(), C.c_int32(), C.c_uint64()
        self._check(lib().mcx_problem_info(self.h, problem, C.byref(nb), C.byref(nm), C.byref(ng), C.byref(nh)))
        return dict(n_bins=nb.value, n_mat=nm.value, n_grp=ng.value, n_histories=nh.value)

    def set_xs(self, problem: int, sigma_t, sigma_s):
        self.generation += 1
        if hasattr(sigma_t, "data_ptr"):
            where = DEVICE if sigma_t.is_cuda else HOST
            self._check(lib().mcx_set_xs(self.h, problem, _ptr(sigma_t.contiguous()), _ptr(sigma_s.contiguous()),
                                         where))
        else:
            st = np.ascontiguousarray(sigma_t, np.float64)
            ss = np.ascontiguousarray(sigma_s, np.float64)
            self._check(lib().mcx_set_xs(self.h, problem, _ptr(st), _ptr(ss), HOST))

    def run(self, **kw):
        o = run_opts(**kw)
        self.generation += 1
        self._check(lib().mcx_run(self.h, C.byref(o)))
        return self

    def run_noalloc(self, **kw):
        """mcx_run_noalloc: the run's device scratch is the library's fixed
        array (no device allocation)."""
        o = run_opts(**kw)
        self.generation += 1
        self._check(lib().mcx_run_noalloc(self.h, C.byref(o)))
        return self

    def workspace_size(self, **kw) -> int:
        """Device scratch bytes a run (and a backward after it) with these
        options needs: the smallest `workspace` they accept."""
        o = run_opts(**kw)
        n = C.c_size_t(0)
        self._check(lib().mcx_workspace_size(self.h, C.byref(o), C.byref(n)))
        return int(n.value)

    def run_eigen(self, n_particles: int, n_cycles: int, n_inactive: int, **kw) -> dict:
        """k-eigenvalue power iteration: returns k and the source size of every
        cycle; the tallies then hold the active cycles' sum."""
        self.generation += 1
        o = run_opts(**kw)
        k = np.zeros(n_cycles, np.float64)
        ns = np.zeros(n_cycles, np.uint64)
        e = EigenOpts(int(n_particles), int(n_cycles), int(n_inactive), _ptr(k), _ptr(ns))
        self._check(lib().mcx_run_eigen(self.h, C.byref(o), C.byref(e)))
        return dict(k=k, n_source=ns.astype(np.int64))

    def tallies(self, problem: int = 0) -> np.ndarray:
        n = self.info(problem)["n_bins"]
        out = np.empty(n, np.int64)
        self._check(lib().mcx_tallies(self.h, problem, _ptr(out), n, HOST))
        return out

    def tallies_into(self, problem: int, out_device):
        """Copy raw tallies into a device int64 tensor (no host round trip)."""
        self._check(lib().mcx_tallies(self.h, problem, _ptr(out_device), out_device.numel(), DEVICE))
        return out_device

    def backward(self, dl_dt, problem: int = -1, **kw):
        """Score-function VJP of the last forward: returns (grad_sigma_t, grad_sigma_s)."""
        o = run_opts(**kw)
        if problem >= 0:
            mg = self.info(problem)["n_mat"] * self.info(problem)["n_grp"]
        else:
            mg = sum(self.info(k)["n_mat"] * self.info(k)["n_grp"] for k in range(self.n_problems))
        if hasattr(dl_dt, "data_ptr") and dl_dt.is_cuda:
            import torch
            w = dl_dt.detach().to(torch.float64).contiguous()
            gt = torch.empty(mg, dtype=torch.float64, device=w.device)
            gs = torch.empty(mg, dtype=torch.float64, device=w.device)
            self._check(lib().mcx_backward(self.h, problem, _ptr(w), _ptr(gt), _ptr(gs), DEVICE, C.byref(o)))
            return gt, gs
        gt = np.empty(mg, np.float64)
        gs = np.empty(mg, np.float64)
        w = np.ascontiguousarray(dl_dt, np.float64)
        self._check(lib().mcx_backward(self.h, problem, _ptr(w), _ptr(gt), _ptr(gs), HOST, C.byref(o)))
        return gt, gs

    def stack_rounds(self) -> np.ndarray:
        """Input particles of each remapping round of the last stack pass."""
        n = C.c_int32(0)
        self._check(lib().mcx_stack_rounds(self.h, None, 0, C.byref(n)))
        out = np.zeros(n.value, np.uint32)
        self._check(lib().mcx_stack_rounds(self.h, _ptr(out), n.value, C.byref(n)))
        return out

    def counters(self) -> dict:
        c = Counters()
        self._check(lib().mcx_counters(self.h, C.byref(c)))
        out = {n: int(getattr(c, n)) for n in COUNTER_NAMES}
        out.update(kernel_ms=c.kernel_ms, grid_blocks=c.grid_blocks, block_threads=c.block_threads,
                   lds_bytes=c.lds_bytes, fissions=int(c.fissions), sites=int(c.sites),
                   roulettes=int(c.roulettes), cdf_scans=int(c.cdf_scans), splits=int(c.splits),
                   generations=int(c.generations))
        return out

