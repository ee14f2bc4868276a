"""Python binding of the C ABI in include/colt.h (argument marshalling only).

Every step of the transport runs in the HIP library libcolt.so; this module
only converts workload dictionaries (see ``inputs``) to the C descriptors,
supplies device memory from torch's caching allocator and torch's current
stream, and copies tallies back to numpy arrays.  Loading fails loudly if the
library is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcolt.so")

COLT_OK = 0
FP64 = 0
FP32_BULK = 1
N_COUNTERS = 16
COUNTER_NAMES = ["emitted", "escaped", "absorbed", "scat_hi", "scat_dust", "crossings",
                 "peels", "upar_tries", "peel_crossings", "capped", "upar_rounds", "passes"]

EXPORTS = ["colt_init_grid", "colt_emit", "colt_transport", "colt_tally", "colt_job_status",
           "colt_grid_bytes", "colt_job_bytes", "colt_last_kernel_ms", "colt_release_job",
           "colt_release_grid", "colt_last_error", "colt_grid_fields", "colt_octree_links",
           "colt_eval_voigt",
           "colt_sample", "colt_grid_nonlocal", "colt_graph_create", "colt_graph_launch",
           "colt_graph_release", "colt_stop_set", "colt_job_pending", "colt_job_footprint",
           "colt_transport_static"]

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class ColtError(RuntimeError):
    pass


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC), ("free", _FREE), ("user", ctypes.c_void_p)]


class GridDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("box_min", ctypes.c_double * 3),
                ("box_max", ctypes.c_double * 3), ("n_cells", ctypes.c_int64),
                ("child", _ip), ("n_HI", _dp), ("T", _dp), ("v", _dp), ("k_dust", _dp),
                ("atau_nl", _dp), ("dust_albedo", ctypes.c_double),
                ("escape_radius", ctypes.c_double)]


class SourceDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_src", ctypes.c_int32), ("pos", _dp),
                ("weight", _dp), ("sigma", ctypes.c_double), ("freq_mode", ctypes.c_int32)]


class JobParams(ctypes.Structure):
    _fields_ = [("n_photons", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("xcrit_mode", ctypes.c_int32),
                ("atau0", ctypes.c_double), ("recoil", ctypes.c_int32),
                ("isotropic", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("n_cams", ctypes.c_int32), ("cam_dir", _dp), ("cam_nbins", ctypes.c_int32),
                ("cam_xmin", ctypes.c_double), ("cam_xmax", ctypes.c_double),
                ("cam_npix", ctypes.c_int32), ("cam_fov", ctypes.c_double),
                ("tau_peel_max", ctypes.c_double), ("record", ctypes.c_int32),
                ("max_events", ctypes.c_uint64), ("march_tasks", ctypes.c_uint64)]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("photons_per_job", ctypes.c_uint64), ("time_kernel", ctypes.c_int32),
                ("march_min", ctypes.c_int32), ("stop_token", ctypes.c_int32),
                ("tail_live", ctypes.c_int32), ("launches", ctypes.c_int32)]


class TallyOut(ctypes.Structure):
    _fields_ = [("spectrum", _dp), ("cam_spec", _dp), ("cam_img", _dp),
                ("counters", ctypes.c_uint64 * N_COUNTERS), ("rec_x", _dp),
                ("rec_nscat", _ip), ("rec_status", _ip), ("rec_pos", _dp),
                ("rec_peel", _dp)]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ColtError(f"HIP library {LIB_PATH} not built; run "
                            "python -m paper_1409_4480_amd.build")
        # torch's HIP runtime must be the process's runtime: load it first so the
        # library's libamdhip64 dependency resolves to the copy torch uses.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.colt_init_grid.argtypes = [ctypes.POINTER(GridDesc), ctypes.POINTER(Allocator), vp,
                                     ctypes.POINTER(vp)]
        L.colt_emit.argtypes = [vp, ctypes.POINTER(SourceDesc), ctypes.POINTER(JobParams),
                                ctypes.POINTER(vp)]
        L.colt_transport.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Launch), vp]
        L.colt_transport_static.argtypes = [ctypes.POINTER(vp), ctypes.c_int32,
                                            ctypes.POINTER(Launch), vp]
        L.colt_tally.argtypes = [vp, ctypes.POINTER(TallyOut), ctypes.c_int32]
        L.colt_job_status.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.colt_grid_bytes.argtypes = [vp]
        L.colt_grid_bytes.restype = ctypes.c_size_t
        L.colt_job_bytes.argtypes = [vp]
        L.colt_job_bytes.restype = ctypes.c_size_t
        L.colt_last_kernel_ms.argtypes = []
        L.colt_last_kernel_ms.restype = ctypes.c_double
        L.colt_release_job.argtypes = [vp]
        L.colt_release_job.restype = None
        L.colt_release_grid.argtypes = [vp]
        L.colt_last_error.restype = ctypes.c_char_p
        L.colt_grid_fields.argtypes = [vp, _dp]
        L.colt_octree_links.argtypes = [_ip, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_int64)]
        L.colt_grid_nonlocal.argtypes = [vp, ctypes.c_double, vp]
        L.colt_graph_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Launch),
                                        vp, ctypes.POINTER(vp)]
        L.colt_graph_launch.argtypes = [vp, vp]
        L.colt_graph_release.argtypes = [vp]
        L.colt_graph_release.restype = None
        L.colt_stop_set.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.colt_job_footprint.argtypes = [ctypes.POINTER(JobParams), ctypes.c_int32]
        L.colt_job_footprint.restype = ctypes.c_size_t
        L.colt_job_pending.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64]
        L.colt_eval_voigt.argtypes = [ctypes.c_int32, _dp, _dp, ctypes.c_int64, _dp, vp]
        L.colt_sample.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_int64, _dp, _ip, vp]
        for name in ("colt_init_grid", "colt_emit", "colt_transport", "colt_tally",
                     "colt_job_status", "colt_release_grid", "colt_grid_fields",
                     "colt_eval_voigt", "colt_sample", "colt_grid_nonlocal",
                     "colt_graph_create", "colt_graph_launch", "colt_stop_set",
                     "colt_job_pending", "colt_transport_static", "colt_octree_links"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(rc):
    if rc != COLT_OK:
        msg = lib().colt_last_error().decode(errors="replace")
        raise ColtError(f"colt error {rc}: {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise ColtError("no HIP device visible")
    return torch


def current_stream():
    """Handle of torch's current HIP stream on the current device."""
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


class _TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self):
        torch = _torch()
        self._torch = torch

        def alloc(nbytes, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
            except Exception:
                return None

        def free(ptr, user):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc = _ALLOC(alloc)
        self._free = _FREE(free)
        self.struct = Allocator(self._alloc, self._free, None)


_allocator = None


def torch_allocator():
    global _allocator
    if _allocator is None:
        _allocator = _TorchAllocator()
    return _allocator


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class Grid:
    """Gas on a Cartesian or octree grid, resident on the device."""

    def __init__(self, grid, stream=None, use_torch_allocator=True):
        L = lib()
        d = GridDesc()
        d.kind = int(grid["kind"])
        n_cells = int(np.asarray(grid["n_HI"]).size)
        if d.kind == 0:
            d.nx, d.ny, d.nz = (int(v) for v in grid["shape"])
        d.box_min[:] = [float(v) for v in grid["box_min"]]
        d.box_max[:] = [float(v) for v in grid["box_max"]]
        d.n_cells = n_cells
        keep = []
        child = grid.get("child")
        if child is not None:
            child = np.ascontiguousarray(child, dtype=np.int32)
            keep.append(child)
        d.child = _ptr(child, _ip)
        for name, key, n in (("n_HI", "n_HI", n_cells), ("T", "T", n_cells),
                             ("v", "v", 3 * n_cells), ("k_dust", "k_dust", n_cells),
                             ("atau_nl", "atau_nl", n_cells)):
            arr = _f64(grid.get(key), n)
            keep.append(arr)
            setattr(d, name, _ptr(arr))
        d.dust_albedo = float(grid.get("albedo", 0.0))
        d.escape_radius = float(grid.get("escape_radius", 0.0))
        self.stream = stream if stream is not None else current_stream()
        alloc = torch_allocator().struct if use_torch_allocator else None
        h = ctypes.c_void_p()
        _check(L.colt_init_grid(ctypes.byref(d), ctypes.byref(alloc) if alloc else None,
                                self.stream, ctypes.byref(h)))
        self.handle = h
        self.kind = d.kind
        self.n_leaves = int(np.sum(np.asarray(child) < 0)) if d.kind == 1 else n_cells
        f_nl = float(grid.get("f_nl", 0.0))
        if f_nl > 0.0:
            self.nonlocal_estimate(f_nl)

    def nonlocal_estimate(self, f_nl):
        """Replaces the per-cell non-local a*tau with the device estimate."""
        _check(lib().colt_grid_nonlocal(self.handle, float(f_nl), self.stream))

    @property
    def nbytes(self):
        return int(lib().colt_grid_bytes(self.handle))

    def fields(self):
        """Device-derived per-cell fields, (n_cells, 11): k0, a, v_th, u (3),
        k_dust, x_cw, g, atau_nl, atau_J."""
        out = np.zeros((self.n_leaves, 11))
        _check(lib().colt_grid_fields(self.handle, _ptr(out)))
        return out

    def release(self):
        if self.handle:
            _check(lib().colt_release_grid(self.handle))
            self.handle = None


def _job_descs(source, params, precision=FP64, record=False, max_events=0, march_tasks=0):
    """C descriptors of a job's sources and parameters (and the arrays they
    point to, which must outlive them)."""
    s = SourceDesc()
    pos = _f64(source["pos"])
    s.kind = int(source["kind"])
    s.n_src = pos.size // 3
    s.pos = _ptr(pos)
    w = _f64(source.get("weight"))
    s.weight = _ptr(w)
    s.sigma = float(source.get("sigma", 0.0))
    s.freq_mode = int(source.get("freq_mode", 0))
    p = JobParams()
    p.n_photons = int(params["n_photons"])
    p.seed = int(params["seed"])
    p.precision = int(precision)
    p.xcrit_mode = int(params.get("xcrit_mode", 0))
    p.atau0 = float(params.get("atau0", 0.0))
    p.recoil = int(params.get("recoil", 0))
    p.isotropic = int(params.get("isotropic", 0))
    p.n_bins = int(params.get("n_bins", 0))
    p.x_min = float(params.get("x_min", -1.0))
    p.x_max = float(params.get("x_max", 1.0))
    cams = params.get("cam_dir")
    cams = None if cams is None else _f64(cams)
    n_cams = 0 if cams is None else cams.size // 3
    p.n_cams = n_cams
    p.cam_dir = _ptr(cams)
    p.cam_nbins = int(params.get("cam_nbins", 0)) if n_cams else 0
    p.cam_xmin = float(params.get("cam_xmin", -1.0))
    p.cam_xmax = float(params.get("cam_xmax", 1.0))
    p.cam_npix = int(params.get("cam_npix", 0)) if n_cams else 0
    p.cam_fov = float(params.get("cam_fov", 1.0))
    p.tau_peel_max = float(params.get("tau_peel_max", 50.0))
    p.record = int(bool(record))
    p.max_events = int(max_events)
    p.march_tasks = int(march_tasks or params.get("march_tasks", 0))
    return s, p, (pos, w, cams)


def octree_links(child):
    """The neighbour links the library builds for an octree node table (host
    only): an (n_leaves, 6) uint32 array, face 2 axis + (step > 0)."""
    child = np.ascontiguousarray(child, np.int32)
    n = ctypes.c_int64(0)
    _check(lib().colt_octree_links(_ptr(child, _ip), len(child), None, ctypes.byref(n)))
    out = np.zeros((n.value, 6), np.uint32)
    _check(lib().colt_octree_links(_ptr(child, _ip), len(child),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                   ctypes.byref(n)))
    return out


def job_footprint(source, params, precision=FP64, record=False):
    """Device bytes the library allocates for a job of these parameters."""
    s, p, keep = _job_descs(source, params, precision, record)
    return int(lib().colt_job_footprint(ctypes.byref(p), int(s.n_src)))


class Job:
    """A transfer job registered on a grid."""

    def __init__(self, grid, source, params, precision=FP64, record=False, max_events=0,
                 march_tasks=0):
        L = lib()
        s, p, keep = _job_descs(source, params, precision, record, max_events, march_tasks)
        self.n_cams = int(p.n_cams)
        h = ctypes.c_void_p()
        _check(L.colt_emit(grid.handle, ctypes.byref(s), ctypes.byref(p), ctypes.byref(h)))
        self.handle = h
        self.params = p
        self._keep = keep
        self.grid = grid

    @property
    def nbytes(self):
        return int(lib().colt_job_bytes(self.handle))

    def status(self):
        """(photons taken and not suspended, total); complete when equal and
        no launch is running."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().colt_job_status(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    @property
    def complete(self):
        a, b = self.status()
        return a == b

    def pending(self, max_ids=0):
        """(next never-started id, suspended count, sorted suspended ids)."""
        nxt, ns = ctypes.c_uint64(), ctypes.c_uint64()
        ids = np.zeros(max(int(max_ids), 1), np.uint64)
        _check(lib().colt_job_pending(self.handle, ctypes.byref(nxt), ctypes.byref(ns),
                                      ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      int(max_ids)))
        return nxt.value, ns.value, ids[:min(int(max_ids), ns.value)]

    def tally(self, wait=True):
        p = self.params
        n = int(p.n_photons)
        out = {"spectrum": np.zeros(p.n_bins + 2),
               "cam_spec": np.zeros((self.n_cams, p.cam_nbins)),
               "cam_img": np.zeros((self.n_cams, p.cam_npix, p.cam_npix))}
        t = TallyOut()
        t.spectrum = _ptr(out["spectrum"])
        t.cam_spec = _ptr(out["cam_spec"])
        t.cam_img = _ptr(out["cam_img"])
        if p.record:
            rec = {"x": np.zeros(n), "nscat": np.zeros(n, np.int32),
                   "status": np.zeros(n, np.int32), "pos": np.zeros((n, 3)),
                   "peel": np.zeros((n, self.n_cams))}
            t.rec_x = _ptr(rec["x"])
            t.rec_nscat = _ptr(rec["nscat"], _ip)
            t.rec_status = _ptr(rec["status"], _ip)
            t.rec_pos = _ptr(rec["pos"])
            t.rec_peel = _ptr(rec["peel"]) if self.n_cams else None
            out["records"] = rec
        _check(lib().colt_tally(self.handle, ctypes.byref(t), int(bool(wait))))
        out["counters"] = {name: int(t.counters[i]) for i, name in enumerate(COUNTER_NAMES)}
        return out

    def release(self):
        if self.handle:
            lib().colt_release_job(self.handle)
            self.handle = None


def transport(jobs, block=0, blocks_per_cu=0, photons_per_job=0, time_kernel=False,
              stream=None, march_min=0, stop_token=0, tail_live=0, launches=1):
    """Runs (the next slice of) each job's photons in `launches` persistent
    launch sequences per precision on the stream (asynchronous).  A launch may
    stop early (a stop token, a camera job's task buffer, or tail_live): then
    call again until complete."""
    jobs = list(jobs)
    arr = (ctypes.c_void_p * max(len(jobs), 1))(*[j.handle for j in jobs])
    lc = Launch(int(block), int(blocks_per_cu), int(photons_per_job), int(bool(time_kernel)),
                int(march_min), int(stop_token), int(tail_live), int(launches))
    _check(lib().colt_transport(arr, len(jobs), ctypes.byref(lc),
                                stream if stream is not None else current_stream()))


class Graph:
    """One transport epoch over fixed jobs captured as a HIP graph; each
    launch() replays an epoch of up to photons_per_job photons per job."""

    def __init__(self, jobs, photons_per_job=0, block=0, blocks_per_cu=0, march_min=0,
                 stop_token=0, tail_live=0, launches=1):
        torch = _torch()
        self.jobs = list(jobs)
        self._capture = torch.cuda.Stream()
        arr = (ctypes.c_void_p * len(self.jobs))(*[j.handle for j in self.jobs])
        lc = Launch(int(block), int(blocks_per_cu), int(photons_per_job), 0, int(march_min),
                    int(stop_token), int(tail_live), int(launches))
        h = ctypes.c_void_p()
        torch.cuda.current_stream().synchronize()
        _check(lib().colt_graph_create(arr, len(self.jobs), ctypes.byref(lc),
                                       ctypes.c_void_p(self._capture.cuda_stream),
                                       ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().colt_graph_launch(self.handle,
                                       stream if stream is not None else current_stream()))

    def release(self):
        if self.handle:
            lib().colt_graph_release(self.handle)
            self.handle = None


def stop_set(token, value=True):
    """Sets or clears stop word `token` (1..63) polled by launches given it."""
    _check(lib().colt_stop_set(int(token), int(bool(value))))


def transport_all(jobs, max_launches=1_000_000, **kw):
    """Launches until every job is complete (a launch can stop early when a
    camera job's next-event task buffer fills); returns the launch count."""
    jobs = list(jobs)
    n = 0
    while True:
        todo = [j for j in jobs if not j.complete]
        if not todo:
            return n
        if n >= max_launches:
            raise ColtError(f"jobs not complete after {n} launches")
        transport(todo, **kw)
        n += 1


def last_kernel_ms():
    return float(lib().colt_last_kernel_ms())


def eval_voigt(a, x, precision=FP64):
    a_b, x_b = np.broadcast_arrays(np.asarray(a, float), np.asarray(x, float))
    a_c = np.ascontiguousarray(a_b).reshape(-1)
    x_c = np.ascontiguousarray(x_b).reshape(-1)
    out = np.zeros(a_c.size)
    _check(lib().colt_eval_voigt(int(precision), _ptr(a_c), _ptr(x_c), a_c.size, _ptr(out),
                                 current_stream()))
    return out.reshape(a_b.shape)


def sample(what, n, seed, p0=0.0, p1=0.0, p2=0.0, precision=FP64):
    """Device sampler draws (see colt_sample): 'upar', 'uperp', 'mu', 'uniform',
    'upar_mixed', 'upar_seq', 'upar_mixed_seq', 'scatter_draws'."""
    code = {"upar": 0, "uperp": 1, "mu": 2, "uniform": 3, "upar_mixed": 4, "upar_seq": 5,
            "upar_mixed_seq": 6, "scatter_draws": 7}[what]
    per = {1: 2, 3: int(p0), 7: 5}.get(code, 1)
    out = np.zeros(n * per)
    draws = np.zeros(n, np.int32)
    _check(lib().colt_sample(code, int(precision), float(p0), float(p1), float(p2), int(seed),
                             int(n), _ptr(out), _ptr(draws, _ip), current_stream()))
    if code in (0, 4, 5, 6):
        return out, draws
    return out.reshape(n, per) if per > 1 else out


def run(workload, precision=FP64, record=False, block=0, blocks_per_cu=0, max_events=0,
        march_min=0):
    """Initialises the grid, runs every photon of one job and returns its tallies."""
    g = Grid(workload["grid"])
    j = Job(g, workload["source"], workload["params"], precision=precision, record=record,
            max_events=max_events)
    try:
        launches = transport_all([j], block=block, blocks_per_cu=blocks_per_cu,
                                 march_min=march_min)
        out = j.tally()
        out["launches"] = launches
        return out
    finally:
        j.release()
        g.release()
