"""Python access to the FP64 CPU oracle of the Monte-Carlo Lyman-alpha method.

TEST INFRASTRUCTURE ONLY: the oracle checks the HIP transport library against
the paper (Smith et al. 2014, Secs. 2-3 and 6.1).  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the GPU path.

Inputs are the plain dictionaries produced by the seeded workload generators
(grid, source, params; see ``run``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")

N_COUNTERS = 16
COUNTER_NAMES = ["emitted", "escaped", "absorbed", "scat_hi", "scat_dust", "crossings",
                 "peels", "upar_tries", "peel_crossings", "capped"]

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class _Grid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("box_min", ctypes.c_double * 3),
                ("box_max", ctypes.c_double * 3), ("n_nodes", ctypes.c_int64),
                ("child", _ip), ("n_HI", _dp), ("T", _dp), ("v", _dp), ("k_dust", _dp),
                ("atau_nl", _dp), ("dust_albedo", ctypes.c_double),
                ("escape_radius", ctypes.c_double)]


class _Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_src", ctypes.c_int32), ("pos", _dp),
                ("weight", _dp), ("sigma", ctypes.c_double), ("freq_mode", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("n_photons", ctypes.c_uint64), ("id_begin", ctypes.c_uint64),
                ("id_end", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("xcrit_mode", ctypes.c_int32), ("atau0", ctypes.c_double),
                ("recoil", ctypes.c_int32), ("isotropic", ctypes.c_int32),
                ("n_bins", ctypes.c_int32), ("x_min", ctypes.c_double),
                ("x_max", ctypes.c_double), ("n_cams", ctypes.c_int32), ("cam_dir", _dp),
                ("cam_nbins", ctypes.c_int32), ("cam_xmin", ctypes.c_double),
                ("cam_xmax", ctypes.c_double), ("cam_npix", ctypes.c_int32),
                ("cam_fov", ctypes.c_double), ("tau_peel_max", ctypes.c_double),
                ("max_events", ctypes.c_uint64)]


class _Out(ctypes.Structure):
    _fields_ = [("spectrum", _dp), ("cam_spec", _dp), ("cam_img", _dp),
                ("counters", ctypes.c_uint64 * N_COUNTERS), ("rec_x", _dp),
                ("rec_nscat", _ip), ("rec_status", _ip), ("rec_pos", _dp),
                ("rec_peel", _dp), ("rec_len", _dp), ("rec_ndust", _ip)]


_libs = {}
_LIB_FMA = os.path.join(_HERE, "liborc_fma.so")


def lib(variant=""):
    """Loads liborc.so (variant "fma": the same sources built with fused
    multiply-adds), building them first if missing."""
    if variant not in _libs:
        path = _LIB_FMA if variant == "fma" else _LIB
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        L.orc_run.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Source),
                              ctypes.POINTER(_Params), ctypes.POINTER(_Out), ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_nonlocal.argtypes = [ctypes.POINTER(_Grid), ctypes.c_double, _dp]
        L.orc_nonlocal.restype = None
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [ctypes.c_uint64] * 3
        L.orc_uniform.restype = ctypes.c_double
        for f in ("orc_H",):
            getattr(L, f).argtypes = [ctypes.c_double, ctypes.c_double]
            getattr(L, f).restype = ctypes.c_double
        for f in ("orc_xcw", "orc_xcrit"):
            getattr(L, f).argtypes = [ctypes.c_double]
            getattr(L, f).restype = ctypes.c_double
        L.orc_cell_constants.argtypes = [ctypes.c_double, ctypes.c_double] + [_dp] * 6
        L.orc_cell_constants.restype = None
        L.orc_sample_upar.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint64, ctypes.c_int64, _dp, _ip]
        L.orc_sample_upar_one.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_uint64, ctypes.c_uint64, _ip]
        L.orc_sample_upar_one.restype = ctypes.c_double
        L.orc_sample_uperp.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, _dp]
        L.orc_sample_mu.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, _dp]
        L.orc_upar_split.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_upar_split.restype = ctypes.c_double
        L.orc_atau_jeans.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_atau_jeans.restype = ctypes.c_double
        L.orc_xcrit_at.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), _dp, _dp,
                                   ctypes.c_double]
        L.orc_xcrit_at.restype = ctypes.c_double
        L.orc_scatter_once.argtypes = [ctypes.c_double, ctypes.c_double, _dp, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_uint64, _dp, _dp, _dp]
        L.orc_scatter_once.restype = None
        _libs[variant] = L
    return _libs[variant]


def _ptr(a, ctype=_dp):
    return None if a is None else a.ctypes.data_as(ctype)


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniform(seed, photon, k):
    return lib().orc_uniform(seed, photon, k)


def H(a, x):
    """H_approx(a, x) elementwise (appendix eq. AB)."""
    a_b, x_b = np.broadcast_arrays(np.asarray(a, float), np.asarray(x, float))
    f = lib().orc_H
    out = np.array([f(float(ai), float(xi)) for ai, xi in zip(a_b.ravel(), x_b.ravel())])
    return out.reshape(a_b.shape)


def xcw(a):
    return lib().orc_xcw(float(a))


def xcrit(atau0):
    return lib().orc_xcrit(float(atau0))


def cell_constants(T, n_HI):
    vals = [ctypes.c_double() for _ in range(6)]
    lib().orc_cell_constants(float(T), float(n_HI), *[ctypes.byref(v) for v in vals])
    names = ["a", "sigma0", "k0", "vth", "xcw", "g"]
    return {n: v.value for n, v in zip(names, vals)}


def sample_upar(a, x, n, seed, xcw_val=None):
    if xcw_val is None:
        xcw_val = xcw(a)
    out = np.zeros(n)
    draws = np.zeros(n, np.int32)
    lib().orc_sample_upar(a, x, xcw_val, seed, n, _ptr(out), _ptr(draws, _ip))
    return out, draws


def sample_upar_one(a, x, seed, photon, xcw_val=None):
    """u_par of one photon stream (seed, photon) from its first draw, and the
    draw index after it."""
    if xcw_val is None:
        xcw_val = xcw(a)
    d = ctypes.c_int32()
    u = lib().orc_sample_upar_one(a, x, xcw_val, seed, photon, ctypes.byref(d))
    return u, d.value


def upar_split(a, x, xcw_val=None):
    if xcw_val is None:
        xcw_val = xcw(a)
    u0 = ctypes.c_double()
    p = lib().orc_upar_split(a, abs(x), xcw_val, ctypes.byref(u0))
    return p, u0.value


def atau_jeans(T, n_HI):
    """a*tau of one Jeans length (Sec. 3.2.4, eq. atau0J)."""
    return lib().orc_atau_jeans(float(T), float(n_HI))


def xcrit_at(grid, params, r, k, x):
    """x_crit of an H I scattering at r (cm) moving along k with comoving
    frequency x, as the transport computes it; -1 outside the domain."""
    keep = {}

    def hold(name, arr):
        keep[name] = arr
        return arr
    g = _grid_struct(grid, hold)
    p = _params_struct(dict(params, n_photons=params.get("n_photons", 1)), 0, 1, hold)
    rr = np.ascontiguousarray(r, dtype=np.float64)
    kk = np.ascontiguousarray(k, dtype=np.float64)
    return lib().orc_xcrit_at(ctypes.byref(g), ctypes.byref(p), _ptr(rr), _ptr(kk), float(x))


def scatter_once(T, x, k_in, xcrit=0.0, recoil=True, isotropic=False, seed=1, photon=0):
    """One H I scattering as the transport performs it; returns (x_f, k_f, u_par)."""
    kk = np.ascontiguousarray(k_in, dtype=np.float64)
    xf, up = ctypes.c_double(), ctypes.c_double()
    kf = np.zeros(3)
    lib().orc_scatter_once(float(T), float(x), _ptr(kk), float(xcrit), int(bool(recoil)),
                           int(bool(isotropic)), int(seed), int(photon), ctypes.byref(xf),
                           _ptr(kf), ctypes.byref(up))
    return xf.value, kf, up.value


def sample_uperp(xcrit_eff, n, seed):
    out = np.zeros((n, 2))
    lib().orc_sample_uperp(xcrit_eff, seed, n, _ptr(out))
    return out


def sample_mu(rW, n, seed):
    out = np.zeros(n)
    lib().orc_sample_mu(rW, seed, n, _ptr(out))
    return out


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _grid_struct(grid, hold):
    g = _Grid()
    g.kind = int(grid["kind"])
    g.nx, g.ny, g.nz = (int(v) for v in grid.get("shape", (0, 0, 0)))
    g.box_min[:] = [float(v) for v in grid["box_min"]]
    g.box_max[:] = [float(v) for v in grid["box_max"]]
    n_cells = int(np.asarray(grid["n_HI"]).size)
    g.n_nodes = n_cells
    child = grid.get("child")
    if child is not None:
        child = hold("child", np.ascontiguousarray(child, dtype=np.int32))
    g.child = _ptr(child, _ip)
    g.n_HI = _ptr(hold("n", _f64(grid["n_HI"])))
    g.T = _ptr(hold("T", _f64(grid["T"])))
    g.v = _ptr(hold("v", _f64(grid.get("v"))))
    g.k_dust = _ptr(hold("kd", _f64(grid.get("k_dust"))))
    g.atau_nl = _ptr(hold("nl", _f64(grid.get("atau_nl"))))
    g.dust_albedo = float(grid.get("albedo", 0.0))
    g.escape_radius = float(grid.get("escape_radius", 0.0))
    return g


def nonlocal_atau(grid, f_nl):
    """Non-local a*tau estimate per cell / octree node (Sec. 3.2.4)."""
    keep = {}

    def hold(name, arr):
        keep[name] = arr
        return arr
    g = _grid_struct(grid, hold)
    out = np.zeros(int(np.asarray(grid["n_HI"]).size))
    lib().orc_nonlocal(ctypes.byref(g), float(f_nl), _ptr(out))
    return out


def _params_struct(params, id_begin, id_end, hold):
    p = _Params()
    p.n_photons = int(params["n_photons"])
    p.id_begin = id_begin
    p.id_end = id_end
    p.seed = int(params["seed"])
    p.xcrit_mode = int(params.get("xcrit_mode", 0))
    p.atau0 = float(params.get("atau0", 0.0))
    p.recoil = int(params.get("recoil", 0))
    p.isotropic = int(params.get("isotropic", 0))
    p.n_bins = int(params.get("n_bins", 0))
    p.x_min = float(params.get("x_min", -1.0))
    p.x_max = float(params.get("x_max", 1.0))
    cams = params.get("cam_dir")
    n_cams = 0 if cams is None else int(np.asarray(cams).size // 3)
    p.n_cams = n_cams
    p.cam_dir = _ptr(hold("cams", _f64(cams).reshape(-1) if n_cams else None))
    p.cam_nbins = int(params.get("cam_nbins", 0))
    p.cam_xmin = float(params.get("cam_xmin", -1.0))
    p.cam_xmax = float(params.get("cam_xmax", 1.0))
    p.cam_npix = int(params.get("cam_npix", 0))
    p.cam_fov = float(params.get("cam_fov", 1.0))
    p.tau_peel_max = float(params.get("tau_peel_max", 50.0))
    p.max_events = int(params.get("max_events", 0))
    return p


def run(grid, source, params, id_begin=0, id_end=None, records=False, threads=None,
        variant=""):
    """Runs photons [id_begin, id_end) of a job through the oracle.

    Returns a dict with the escape spectrum (under/overflow at both ends), the
    camera spectra and images (raw sums of W exp(-tau)), the event counters
    and, if ``records``, per-photon final lab x, scattering count, status,
    position, summed peel-off weight per camera and path length travelled (cm).
    """
    n_ph = int(params["n_photons"])
    if id_end is None:
        id_end = n_ph
    n_run = id_end - id_begin
    if threads is None:
        threads = os.cpu_count() or 1
    keep = {}

    def hold(name, arr):
        keep[name] = arr
        return arr

    g = _grid_struct(grid, hold)

    s = _Source()
    pos = hold("pos", _f64(source["pos"]).reshape(-1))
    s.kind = int(source["kind"])
    s.n_src = pos.size // 3
    s.pos = _ptr(pos)
    s.weight = _ptr(hold("w", _f64(source.get("weight"))))
    s.sigma = float(source.get("sigma", 0.0))
    s.freq_mode = int(source.get("freq_mode", 0))

    p = _params_struct(params, id_begin, id_end, hold)
    n_cams = int(p.n_cams)

    o = _Out()
    spectrum = np.zeros(p.n_bins + 2)
    cam_spec = np.zeros((n_cams, p.cam_nbins))
    cam_img = np.zeros((n_cams, p.cam_npix, p.cam_npix))
    o.spectrum = _ptr(spectrum)
    o.cam_spec = _ptr(cam_spec)
    o.cam_img = _ptr(cam_img)
    rec = {}
    if records:
        rec = {"x": np.zeros(n_run), "nscat": np.zeros(n_run, np.int32),
               "status": np.zeros(n_run, np.int32), "pos": np.zeros((n_run, 3)),
               "peel": np.zeros((n_run, max(n_cams, 1))), "len": np.zeros(n_run),
               "ndust": np.zeros(n_run, np.int32)}
        o.rec_x = _ptr(rec["x"])
        o.rec_nscat = _ptr(rec["nscat"], _ip)
        o.rec_status = _ptr(rec["status"], _ip)
        o.rec_pos = _ptr(rec["pos"])
        o.rec_peel = _ptr(rec["peel"]) if n_cams else None
        o.rec_len = _ptr(rec["len"])
        o.rec_ndust = _ptr(rec["ndust"], _ip)
    rc = lib(variant).orc_run(ctypes.byref(g), ctypes.byref(s), ctypes.byref(p),
                              ctypes.byref(o), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle run failed ({rc})")
    counters = {name: int(o.counters[i]) for i, name in enumerate(COUNTER_NAMES)}
    out = {"spectrum": spectrum, "cam_spec": cam_spec, "cam_img": cam_img,
           "counters": counters}
    if records:
        if not n_cams:
            rec["peel"] = rec["peel"][:, :0]
        out["records"] = rec
    return out
