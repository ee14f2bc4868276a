"""Seeded synthetic workloads shaped like the paper's transfer problems.

This module only builds inputs: gas fields on a grid (n_HI, T, bulk velocity,
dust opacity), photon sources, and job options.  It contains none of the
transfer arithmetic, so both the HIP library and the CPU oracle can be fed from
it.  Every generator is deterministic for its seed.

Workloads (sizes as used throughout the tests and the benchmark):

* ``static_sphere``: uniform static H I sphere of line-centre radial optical
  depth tau0 on an N^3 Cartesian grid, central point source at x = 0
  (the analytic sphere of Sec. 3.2.4, eq. sphere).
* ``dusty_sphere``: the same sphere with grey dust (tau_dust = 1, albedo 0.32)
  and global core-skipping.
* ``halo``: idealised first-galaxy halo on a 128^3 grid: n_HI ~ r^-2 between
  1e-2 and 1e2 cm^-3, a bipolar ionised cone (45 degree half-angle, neutral
  fraction 1e-4), radial wind rising linearly to 200 km/s, Gaussian central
  source, eight cameras (Secs. 5.1 and 6.1 in spirit).
* ``nfw_octree``: synthetic cosmological halo on an octree (64^3 base, four
  refinement levels) with NFW density, Kolmogorov turbulence plus Hubble flow
  and 64 Poisson-placed sources (a stand-in for the simulated halo of Sec. 5.2,
  whose data is not available).
* ``job_stream``: a serving stream of uniform and Hubble-expanding spheres
  (Sec. 4.2) with Poisson arrivals.
"""
import numpy as np

PC = 3.0856775814913673e18          # cm
KPC = 1.0e3 * PC
MPC = 1.0e6 * PC
VTH_REF = 12.85                     # km/s, thermal speed at 1e4 K (Sec. 2)
SIGMA0_1E4 = 5.898e-14              # cm^2, line-centre cross section at 1e4 K (Sec. 2)
A_1E4 = 4.702e-4                    # Voigt damping parameter at 1e4 K (Sec. 2)

AXIS_CAMERAS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                        dtype=np.float64)


def _sigma0(T):
    return SIGMA0_1E4 / np.sqrt(T / 1.0e4)


def velocity_window(vmax_kms):
    """Lab-frame x range covering Doppler velocities -vmax..vmax (x = -dv/v_ref)."""
    x = vmax_kms / VTH_REF
    return -x, x


def cell_centres(n, box_min, box_max):
    """Centres of an n^3 Cartesian grid, as three (n, n, n) arrays indexed [z, y, x]."""
    w = (np.asarray(box_max, float) - np.asarray(box_min, float)) / n
    c = [box_min[d] + (np.arange(n) + 0.5) * w[d] for d in range(3)]
    z, y, x = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return x, y, z


def static_sphere(n=16, tau0=1.0e4, T=1.0e4, radius=PC, n_photons=2000,
                  seed=1409448001, n_bins=200, x_range=(-50.0, 50.0), isotropic=True,
                  recoil=False, k_dust=0.0, albedo=0.0, xcrit_mode=0, atau0=None,
                  v_max=0.0, cameras=None, cam_nbins=0, cam_npix=0, freq_mode=0):
    """Uniform sphere of radius `radius` inside an n^3 cube of side 2*radius.

    Every cell holds the same gas, so the escape sphere is exact on the grid.
    n_HI is set so that the line-centre optical depth from the centre to the
    surface is tau0.  A Hubble-like outflow v = v_max r/R (Sec. 4.2) is added
    when v_max != 0.  Dust is grey with extinction k_dust (cm^-1).
    """
    n_HI = tau0 / (_sigma0(T) * radius)
    box_min = np.array([-radius] * 3)
    box_max = np.array([radius] * 3)
    n_cells = n ** 3
    v = None
    if v_max != 0.0:
        x, y, z = cell_centres(n, box_min, box_max)
        v = np.stack([x, y, z], axis=-1).reshape(-1, 3) * (v_max / radius)
    grid = {
        "kind": 0, "shape": (n, n, n), "box_min": box_min, "box_max": box_max,
        "n_HI": np.full(n_cells, n_HI), "T": np.full(n_cells, float(T)), "v": v,
        "k_dust": np.full(n_cells, float(k_dust)) if k_dust > 0 else None,
        "albedo": float(albedo), "escape_radius": float(radius),
    }
    source = {"kind": 0, "pos": np.zeros((1, 3)), "freq_mode": int(freq_mode)}
    if atau0 is None:
        atau0 = A_1E4 / np.sqrt(T / 1.0e4) * tau0
    params = {
        "n_photons": int(n_photons), "seed": int(seed), "xcrit_mode": int(xcrit_mode),
        "atau0": float(atau0), "recoil": int(recoil), "isotropic": int(isotropic),
        "n_bins": int(n_bins), "x_min": float(x_range[0]), "x_max": float(x_range[1]),
        "tau_peel_max": 50.0,
    }
    if cameras is not None:
        params.update({"cam_dir": np.asarray(cameras, float).reshape(-1, 3),
                       "cam_nbins": int(cam_nbins or n_bins), "cam_xmin": float(x_range[0]),
                       "cam_xmax": float(x_range[1]), "cam_npix": int(cam_npix or 16),
                       "cam_fov": 2.0 * radius})
    return {"name": f"static_sphere_{n}_tau{tau0:g}", "grid": grid, "source": source,
            "params": params}


def slab(tau0=1.0e7, T=1.0e4, half_thickness=PC, n_xy=64, n_photons=10_000,
         seed=1409448010, n_bins=400, x_range=(-80.0, 80.0), xcrit_mode=1, cameras=None,
         cam_npix=16):
    """Static uniform slab of line-centre optical depth tau0 from the mid-plane
    to each face (the test of Sec. 4.1): two cells across the thickness and
    n_xy cells across each horizontal direction (box n_xy/2 times wider than
    thick), central point source at x = 0, no recoil, global core-skipping."""
    Z = half_thickness
    n_HI = tau0 / (_sigma0(T) * Z)
    box_min = np.array([-n_xy * Z / 2, -n_xy * Z / 2, -Z])
    box_max = -box_min
    n_cells = n_xy * n_xy * 2
    grid = {"kind": 0, "shape": (n_xy, n_xy, 2), "box_min": box_min, "box_max": box_max,
            "n_HI": np.full(n_cells, n_HI), "T": np.full(n_cells, float(T)), "v": None,
            "k_dust": None, "albedo": 0.0, "escape_radius": 0.0}
    atau0 = A_1E4 / np.sqrt(T / 1.0e4) * tau0
    params = {"n_photons": int(n_photons), "seed": int(seed), "xcrit_mode": int(xcrit_mode),
              "atau0": float(atau0), "recoil": 0, "isotropic": 0, "n_bins": int(n_bins),
              "x_min": float(x_range[0]), "x_max": float(x_range[1]), "tau_peel_max": 50.0}
    if cameras is not None:
        params.update({"cam_dir": np.asarray(cameras, float).reshape(-1, 3),
                       "cam_nbins": int(n_bins), "cam_xmin": float(x_range[0]),
                       "cam_xmax": float(x_range[1]), "cam_npix": int(cam_npix),
                       "cam_fov": float(box_max[0] - box_min[0])})
    return {"name": f"slab_tau{tau0:g}", "grid": grid, "source":
            {"kind": 0, "pos": np.zeros((1, 3)), "freq_mode": 0}, "params": params}


def dusty_sphere(n=64, tau0=1.0e7, n_photons=1_000_000, seed=1409448002, n_bins=500,
                 tau_dust=1.0, albedo=0.32, radius=PC, **kw):
    """Sphere of tau0 = 1e7 with grey dust of optical depth tau_dust over the
    radius, albedo 0.32, global core-skipping from a*tau0, anisotropic
    scattering, no recoil (so the dust-free twin is the analytic sphere)."""
    wl = static_sphere(n=n, tau0=tau0, radius=radius, n_photons=n_photons, seed=seed,
                       n_bins=n_bins, isotropic=False, recoil=False,
                       k_dust=tau_dust / radius, albedo=albedo, xcrit_mode=1, **kw)
    wl["name"] = f"dusty_sphere_{n}_tau{tau0:g}"
    return wl


def halo(n=128, L=200.0 * PC, n_photons=10_000_000, seed=1409448003, n_cams=8,
         npix=256, n_bins=1000, v_wind=200.0, r_wind=100.0 * PC, n_max=1.0e2,
         n_floor=1.0e-2, cone_deg=45.0, x_HI_cone=1.0e-4, f_nl=0.5):
    """Idealised first-galaxy halo: n_HI = n_max min(1, (r/dx)^-2) floored at
    n_floor; cells within cone_deg of the +-z axis are ionised (n_HI times
    x_HI_cone); radial outflow rising linearly to v_wind at r_wind.  Local
    core-skipping with the non-local density threshold f_nl (Sec. 3.2.4)."""
    box_min = np.array([-L / 2] * 3)
    box_max = np.array([L / 2] * 3)
    dx = L / n
    x, y, z = cell_centres(n, box_min, box_max)
    r = np.sqrt(x * x + y * y + z * z)
    nh = n_max * np.minimum(1.0, (np.maximum(r, 1e-30) / dx) ** -2)
    nh = np.maximum(nh, n_floor)
    cos_pol = np.abs(z) / np.maximum(r, 1e-30)
    cone = cos_pol >= np.cos(np.radians(cone_deg))
    nh = np.where(cone, nh * x_HI_cone, nh)
    vr = v_wind * np.minimum(r / r_wind, 1.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        unit = np.stack([x, y, z], axis=-1) / np.maximum(r, 1e-30)[..., None]
    v = (unit * vr[..., None]).reshape(-1, 3)
    grid = {"kind": 0, "shape": (n, n, n), "box_min": box_min, "box_max": box_max,
            "n_HI": nh.reshape(-1), "T": np.full(n ** 3, 1.0e4), "v": v, "k_dust": None,
            "albedo": 0.0, "escape_radius": 0.0, "f_nl": float(f_nl)}
    cams = np.vstack([AXIS_CAMERAS, [1, 1, 1], [1, -1, 0]])[:n_cams].astype(float)
    cams /= np.linalg.norm(cams, axis=1, keepdims=True)
    xlo, xhi = velocity_window(1000.0)
    params = {"n_photons": int(n_photons), "seed": int(seed), "xcrit_mode": 2,
              "atau0": 0.0, "recoil": 1, "isotropic": 0, "n_bins": int(n_bins),
              "x_min": xlo, "x_max": xhi, "cam_dir": cams, "cam_nbins": int(n_bins),
              "cam_xmin": xlo, "cam_xmax": xhi, "cam_npix": int(npix), "cam_fov": float(L),
              "tau_peel_max": 50.0}
    source = {"kind": 1, "pos": np.zeros((1, 3)), "sigma": dx, "freq_mode": 1}
    return {"name": f"halo_{n}", "grid": grid, "source": source, "params": params}


# --------------------------------------------------------------------------- #
# Octree workload                                                             #
# --------------------------------------------------------------------------- #
def gaussian_random_field(n, slope=-11.0 / 3.0, rms=1.0, seed=0):
    """Periodic Gaussian random field on an n^3 grid with P(k) ~ k^slope,
    rescaled to the given rms."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n)[:, None, None]
    ky = np.fft.fftfreq(n)[None, :, None]
    kz = np.fft.rfftfreq(n)[None, None, :]
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    k[0, 0, 0] = np.inf
    fk *= k ** (slope / 2.0)
    f = np.fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2))
    f -= f.mean()
    f *= rms / f.std()
    return f


def _trilinear_periodic(field, u):
    """Periodic trilinear interpolation; u in grid units, shape (m, 3) (x, y, z),
    field indexed [x, y, z]."""
    n = field.shape[0]
    u = u - 0.5
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    out = np.zeros(len(u))
    for dx in (0, 1):
        wx = f[:, 0] if dx else 1 - f[:, 0]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1 - f[:, 1]
            for dz in (0, 1):
                wz = f[:, 2] if dz else 1 - f[:, 2]
                out += wx * wy * wz * field[(i0[:, 0] + dx) % n, (i0[:, 1] + dy) % n,
                                            (i0[:, 2] + dz) % n]
    return out


def build_octree(box_min, size, base_level, max_extra, refine, max_nodes=None):
    """Octree with every node down to `base_level` present, then nodes refined
    while refine(centres, widths, level) is true, up to `max_extra` levels more.

    Returns (child, centre, width, level): child[i] is the index of the first of
    node i's eight children (octant bits x=1, y=2, z=4) or -1 for a leaf.
    Returns None as soon as the tree would exceed `max_nodes` nodes.
    """
    box_min = np.asarray(box_min, float)
    childs, centres, widths, levels = [], [], [], []
    coords = np.zeros((1, 3), np.int64)          # integer coordinates at this level
    start = 0
    octs = np.array([[b & 1, (b >> 1) & 1, (b >> 2) & 1] for b in range(8)], np.int64)
    level = 0
    while True:
        w = size / (1 << level)
        cen = box_min + (coords + 0.5) * w
        m = len(coords)
        if level < base_level:
            split = np.ones(m, bool)
        elif level < base_level + max_extra:
            split = refine(cen, w, level)
        else:
            split = np.zeros(m, bool)
        nxt_start = start + m
        ch = np.full(m, -1, np.int64)
        ns = int(split.sum())
        ch[split] = nxt_start + 8 * np.arange(ns)
        childs.append(ch)
        centres.append(cen)
        widths.append(np.full(m, w))
        levels.append(np.full(m, level, np.int32))
        if ns == 0:
            break
        if max_nodes is not None and nxt_start + 8 * ns > max_nodes:
            return None
        coords = (2 * coords[split][:, None, :] + octs[None, :, :]).reshape(-1, 3)
        start = nxt_start
        level += 1
    return (np.concatenate(childs).astype(np.int32), np.concatenate(centres),
            np.concatenate(widths), np.concatenate(levels))


def nfw_octree(L=4.0 * KPC, base_level=6, max_extra=4, r_vir=600.0 * PC, conc=5.0,
               tau0_max=1.0e8, leaves_target=(1.9e6, 2.1e6), turb_n=256, turb_rms=20.0,
               hubble=2139.6, n_src=64, n_photons=10_000_000, seed=1409448004,
               n_bins=1000, npix=512, turb_seed=4480, src_seed=4481, r_floor=1.95 * PC,
               f_nl=0.5):
    """Synthetic cosmological halo on an octree (stand-in for the simulated
    first galaxy of Sec. 5.2): NFW n_H with concentration `conc`, refined on
    n_H * width^3 until the leaf count lies in `leaves_target`; turbulent
    velocity (k^-11/3, rms turb_rms per component) plus Hubble flow `hubble`
    km/s/Mpc; n_src sources uniform within the scale radius; local
    core-skipping with the non-local density threshold f_nl (Sec. 3.2.4)."""
    r_s = r_vir / conc
    box_min = np.array([-L / 2] * 3)

    def n_of_r(r):
        q = np.maximum(r, r_floor) / r_s
        return 1.0 / (q * (1.0 + q) ** 2)

    # normalise so the largest centre-to-edge axis column gives tau0_max
    rr = np.linspace(0.0, L / 2, 200001)
    prof = n_of_r(rr)
    col = np.sum(0.5 * (prof[1:] + prof[:-1]) * np.diff(rr))
    n_s = tau0_max / (SIGMA0_1E4 * col)

    def refine_with(thr):
        def refine(cen, w, level):
            r = np.linalg.norm(cen, axis=1)
            return n_s * n_of_r(r) * w ** 3 > thr
        return refine

    # bisect the threshold on n_H * width^3 (log space) for the leaf count
    lo, hi = 0.0, 12.0
    tree = None
    cap = int(4 * leaves_target[1])
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        t = build_octree(box_min, L, base_level, max_extra,
                         refine_with(10.0 ** mid * n_s * PC ** 3), max_nodes=cap)
        leaves = np.inf if t is None else int((t[0] < 0).sum())
        if t is not None:
            tree = t
        if leaves_target[0] <= leaves <= leaves_target[1]:
            break
        if leaves > leaves_target[1]:
            lo = mid
        else:
            hi = mid
    child, cen, width, level = tree
    r = np.linalg.norm(cen, axis=1)
    n_HI = n_s * n_of_r(r)
    # turbulence on a periodic grid spanning the box, plus Hubble flow
    v = np.zeros((len(child), 3))
    leaf = child < 0
    u = (cen[leaf] - box_min) / L * turb_n
    for d in range(3):
        f = gaussian_random_field(turb_n, rms=turb_rms, seed=turb_seed + d)
        v[leaf, d] = _trilinear_periodic(f, u)
    v += cen * (hubble / MPC)
    rng = np.random.default_rng(src_seed)
    dirs = rng.standard_normal((n_src, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    src = dirs * (r_s * rng.random(n_src) ** (1.0 / 3.0))[:, None]
    grid = {"kind": 1, "box_min": box_min, "box_max": box_min + L, "child": child,
            "n_HI": n_HI, "T": np.full(len(child), 1.0e4), "v": v, "k_dust": None,
            "albedo": 0.0, "escape_radius": 0.0, "level": level, "f_nl": float(f_nl)}
    cams = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    cams /= np.linalg.norm(cams, axis=1, keepdims=True)
    xlo, xhi = velocity_window(1000.0)
    params = {"n_photons": int(n_photons), "seed": int(seed), "xcrit_mode": 2, "atau0": 0.0,
              "recoil": 1, "isotropic": 0, "n_bins": int(n_bins), "x_min": xlo, "x_max": xhi,
              "cam_dir": cams, "cam_nbins": int(n_bins), "cam_xmin": xlo, "cam_xmax": xhi,
              "cam_npix": int(npix), "cam_fov": float(L), "tau_peel_max": 50.0}
    source = {"kind": 2, "pos": src, "freq_mode": 1}
    return {"name": f"nfw_octree_{base_level}+{max_extra}", "grid": grid, "source": source,
            "params": params, "leaves": int(leaf.sum())}


# --------------------------------------------------------------------------- #
# Serving stream                                                              #
# --------------------------------------------------------------------------- #
def job_stream(n_jobs=512, seed=5, rate=None, n_range=(32, 128), tau_range=(1e4, 1e8),
               ph_range=(1e4, 1e6), vmax_max=200.0, base_seed=1409448500):
    """Serving stream: uniform or Hubble-expanding spheres (probability 1/2
    each) with log-uniform grid size, tau0 and photon count, Poisson arrival
    times at `rate` jobs/s (arrivals all zero when rate is None)."""
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for j in range(n_jobs):
        wind = rng.random() < 0.5
        vmax = rng.uniform(0.0, vmax_max) if wind else 0.0
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))) / 8.0) * 8)
        tau0 = float(np.exp(rng.uniform(np.log(tau_range[0]), np.log(tau_range[1]))))
        nph = int(np.exp(rng.uniform(np.log(ph_range[0]), np.log(ph_range[1]))))
        atau0 = A_1E4 * tau0
        half = 2.5 * 0.931 * atau0 ** (1.0 / 3.0) + 2.0 * vmax / VTH_REF + 5.0
        if rate:
            t += rng.exponential(1.0 / rate)
        wl = static_sphere(n=n, tau0=tau0, n_photons=nph, seed=base_seed + j, n_bins=200,
                           x_range=(-half, half), isotropic=False, recoil=True,
                           xcrit_mode=1, v_max=vmax)
        wl["arrival"] = t
        wl["name"] = f"job{j}"
        jobs.append(wl)
    return jobs
