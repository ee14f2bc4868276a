"""Parity of the HIP transport library with the FP64 CPU oracle.

FP64 mode follows the same written draw-order contract as the oracle, so each
photon's history is the same: identical scattering counts and status, and final
frequencies and positions equal to accumulated rounding.  Rounding differs
between the two (library transcendentals, fused multiply-adds, cm versus
cell-width units) and some steps amplify it: a direction drawn with mu close to
+-1 is only defined to sqrt(ulp) ~ 1e-8 rad, and local core-skipping makes the
frequency depend on the distance to the nearest face.  Long histories can
therefore flip a branch and continue differently.  How many do is a property
of the workload, measured on the oracle itself (tests/rounding.py: the same
photons with fused multiply-adds on a translated box); the allowed fraction is
derived from that measurement, with FLIP as the floor.  Whole-job results are
held to the statistical bar: spectra chi^2 p > 0.01, escape fraction within
3 sigma.  FP32-bulk mode is checked statistically.
"""
import math
import sys

import numpy as np
import pytest
from scipy import stats as sst

import oracle
from paper_1409_4480_amd import colt, inputs
from tests import stats
from tests.rounding import flip_tolerance, self_divergence

pytestmark = pytest.mark.gpu

PC = inputs.PC
FLIP = 0.005          # floor of the fraction of histories allowed to diverge by a branch flip
X_ATOL = 1e-5         # Doppler widths
POS_RTOL = 1e-6       # of the box size


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_grid(grid):
    """The grid as the oracle sees it: a non-local threshold f_nl is turned
    into the oracle's own per-cell estimate."""
    f_nl = float(grid.get("f_nl", 0.0))
    if f_nl > 0.0 and grid.get("atau_nl") is None:
        grid = dict(grid, atau_nl=oracle.nonlocal_atau(grid, f_nl))
    return grid


def run_both(wl, precision=colt.FP64, id_range=None, **kw):
    say(f"[gpu] {wl.get('name', '?')} precision={precision} n={wl['params']['n_photons']}")
    g = colt.run(wl, precision=precision, record=True, **kw)
    lo, hi = id_range if id_range else (0, wl["params"]["n_photons"])
    r = oracle.run(oracle_grid(wl["grid"]), wl["source"], wl["params"], id_begin=lo,
                   id_end=hi, records=True)
    return g, r


def measured_flip(wl, lo=0, hi=None):
    """Allowed diverging fraction for photons [lo, hi) of a workload, from the
    oracle's own divergence under a rounding perturbation."""
    hi = wl["params"]["n_photons"] if hi is None else hi
    d = self_divergence(oracle_grid(wl["grid"]), wl["source"], wl["params"], lo, hi)
    tol = flip_tolerance(d, hi - lo, FLIP)
    say(f"    oracle self-divergence {d:.4f}: diverging fraction allowed {tol:.4f}")
    return tol


def compare_records(g, r, box, lo=0, hi=None, peel=False, flip=FLIP):
    gr = {k: v[lo:hi] for k, v in g["records"].items()}
    rr = r["records"]
    same = (gr["nscat"] == rr["nscat"]) & (gr["status"] == rr["status"])
    say(f"    identical histories: {same.sum()} of {len(same)}")
    assert same.mean() >= 1.0 - flip, f"only {same.mean():.4f} of histories match"
    close = (np.abs(gr["x"] - rr["x"]) <= X_ATOL) & \
        (np.abs(gr["pos"] - rr["pos"]).max(axis=1) <= POS_RTOL * box)
    if peel:
        close &= np.all(np.isclose(gr["peel"], rr["peel"], rtol=1e-5, atol=1e-12), axis=1)
    assert (same & ~close).sum() <= flip * len(same), \
        f"{(same & ~close).sum()} histories with equal counts end apart"
    return same & close


def statistically_equal(g, r, n):
    """Whole-job parity: escape fraction within 3 sigma, spectra chi^2 p > 0.01."""
    fe_g, fe_r = g["counters"]["escaped"] / n, r["counters"]["escaped"] / n
    se = math.sqrt(max(fe_g * (1 - fe_g) + fe_r * (1 - fe_r), 1e-30) / n)
    assert abs(fe_g - fe_r) <= 3 * se + 1e-12
    assert stats.chi2_two_hist_p(g["spectrum"], r["spectrum"]) > 0.01


# --------------------------------------------------------------------------- #
# Building blocks                                                             #
# --------------------------------------------------------------------------- #
def test_device_uniforms_are_the_oracle_stream():
    n, m = 70, 9
    u = colt.sample("uniform", n, seed=0x123456789, p0=m)
    ref = np.array([[oracle.uniform(0x123456789, i, k) for k in range(m)] for i in range(n)])
    assert np.array_equal(u, ref)
    # FP32 stream: word k % 4 of counter block k / 4, u = float(w) 2^-32 + 2^-33
    u32 = colt.sample("uniform", n, seed=77, p0=m, precision=colt.FP32_BULK)
    for i in range(n):
        for k in range(m):
            w = oracle.philox([k // 4, 0, i, 0], [77, 0])[k % 4]
            exp = np.float32(np.float32(w) * np.float32(2.0 ** -32) + np.float32(2.0 ** -33))
            assert u32[i, k] == float(exp)


@pytest.mark.parametrize("prec", [colt.FP64, colt.FP32_BULK])
def test_scattering_draws_are_the_stream(prec):
    """The five draws of a scattering, which FP32 takes from two generator
    blocks computed together when they start on a block boundary (skip a
    multiple of 4) and one by one otherwise, are draws skip .. skip+4 of the
    photon's stream."""
    n = 200
    for skip in (0, 4, 8, 1, 2, 3, 6):
        d = colt.sample("scatter_draws", n, seed=0x5EED + skip, p0=skip, precision=prec)
        u = colt.sample("uniform", n, seed=0x5EED + skip, p0=skip + 5, precision=prec)
        assert np.array_equal(d, u[:, skip:skip + 5]), skip


def test_device_voigt_matches_oracle():
    a = np.concatenate([np.full(4000, 4.702e-4), np.full(2000, 0.047)])
    x = np.concatenate([np.linspace(-30, 30, 4000), np.linspace(0, 8, 2000)])
    ref = oracle.H(a, x)
    h64 = colt.eval_voigt(a, x, colt.FP64)
    assert np.allclose(h64, ref, rtol=1e-13, atol=0)
    h32 = colt.eval_voigt(a, x, colt.FP32_BULK)
    assert np.allclose(h32, ref, rtol=2e-5, atol=1e-30)


@pytest.mark.parametrize("x", [0.3, 1.0, 2.5, 3.0, 4.6, 8.9, -9.5, -2.0])
@pytest.mark.parametrize("how", ["upar", "upar_seq"])
def test_device_upar_fp64_is_the_oracle_sampler(x, how):
    """The wave-cooperative sampler returns exactly the sequential result."""
    a = 4.702e-4
    xcw = oracle.xcw(a)
    u, d = colt.sample(how, 3000, seed=5, p0=a, p1=x, p2=xcw)
    ru, rd = oracle.sample_upar(a, x, 3000, seed=5, xcw_val=xcw)
    assert np.array_equal(d, rd)
    assert np.allclose(u, ru, rtol=1e-10, atol=1e-12)


def test_device_upar_cooperative_mixed_requests():
    """Requests of all three regimes interleaved within each wave, n ragged."""
    a, xcw, n = 4.702e-4, oracle.xcw(4.702e-4), 2999
    u, d = colt.sample("upar_mixed", n, seed=17, p0=a, p1=0.2, p2=xcw)
    assert np.all(d > 0)
    for i in range(n):
        x = 0.2 + 0.41 * (i % 23) * (-1.0 if i & 1 else 1.0)
        ru, rd = oracle.sample_upar_one(a, x, 17, i, xcw_val=xcw)
        assert d[i] == rd and abs(u[i] - ru) <= 1e-10 * max(1.0, abs(u[i])), i
    # FP32 evaluates two candidates per generator block; the cooperative result
    # is still the sequential one, bit for bit, with the same stream advance
    for prec in (colt.FP64, colt.FP32_BULK):
        uc, dc = colt.sample("upar_mixed", n, seed=17, p0=a, p1=0.2, p2=xcw, precision=prec)
        us, ds = colt.sample("upar_mixed_seq", n, seed=17, p0=a, p1=0.2, p2=xcw,
                             precision=prec)
        assert np.all(dc > 0)
        assert np.array_equal(dc, ds) and np.array_equal(uc, us)


@pytest.mark.parametrize("x", [0.0, 1.5, 3.0, 3.5, 6.0, -12.0])
def test_device_upar_fp32_distribution(x):
    a = 4.702e-4
    u, d = colt.sample("upar", 100000, seed=8, p0=a, p1=x, p2=oracle.xcw(a),
                       precision=colt.FP32_BULK)
    if abs(x) >= 9:
        assert sst.kstest(u, "norm", args=(1 / x, math.sqrt(0.5))).pvalue > 1e-3
    else:
        assert stats.ks_p(u, stats.upar_cdf_factory(a, x)) > 1e-3


@pytest.mark.parametrize("prec", [colt.FP64, colt.FP32_BULK])
def test_device_uperp_and_mu(prec):
    s = colt.sample("uperp", 50000, seed=3, p0=3.35, precision=prec)
    r2 = (s ** 2).sum(axis=1) - 3.35 ** 2
    assert sst.kstest(r2, "expon").pvalue > 1e-3
    if prec == colt.FP64:
        assert np.allclose(s, oracle.sample_uperp(3.35, 50000, seed=3), rtol=1e-12, atol=1e-13)
    for rW in (0.0, 3.0 / 11.0, 1.0):
        mu = colt.sample("mu", 50000, seed=4, p0=rW, precision=prec)
        assert np.all(np.abs(mu) <= 1)
        assert stats.ks_p(mu, stats.mu_cdf_factory(rW)) > 1e-3
        if prec == colt.FP64:
            assert np.allclose(mu, oracle.sample_mu(rW, 50000, seed=4), rtol=0, atol=1e-13)


def test_grid_setup_matches_oracle_cell_constants():
    wl = inputs.halo(n=16, n_photons=1)
    wl["grid"]["T"] = np.geomspace(10.0, 1e5, 16 ** 3)
    wl["grid"]["k_dust"] = np.linspace(0, 1e-20, 16 ** 3)
    g = colt.Grid(wl["grid"])
    f = g.fields()
    g.release()
    for i in range(0, 16 ** 3, 97):
        c = oracle.cell_constants(wl["grid"]["T"][i], wl["grid"]["n_HI"][i])
        assert abs(f[i, 0] / c["k0"] - 1) < 1e-13
        assert abs(f[i, 1] / c["a"] - 1) < 1e-14
        assert abs(f[i, 2] / c["vth"] - 1) < 1e-14
        assert np.allclose(f[i, 3:6], wl["grid"]["v"][i] / c["vth"], rtol=1e-14, atol=1e-14)
        assert abs(f[i, 6] - wl["grid"]["k_dust"][i]) <= 1e-14 * max(abs(f[i, 6]), 1e-300)
        assert abs(f[i, 7] / c["xcw"] - 1) < 1e-14
        assert abs(f[i, 8] / c["g"] - 1) < 1e-14


# --------------------------------------------------------------------------- #
# Transport, FP64: photon-by-photon against the oracle                         #
# --------------------------------------------------------------------------- #
def test_static_sphere_16_tau1e4_parity():
    """Static uniform sphere, 16^3, tau0 = 1e4, 2000 photons, isotropic."""
    wl = inputs.static_sphere()
    g, r = run_both(wl)
    compare_records(g, r, 2 * PC)
    assert g["counters"]["escaped"] == 2000 == r["counters"]["escaped"]
    for k in ("emitted", "escaped", "absorbed"):
        assert g["counters"][k] == r["counters"][k]
    assert abs(g["counters"]["scat_hi"] / r["counters"]["scat_hi"] - 1) < 1e-3
    assert np.abs(g["spectrum"] - r["spectrum"]).sum() <= 4


def test_dusty_sphere_core_skip_parity():
    """Dust (tau_d = 1, albedo 0.32) and global core-skipping, ragged count."""
    wl = inputs.dusty_sphere(n=16, tau0=1e6, n_photons=1537, seed=7)
    g, r = run_both(wl)
    compare_records(g, r, 2 * PC)
    c, rc = g["counters"], r["counters"]
    assert c["escaped"] + c["absorbed"] == c["emitted"] == 1537
    assert abs(c["escaped"] - rc["escaped"]) <= 3
    assert abs(c["scat_dust"] / max(rc["scat_dust"], 1) - 1) < 0.01


def test_halo_cameras_local_core_skip_parity():
    """Halo with cone, wind, Gaussian source, Voigt emission, recoil, local
    core-skipping and eight cameras, on a 32^3 grid (central density lowered
    to 0.03 cm^-3 so the oracle finishes in about a second)."""
    wl = inputs.halo(n=32, n_photons=300, npix=16, n_bins=200, seed=33, n_max=0.03,
                     n_floor=1e-4, f_nl=0.0)
    g, r = run_both(wl)
    compare_records(g, r, 200 * PC, peel=True, flip=measured_flip(wl))
    statistically_equal(g, r, 300)
    tot_g, tot_r = g["cam_spec"].sum(axis=1), r["cam_spec"].sum(axis=1)
    assert np.allclose(tot_g, tot_r, rtol=0.02)
    assert np.allclose(g["cam_img"].sum(axis=(1, 2)), r["cam_img"].sum(axis=(1, 2)), rtol=0.02)


def test_octree_nfw_parity():
    """Octree (8^3 base + 2 levels) with NFW gas, turbulence, 64 sources."""
    wl = inputs.nfw_octree(base_level=3, max_extra=2, leaves_target=(2500, 3500), turb_n=16,
                           n_photons=200, npix=16, n_bins=100, tau0_max=1e5)
    g, r = run_both(wl)
    compare_records(g, r, 4000 * PC, peel=True, flip=measured_flip(wl))
    statistically_equal(g, r, 200)
    # camera flux per photon: means agree within the Monte-Carlo error
    gp, rp = g["records"]["peel"], r["records"]["peel"]
    for i in range(gp.shape[1]):
        se = math.sqrt((gp[:, i].var() + rp[:, i].var()) / gp.shape[0]) + 1e-300
        assert abs(gp[:, i].mean() - rp[:, i].mean()) < 3 * se


def test_octree_crossings_match_the_oracle_without_core_skipping():
    """Octree with NFW gas, turbulence and 64 sources, no core-skipping (so no
    position-dependent branch): FP64 histories, camera sums included, equal
    the oracle's, whose octree crossings search from the root while the device
    follows its per-leaf neighbour links."""
    wl = inputs.nfw_octree(base_level=3, max_extra=3, leaves_target=(4000, 9000), turb_n=16,
                           n_photons=400, npix=16, n_bins=100, tau0_max=3e3)
    wl["params"]["xcrit_mode"] = 0
    g, r = run_both(wl)
    ok = compare_records(g, r, 4000 * PC, peel=True)
    say(f"    crossings: device {g['counters']['crossings']}, oracle {r['counters']['crossings']}")
    assert g["counters"]["crossings"] > 20 * 400
    assert abs(g["counters"]["crossings"] - r["counters"]["crossings"]) <= \
        FLIP * r["counters"]["crossings"]
    assert ok.mean() >= 1.0 - FLIP


def test_nonlocal_estimate_matches_oracle():
    """Device non-local a*tau (Sec. 3.2.4) against the oracle, Cartesian halo
    and NFW octree (per leaf)."""
    for wl in (inputs.halo(n=32, n_photons=1),
               inputs.nfw_octree(base_level=3, max_extra=2, leaves_target=(2500, 3500),
                                 turb_n=16, n_photons=1)):
        g = colt.Grid(wl["grid"])          # computes the estimate for f_nl = 0.5
        f = g.fields()
        g.release()
        ref = oracle.nonlocal_atau(wl["grid"], 0.5)
        if wl["grid"]["kind"] == 1:
            ref = ref[np.asarray(wl["grid"]["child"]) < 0]
        assert ref.max() > 1.0
        assert np.allclose(f[:, 9], ref, rtol=1e-11, atol=1e-14)


def test_halo_nonlocal_core_skip_parity():
    """Denser halo (n_max = 0.3 cm^-3) with local + non-local core-skipping."""
    wl = inputs.halo(n=32, n_photons=200, npix=16, n_bins=200, seed=35, n_max=0.3,
                     n_floor=1e-4)
    g, r = run_both(wl)
    compare_records(g, r, 200 * PC, peel=True, flip=measured_flip(wl))
    statistically_equal(g, r, 200)


def test_octree_and_cartesian_agree_on_uniform_gas():
    base = inputs.static_sphere(n=16, tau0=3e3, n_photons=400, seed=11, isotropic=False,
                                recoil=True)
    child, cen, width, level = inputs.build_octree(
        base["grid"]["box_min"], 2 * PC, 3, 2,
        lambda c, w_, l: (np.linalg.norm(c, axis=1) < 0.5 * PC) & (c[:, 2] > 0))
    oct_wl = {"grid": {"kind": 1, "box_min": base["grid"]["box_min"],
                       "box_max": base["grid"]["box_max"], "child": child,
                       "n_HI": np.full(len(child), base["grid"]["n_HI"][0]),
                       "T": np.full(len(child), 1e4), "escape_radius": PC},
              "source": base["source"], "params": base["params"], "name": "octree_uniform"}
    a = colt.run(base, record=True)["records"]
    b = colt.run(oct_wl, record=True)["records"]
    same = (a["nscat"] == b["nscat"]) & (a["status"] == b["status"])
    assert same.mean() > 0.99
    assert np.allclose(a["x"][same], b["x"][same], atol=1e-6)


# --------------------------------------------------------------------------- #
# Launch shapes, batching, slicing, edge cases                                #
# --------------------------------------------------------------------------- #
def test_results_independent_of_launch_shape_and_batching():
    wl1 = inputs.static_sphere(n=8, tau0=5e3, n_photons=700, seed=1, isotropic=False)
    wl2 = inputs.dusty_sphere(n=8, tau0=1e5, n_photons=333, seed=2)
    ref1 = colt.run(wl1, record=True)["records"]
    ref2 = colt.run(wl2, record=True)["records"]
    alt1 = colt.run(wl1, record=True, block=64, blocks_per_cu=1)["records"]
    for k in ref1:
        assert np.array_equal(ref1[k], alt1[k]), k
    # where the passes of the wave loop cut the flights does not matter either
    for prec in (colt.FP64, colt.FP32_BULK):
        base = colt.run(wl2, precision=prec, record=True, march_min=1)["records"]
        for mm in (4, 64):
            alt = colt.run(wl2, precision=prec, record=True, march_min=mm)["records"]
            for k in base:
                assert np.array_equal(base[k], alt[k]), (prec, mm, k)
    g1, g2 = colt.Grid(wl1["grid"]), colt.Grid(wl2["grid"])
    j1 = colt.Job(g1, wl1["source"], wl1["params"], record=True)
    j2 = colt.Job(g2, wl2["source"], wl2["params"], record=True)
    # both jobs in one launch, in three slices of at most 250 photons per job
    while j1.status()[0] < 700 or j2.status()[0] < 333:
        colt.transport([j1, j2], photons_per_job=250)
    b1, b2 = j1.tally()["records"], j2.tally()["records"]
    for k in ref1:
        assert np.array_equal(ref1[k], b1[k]), k
        assert np.array_equal(ref2[k], b2[k]), k
    j1.release(); j2.release(); g1.release(); g2.release()


def test_empty_single_and_outside_born_photons():
    wl = inputs.static_sphere(n=8, tau0=1e3, n_photons=0)
    out = colt.run(wl, record=True)
    assert out["spectrum"].sum() == 0 and out["counters"]["emitted"] == 0
    wl = inputs.static_sphere(n=8, tau0=1e3, n_photons=1, seed=9)
    g, r = run_both(wl)
    compare_records(g, r, 2 * PC)
    # a wide Gaussian source puts some photons outside the escape sphere at birth
    wl = inputs.static_sphere(n=8, tau0=1e2, n_photons=500, seed=10)
    wl["source"] = {"kind": 1, "pos": np.zeros((1, 3)), "sigma": 0.8 * PC, "freq_mode": 1}
    g, r = run_both(wl)
    compare_records(g, r, 2 * PC)
    born_out = (r["records"]["nscat"] == 0) & (np.linalg.norm(r["records"]["pos"], axis=1) > PC)
    assert born_out.sum() > 10
    assert g["counters"]["escaped"] == 500


def test_event_cap_stops_photons_and_counts_them():
    wl = inputs.static_sphere(n=8, tau0=1e4, n_photons=200, seed=12)
    out = colt.run(wl, record=True, max_events=50)
    c = out["counters"]
    assert c["capped"] > 0
    assert c["escaped"] + c["absorbed"] + c["capped"] == 200
    assert np.all(out["records"]["nscat"] <= 50)
    assert ((out["records"]["status"] == 3).sum()) == c["capped"]


# --------------------------------------------------------------------------- #
# FP32-bulk: statistical parity                                               #
# --------------------------------------------------------------------------- #
def test_fp32_bulk_static_sphere_statistics():
    wl = inputs.static_sphere(n=16, tau0=1e4, n_photons=4000, seed=21, isotropic=False)
    g = colt.run(wl, precision=colt.FP32_BULK, record=True)
    r = oracle.run(wl["grid"], wl["source"], wl["params"], records=True)
    gx, rx = g["records"]["x"], r["records"]["x"]
    assert sst.ks_2samp(gx, rx).pvalue > 0.01
    gn, rn = g["records"]["nscat"], r["records"]["nscat"]
    se = math.sqrt(gn.var() / len(gn) + rn.var() / len(rn))
    assert abs(gn.mean() - rn.mean()) < 4 * se
    assert stats.chi2_two_hist_p(g["spectrum"], r["spectrum"]) > 0.01


def test_fp32_bulk_dusty_sphere_escape_fraction():
    wl = inputs.dusty_sphere(n=16, tau0=1e6, n_photons=20000, seed=22, tau_dust=0.3)
    g = colt.run(wl, precision=colt.FP32_BULK)
    d = colt.run(wl, precision=colt.FP64)
    n = 20000
    fg, fd = g["counters"]["escaped"] / n, d["counters"]["escaped"] / n
    se = math.sqrt(fg * (1 - fg) / n + fd * (1 - fd) / n)
    assert abs(fg - fd) < 4 * se
    assert stats.chi2_two_hist_p(g["spectrum"], d["spectrum"]) > 0.01
