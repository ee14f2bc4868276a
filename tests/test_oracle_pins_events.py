"""Pins of the oracle's per-event arithmetic that the transport's invariants do
not reach: the emission frequency (Sec. 3.1.1, eq. init_freq), the recoil term
of the redistribution (Sec. 3.1.3, eq. x_f with eq. recoil_parameter), the
core-skipping frequency at a scattering (Sec. 3.2.4: eq. xcrit of the local
eq. atau0min, the non-local eq. atauNL and the Jeans eq. atau0J), and the
camera projection and attenuation of the next-event estimator (Sec. 6.1,
eq. SB).

Each expected value comes from outside the oracle: the exact Voigt profile
(scipy's Faddeeva function), physical constants, numbers printed in the paper,
or positions worked out by hand from the geometry of the test.
"""
import math

import numpy as np
import pytest
from scipy import special, stats as sst

import oracle
from paper_1409_4480_amd import inputs

PC = inputs.PC
VTH_REF = 12.85


def empty_box(T=1.0e4, n=8, half=PC, k_dust=0.0, albedo=0.0, n_HI=0.0):
    """A cube of side 2*half holding gas of density n_HI (0: no H I) at T."""
    nc = n ** 3
    return {"kind": 0, "shape": (n, n, n), "box_min": np.full(3, -half),
            "box_max": np.full(3, half), "n_HI": np.full(nc, float(n_HI)),
            "T": np.full(nc, float(T)), "v": None,
            "k_dust": np.full(nc, float(k_dust)) if k_dust > 0 else None,
            "albedo": float(albedo), "escape_radius": 0.0}


# --------------------------------------------------------------------------- #
# Emission frequency, eq. init_freq                                           #
# --------------------------------------------------------------------------- #
def voigt_cdf(a):
    """CDF of the normalised Voigt profile H(a,x)/sqrt(pi), from the exact
    H = Re w(x + i a) integrated on a sinh-spaced grid; the Lorentzian tails
    beyond |x| = 1e4 carry a/(pi 1e4) each and are added analytically."""
    u = np.linspace(-math.asinh(1.0e4), math.asinh(1.0e4), 400001)
    x = np.sinh(u)
    f = special.wofz(x + 1j * a).real / math.sqrt(math.pi)
    tail = a / (math.pi * 1.0e4)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(x))])
    cum = tail + cum
    return lambda t: np.interp(t, x, cum, left=0.0, right=1.0)


@pytest.mark.parametrize("T", [1.0e4, 0.8843])        # a = 4.702e-4 and a = 0.05
def test_emission_frequency_is_the_voigt_profile(threads, T):
    """With no H I every photon leaves unscattered with the frequency it was
    born with.  eq. init_freq draws x = x_nat + k.u_atom, a Lorentzian of
    width a plus the line-of-sight component of a Maxwellian atom velocity
    (variance 1/2 per component): the sum follows H(a,x)/sqrt(pi)."""
    a = oracle.cell_constants(T, 1.0)["a"]
    grid = empty_box(T=T)
    src = {"kind": 0, "pos": np.array([[0.1, -0.2, 0.3]]) * PC, "freq_mode": 1}
    n = 100_000
    params = {"n_photons": n, "seed": 1409448020, "n_bins": 10, "x_min": -5.0, "x_max": 5.0}
    out = oracle.run(grid, src, params, records=True, threads=threads)
    rec = out["records"]
    assert (rec["status"] == 1).all() and (rec["nscat"] == 0).all()
    vth = oracle.cell_constants(T, 1.0)["vth"]
    x = rec["x"] * VTH_REF / vth                      # comoving x (v = 0)
    assert sst.kstest(x, voigt_cdf(a)).pvalue > 1e-3
    # the Gaussian core alone (|x| < 1.5) has the variance of exp(-x^2)
    core = x[np.abs(x) < 1.5]
    g = sst.truncnorm(-1.5 * math.sqrt(2), 1.5 * math.sqrt(2), scale=math.sqrt(0.5))
    if a < 1e-3:
        assert abs(core.var() / g.var() - 1.0) < 0.03


# --------------------------------------------------------------------------- #
# Recoil, eq. x_f and eq. recoil_parameter                                    #
# --------------------------------------------------------------------------- #
def test_recoil_parameter_from_physical_constants():
    """g = h dnu_D / (2 k_B T) = h nu0 / (m_H c v_th) (eq. recoil_parameter)."""
    h, nu0, mH, c_light, kB = 6.62607015e-27, 2.466e15, 1.6735575e-24, 2.99792458e10, 1.380649e-16
    for T in (10.0, 1.0e4):
        vth = math.sqrt(2 * kB * T / mH)
        g = h * nu0 / (mH * c_light * vth)
        assert abs(oracle.cell_constants(T, 1.0)["g"] / g - 1.0) < 2e-3


@pytest.mark.parametrize("x,isotropic", [(0.4, False), (5.0, False), (0.4, True)])
def test_recoil_is_an_energy_loss_of_g_per_scattering(x, isotropic):
    """The recoil term of eq. x_f, g (k_i.k_f - 1), takes energy from the
    photon: scattering the same atom into the same direction with recoil on
    gives a frequency lower by g (1 - mu) in [0, 2g], and for a phase function
    even in mu the mean loss is g (momentum conservation: the atom carries
    away h nu (1 - cos theta) / (m_H c^2) on average with <cos theta> = 0).
    At T = 10 K, g = 8.0e-3."""
    T = 10.0
    g = oracle.cell_constants(T, 1.0)["g"]
    k_in = np.array([0.36, -0.48, 0.8])
    n = 20_000
    d, mus = np.empty(n), np.empty(n)
    for i in range(n):
        xf1, kf1, up1 = oracle.scatter_once(T, x, k_in, recoil=True, isotropic=isotropic,
                                            seed=11, photon=i)
        xf0, kf0, up0 = oracle.scatter_once(T, x, k_in, recoil=False, isotropic=isotropic,
                                            seed=11, photon=i)
        assert up1 == up0 and (kf1 == kf0).all()      # recoil changes no draw
        d[i] = xf1 - xf0
        mus[i] = float(k_in @ kf1)
    assert (d <= 1e-12).all() and (d >= -2 * g - 1e-12).all()
    assert np.allclose(d, -g * (1.0 - mus), rtol=0, atol=1e-12)
    loss = -d.mean()
    se = d.std() / math.sqrt(n)
    assert abs(loss - g) < 4 * se, (loss, g, se)


def test_recoil_reddens_a_cold_slab(threads):
    """Without bulk motion a static slab's spectrum is symmetric about x = 0;
    at low temperature the recoil loss at each scattering shifts the escaping
    photons to the red (the thermal tests of the appendix).  T = 10 K,
    tau0 = 1e4 from the mid-plane, same photons with recoil off and on."""
    wl = inputs.slab(tau0=1.0e4, T=10.0, n_photons=4000, n_xy=16, xcrit_mode=0,
                     x_range=(-60.0, 60.0))
    vth = oracle.cell_constants(10.0, 1.0)["vth"]
    mean, se = {}, {}
    for rec in (0, 1):
        p = dict(wl["params"], recoil=rec)
        r = oracle.run(wl["grid"], wl["source"], p, records=True, threads=threads)["records"]
        x = r["x"][r["status"] == 1] * VTH_REF / vth
        mean[rec], se[rec] = x.mean(), x.std() / math.sqrt(x.size)
    assert abs(mean[0]) < 4 * se[0]
    assert mean[1] < -5 * se[1], (mean, se)


# --------------------------------------------------------------------------- #
# Core-skipping frequency at a scattering, eq. xcrit                          #
# --------------------------------------------------------------------------- #
def xcrit_formula(atau):
    return 0.0 if atau < 1.0 else atau ** (1.0 / 3.0) / 5.0


def local_grid(n_HI=2.0, T=1.0e4, atau_nl=0.0):
    """16^3 cells of 1 pc over [-8, 8) pc; cell (8, 8, 8) spans [0, 1) pc."""
    g = empty_box(T=T, n=16, half=8 * PC, n_HI=n_HI)
    if atau_nl:
        g["atau_nl"] = np.full(16 ** 3, float(atau_nl))
    return g


# (position in the cell [0,1)^3 pc, direction, shortest distance to a face in pc)
LOCAL_CASES = [
    ((0.10, 0.50, 0.50), (1.0, 0.0, 0.0), 0.10),       # exit 0.90 pc away
    ((0.10, 0.50, 0.50), (-1.0, 0.0, 0.0), 0.10),
    ((0.70, 0.35, 0.52), (0.0, 0.6, -0.8), 0.30),      # nearest face on x, exit on z
    ((0.50, 0.93, 0.50), (0.0, -1.0, 0.0), 0.07),      # exit 0.93 pc away
    ((0.45, 0.50, 0.04), (0.0, 0.0, 1.0), 0.04),
]


@pytest.mark.parametrize("pos,k,l_min", LOCAL_CASES)
def test_local_xcrit_uses_the_shortest_distance_to_the_cell_boundary(pos, k, l_min):
    """Local mode: a*tau_cell = 85.56 T4^-1 n_HI l_cell/pc (eq. atau0min, the
    printed coefficient), l_cell the shortest distance from the scattering point
    to the cell boundary whatever the photon's direction, plus the cell's
    non-local a*tau (eq. atauNL)."""
    n_HI = 2.0
    r = np.array(pos) * PC
    k = np.array(k) / np.linalg.norm(k)
    params = {"n_photons": 1, "seed": 1, "xcrit_mode": 2}
    for nl in (0.0, 150.0):
        got = oracle.xcrit_at(local_grid(n_HI, atau_nl=nl), params, r, k, x=0.5)
        want = xcrit_formula(85.56 * n_HI * l_min + nl)
        assert abs(got / want - 1.0) < 1e-3, (pos, nl, got, want)


def test_local_xcrit_limits():
    """Below a*tau = 1 there is no cut-off, nor for a photon in the wing
    (|x| >= x_cw, Sec. 3.2.4); at T = 1e4 K x_cw = 3.26."""
    params = {"n_photons": 1, "seed": 1, "xcrit_mode": 2}
    g = local_grid(2.0)
    k = np.array([1.0, 0.0, 0.0])
    r = np.array([0.004, 0.5, 0.5]) * PC                 # a tau = 0.68
    assert oracle.xcrit_at(g, params, r, k, 0.5) == 0.0
    r = np.array([0.3, 0.5, 0.5]) * PC
    assert oracle.xcrit_at(g, params, r, k, 3.2) > 0.0
    assert oracle.xcrit_at(g, params, r, k, 3.3) == 0.0
    assert oracle.xcrit_at(g, params, r, k, -3.3) == 0.0
    assert oracle.xcrit_at(g, params, np.array([9.0, 0.0, 0.0]) * PC, k, 0.5) == -1.0
    # global mode ignores the position: x_crit(a tau0 = 4702) = 3.3506
    pg = {"n_photons": 1, "seed": 1, "xcrit_mode": 1, "atau0": 4702.0}
    assert abs(oracle.xcrit_at(g, pg, r, k, 0.5) - 3.3506) < 1e-4


def test_jeans_atau_from_the_jeans_length():
    """eq. atau0J: a*tau across one Jeans length lambda_J = (15 k T / (4 pi G mu
    rho))^1/2 of primordial gas (mu = 1.23 m_H, rho = m_H n_HI / X, X = 0.75),
    which the paper gives as 6.428e4 T4^-1/2 n^1/2 and x_crit,J ~ 8 at n = 1,
    T = 1e4 K.  Mode 3 uses it for every scattering of the cell."""
    kB, G, mH = 1.380649e-16, 6.674e-8, 1.6735575e-24
    for T, n in ((1.0e4, 1.0), (1.0e4, 30.0), (500.0, 0.2)):
        rho = mH * n / 0.75
        lam = math.sqrt(15 * kB * T / (4 * math.pi * G * 1.23 * mH * rho))
        c = oracle.cell_constants(T, n)
        assert abs(oracle.atau_jeans(T, n) / (c["a"] * c["k0"] * lam) - 1.0) < 2e-3
    assert abs(oracle.xcrit(oracle.atau_jeans(1.0e4, 1.0)) - 8.0) < 0.05
    params = {"n_photons": 1, "seed": 1, "xcrit_mode": 3}
    k = np.array([0.0, 0.0, 1.0])
    for n_HI in (1.0, 40.0):
        for pos in ((0.5, 0.5, 0.5), (0.01, 0.5, 0.99)):   # independent of the position
            got = oracle.xcrit_at(local_grid(n_HI), params, np.array(pos) * PC, k, 0.2)
            assert abs(got / xcrit_formula(6.428e4 * math.sqrt(n_HI)) - 1.0) < 1e-9


# --------------------------------------------------------------------------- #
# Next-event estimator: projection and attenuation (Sec. 6.1, eq. SB)         #
# --------------------------------------------------------------------------- #
# Image axes of each axis camera: up = +z (+y for the cameras along z),
# u = up x d / |up x d|, v = d x u.  (u, v) of a point (x, y, z) about the
# box centre, worked out by hand for the six axis observers:
AXIS_UV = {(1, 0, 0): lambda x, y, z: (y, z), (-1, 0, 0): lambda x, y, z: (-y, z),
           (0, 1, 0): lambda x, y, z: (-x, z), (0, -1, 0): lambda x, y, z: (x, z),
           (0, 0, 1): lambda x, y, z: (x, y), (0, 0, -1): lambda x, y, z: (-x, y)}


def point_source_job(k_dust=0.0, n_photons=500):
    pos = np.array([0.3, -0.55, 0.8]) * PC
    grid = empty_box(k_dust=k_dust)
    cams = np.array(list(AXIS_UV.keys()), float)
    params = {"n_photons": n_photons, "seed": 5, "n_bins": 4, "x_min": -1.0, "x_max": 1.0,
              "cam_dir": cams, "cam_nbins": 4, "cam_xmin": -1.0, "cam_xmax": 1.0,
              "cam_npix": 10, "cam_fov": 2 * PC, "tau_peel_max": 50.0}
    return grid, {"kind": 0, "pos": pos[None, :], "freq_mode": 0}, params, pos, cams


def test_emission_peel_lands_on_the_projected_pixel(threads):
    """In empty space every photon escapes unscattered and its only next-event
    contribution is the emission's, W = 1 and e^-tau = 1, so each camera image
    holds N in the pixel of the source's orthographic projection and nothing
    else, and the camera spectrum holds N in the bin of x = 0."""
    grid, src, params, pos, cams = point_source_job()
    n = params["n_photons"]
    out = oracle.run(grid, src, params, threads=threads)
    for i, d in enumerate(cams):
        u, v = AXIS_UV[tuple(int(t) for t in d)](*pos)
        iu = int((u / (2 * PC) + 0.5) * 10)
        iv = int((v / (2 * PC) + 0.5) * 10)
        img = out["cam_img"][i]
        assert img[iv, iu] == n, (d, iu, iv, np.argwhere(img))
        assert img.sum() == n
        assert out["cam_spec"][i, 2] == n and out["cam_spec"][i].sum() == n


def test_emission_peel_is_attenuated_by_the_dust_to_the_edge(threads):
    """Grey dust of extinction k_d and albedo 0 around the same source: a
    camera along +-axis sees e^-(k_d s), s the distance from the source to the
    box face that camera looks through, per photon (the emission peel; an
    absorbed photon contributes nothing more, an escaping one only at birth)."""
    kd = 0.7 / PC
    grid, src, params, pos, cams = point_source_job(k_dust=kd, n_photons=300)
    n = params["n_photons"]
    out = oracle.run(grid, src, params, records=True, threads=threads)
    for i, d in enumerate(cams):
        axis = int(np.argmax(np.abs(d)))
        s = PC - pos[axis] * d[axis]                    # to the face at +-1 pc
        assert abs(out["cam_img"][i].sum() / (n * math.exp(-kd * s)) - 1.0) < 1e-12
        assert np.allclose(out["records"]["peel"][:, i], math.exp(-kd * s), rtol=1e-12, atol=0)
