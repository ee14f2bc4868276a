"""Idealised first-galaxy generator (Sec. 5.1) and observables (Sec. 6.1), on
the CPU: pinned to the numbers the paper prints and to closed forms."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1409_4480_amd import galaxy as gx
from paper_1409_4480_amd import inputs
from paper_1409_4480_amd import observables as ob

MODELS = (1e5, 1e6, 1e7, 1e8)


# --------------------------------------------------------------------------- #
# Galaxy model                                                                 #
# --------------------------------------------------------------------------- #
def test_background_density_and_chi_match_the_printed_scalings():
    # n_IGM ~ 2e-4 ((1+z)/10)^3 cm^-3 and chi = 560 (M/1e7)^1/3 ((1+z)/10)^-1 (Sec. 5.1)
    for z in (9.0, 12.0):
        assert gx.n_igm(z) == pytest.approx(2.0e-4 * ((1 + z) / 10) ** 3, rel=0.07)
        for m in MODELS:
            assert gx.chi(m, z) == pytest.approx(560.0 * (m / 1e7) ** (1 / 3) / ((1 + z) / 10),
                                                 rel=0.01)


def test_edge_radii_of_the_profile_caption():
    """The radial-profile caption gives r_edge = 1.09, 2.35, 5.05, 10.88 kpc for
    the 5-8 models at z = 9; they follow from the exact central density with the
    background density rho_cr Omega_b (1+z)^3 / m_H, i.e. without the hydrogen
    fraction X that the text puts in n_IGM (a reading: the figures used X = 1)."""
    printed = (1.09, 2.35, 5.05, 10.88)
    for m, r in zip(MODELS, printed):
        _, r_edge = gx.core_density(m, 9.0, x_h=1.0)
        assert r_edge / gx.KPC == pytest.approx(r, abs=0.006)


def test_central_density_exact_series_and_mass_integral():
    for m in MODELS:
        n0, r_edge = gx.core_density(m, 9.0)
        # eq. nH0 is the large-mass expansion: better than ~1e-9 above 1e6 Msun
        rel = abs(gx.core_density_series(m, 9.0) / n0 - 1)
        assert rel < (3e-9 if m <= 1e6 else 1e-9) or m < 1e6
        # the profile integrates back to the mass (numerical quadrature of eq. nHprofile)
        model = gx.Model(f"SE{int(round(math.log10(m)))}", z=9.0)
        f = lambda r: 4 * math.pi * gx.M_H * float(model.n_h(r)) * r * r
        mass = (integrate.quad(f, 0, model.r_core, epsrel=1e-12)[0] +
                integrate.quad(f, model.r_core, r_edge, epsrel=1e-12, limit=200)[0]) / gx.M_SUN
        assert mass == pytest.approx(m, rel=1e-9)
        assert gx.total_mass_msun(n0, 9.0) == pytest.approx(m, rel=1e-12)
        # leading orders: n0 ~ chi^2 n_IGM, r_edge ~ chi r_core
        c = gx.chi(m, 9.0)
        assert n0 / gx.n_igm(9.0) == pytest.approx(c * c, rel=2.0 / c)
        assert r_edge / gx.R_CORE == pytest.approx(c, rel=1.0 / c)


def test_jeans_and_stromgren_lengths():
    # lambda_J = 0.75 kpc T4^1/2 n^-1/2 (Sec. 3.2.4); R_S = 15 pc at N51 = n100 = T4 = 1
    assert gx.jeans_length(1.0) / gx.KPC == pytest.approx(0.75, rel=0.01)
    assert gx.jeans_length(100.0, T=4e4) / gx.KPC == pytest.approx(0.075 * 2, rel=0.01)
    assert gx.stromgren_radius(1e51, 100.0) / gx.PC == pytest.approx(15.0, rel=0.02)
    assert gx.stromgren_radius(8e51, 100.0) / gx.stromgren_radius(1e51, 100.0) == \
        pytest.approx(2.0, rel=1e-12)


def test_wind_law_and_gradient():
    r = np.array([0.5, 1.0, 4.0, 1e6]) * gx.R_STAR
    v = gx.wind_speed(r)
    assert v[0] == 0 and v[1] == 0
    assert v[2] == pytest.approx(gx.V_INF * math.sqrt(0.75), rel=1e-12)
    assert v[3] == pytest.approx(gx.V_INF, rel=1e-6)
    rr = np.geomspace(1.01, 100.0, 50) * gx.R_STAR
    h = 1e-6 * rr
    fd = (gx.wind_speed(rr + h) - gx.wind_speed(rr - h)) / (2 * h)
    assert np.allclose(gx.wind_gradient(rr), fd, rtol=1e-5)


def test_ionised_regions_and_fields():
    early, late = gx.Model("SE6"), gx.Model("WL6")
    on_axis = np.array([[0, 0, 0.5 * late.r_edge]])
    equator = np.array([[0.5 * late.r_edge, 0, 0]])
    centre = np.array([[0.2 * early.r_core, 0, 0]])
    assert early.n_hi(centre)[0] == 0 and early.n_hi(on_axis)[0] > 0
    assert late.n_hi(on_axis)[0] == 0 and late.n_hi(equator)[0] > 0
    assert late.n_hi(np.array([[0, 0, 1.5 * late.r_edge]]))[0] == pytest.approx(late.n_igm)
    # 30 degree half-angle: just inside and just outside the cone
    t_in, t_out = math.radians(29.0), math.radians(31.0)
    r = 0.3 * late.r_edge
    assert late.n_hi(np.array([[r * math.sin(t_in), 0, r * math.cos(t_in)]]))[0] == 0
    assert late.n_hi(np.array([[r * math.sin(t_out), 0, r * math.cos(t_out)]]))[0] > 0
    v = late.velocity(equator)[0]
    assert v[1] == 0 and v[2] == 0 and v[0] == pytest.approx(gx.wind_speed(0.5 * late.r_edge))
    assert np.all(early.velocity(equator) == 0)


def test_refinement_criteria_hold_on_the_tree():
    m = gx.Model("WL5")
    factors = (8, 4, 8, 64)
    base, extra = 3, 5
    wl = m.workload(base_level=base, max_extra=extra, factors=factors, n_photons=1)
    g = wl["grid"]
    child, level, cen, width = g["child"], g["level"], wl["centres"], wl["widths"]
    L = g["box_max"][0] - g["box_min"][0]
    assert np.allclose(width, L / 2.0 ** level, rtol=1e-15)
    flags = np.array([m.refine(cen[i:i + 1], width[i], *factors)[0]
                      for i in range(len(child))])
    leaf = child < 0
    deep = level >= base + extra
    # every leaf above the deepest level meets every criterion; every refined node
    # below the base levels violated one
    assert not np.any(flags[leaf & ~deep])
    assert np.all(flags[~leaf & (level >= base)])
    assert np.all(g["n_HI"] >= 0) and wl["leaves"] == leaf.sum()


def test_model_names():
    for bad in ("XE5", "SZ5", "SE9", "SE"):
        with pytest.raises(ValueError):
            gx.Model(bad)


# --------------------------------------------------------------------------- #
# Observables                                                                  #
# --------------------------------------------------------------------------- #
def test_luminosity_distance_closed_forms():
    # Einstein-de Sitter: d_L = (2c/H0)(1+z)(1 - (1+z)^-1/2)
    for z in (0.5, 3.0, 9.0):
        eds = 2 * ob.C_KMS / 70.0 * (1 + z) * (1 - (1 + z) ** -0.5) * inputs.MPC
        assert ob.luminosity_distance(z, h0=70.0, om=1.0, ol=0.0) == pytest.approx(eds, rel=1e-9)
    # low redshift: c z / H0 (1 + (1 - q0) z / 2), q0 = om / 2 - ol
    z = 1e-3
    q0 = gx.OMEGA_M / 2 - gx.OMEGA_L
    lin = ob.C_KMS * z / gx.H0_KMS_MPC * (1 + (1 - q0) * z / 2) * inputs.MPC
    assert ob.luminosity_distance(z) == pytest.approx(lin, rel=1e-6)
    assert ob.angular_diameter_distance(9.0) == pytest.approx(
        ob.luminosity_distance(9.0) / 100.0, rel=1e-14)


def test_surface_brightness_forms_and_flux():
    rng = np.random.default_rng(3)
    img = rng.random((32, 32))
    n_ph, L, z, fov = 1e6, 3.9e8 * gx.L_SUN, 9.0, 20.0 * gx.KPC
    sb = ob.sb_image(img, n_ph, L, z, fov)
    # the footnote's units and eq. SB's defining form agree (d_L = (1+z)^2 d_A)
    assert np.allclose(sb, ob.sb_image_direct(img, n_ph, L, z, fov), rtol=1e-10)
    # surface brightness summed over the pixels' solid angle is the flux
    omega = (fov / 32 / ob.angular_diameter_distance(z)) ** 2 * ob.ARCSEC_PER_RAD ** 2
    assert (sb * omega).sum() == pytest.approx(ob.line_flux(img, n_ph, L, z), rel=1e-10)
    # f_lambda integrates over observed wavelength to the same flux
    spec = rng.random(200)
    x0, x1 = -40.0, 40.0
    f_lam = ob.flux_density(spec, n_ph, L, z, x0, x1)
    dlam_obs = (1 + z) * ob.rest_bin_widths(x0, x1, 200)
    assert (f_lam * dlam_obs).sum() == pytest.approx(ob.line_flux(spec, n_ph, L, z), rel=1e-12)


def test_half_light_radius_and_profile_of_a_gaussian():
    n, fov, s = 512, 40.0, 3.0
    c = (np.arange(n) + 0.5) / n * fov - fov / 2
    X, Y = np.meshgrid(c, c)
    img = np.exp(-(X ** 2 + Y ** 2) / (2 * s * s))
    # a circular Gaussian encloses half its light within s (2 ln 2)^1/2
    assert ob.half_light_radius(img, fov) == pytest.approx(s * math.sqrt(2 * math.log(2)),
                                                           rel=2e-3)
    r, prof = ob.radial_profile(img, fov, n_rings=40, r_max=12.0)
    assert np.allclose(prof, np.exp(-r ** 2 / (2 * s * s)), atol=0.01)
    rr, frac = ob.enclosed_light(img, fov)
    assert frac[-1] == pytest.approx(1.0) and np.all(np.diff(frac) >= 0)


def test_red_blue_ratio_and_flux_ratio():
    x0, x1, n = -50.0, 50.0, 100
    sym = np.exp(-np.linspace(-49.5, 49.5, n) ** 2 / 200)
    assert ob.red_blue_ratio(sym, x0, x1) == pytest.approx(1.0, rel=1e-12)
    red_only = np.where(np.linspace(-49.5, 49.5, n) < 0, 1.0, 0.0)
    assert ob.red_blue_ratio(red_only, x0, x1) == math.inf
    # a bin straddling x = 0 is shared by width
    assert ob.red_blue_ratio(np.array([1.0, 0.0, 0.0]), -1.0, 5.0) == pytest.approx(1.0)
    assert ob.red_blue_ratio(np.array([1.0, 1.0, 0.0]), -1.0, 5.0) == pytest.approx(1 / 3)
    assert ob.flux_ratio_to_average(np.full(10, 0.1), 1000, 1.0) == pytest.approx(1.0)


def test_gunn_peterson_red_wing():
    assert ob.tau_gp_centre(9.0) == pytest.approx(7.0e5)
    # away from resonance R_alpha^2 x^6 is negligible and the integral has the
    # closed form x^9/2/(1-x) + 9/7 x^7/2 + 9/5 x^5/2 + 3 x^3/2 + 9 x^1/2
    #                 - 9/2 ln[(1 + x^1/2)/(1 - x^1/2)]
    def prim(x):
        q = math.sqrt(x)
        return (x ** 4.5 / (1 - x) + 9 / 7 * x ** 3.5 + 9 / 5 * x ** 2.5 + 3 * x ** 1.5 +
                9 * q - 4.5 * math.log((1 + q) / (1 - q)))
    z_em, z_i, z_rei = 9.0, 8.9, 6.0
    for dv in (100.0, 300.0, 1000.0):
        lam = ob.LAMBDA_ALPHA_CM * (1 + z_em) * (1 + dv / ob.C_KMS)
        x_rei = (1 + z_rei) * ob.LAMBDA_ALPHA_CM / lam
        x_i = (1 + z_i) * ob.LAMBDA_ALPHA_CM / lam
        closed = ob.tau_gp_centre(z_em) * ob.R_ALPHA / math.pi * \
            (ob.LAMBDA_ALPHA_CM * (1 + z_em) / lam) ** 1.5 * (prim(x_i) - prim(x_rei))
        assert ob.tau_gp_red(lam, z_em, z_i, z_rei) == pytest.approx(closed, rel=1e-7)
    # farther red means less damping; a bigger H II region means less damping
    t = ob.tau_gp_red(ob.LAMBDA_ALPHA_CM * (1 + z_em) * (1 + np.array([100, 500, 2000]) /
                                                         ob.C_KMS), z_em, z_i, z_rei)
    assert np.all(np.diff(t) < 0)
    lam = ob.LAMBDA_ALPHA_CM * (1 + z_em) * (1 + 200 / ob.C_KMS)
    assert ob.tau_gp_red(lam, z_em, 8.5, z_rei) < ob.tau_gp_red(lam, z_em, 8.9, z_rei)
    tr = ob.igm_transmission(np.array([-20.0, -5.0]), z_em, z_i, z_rei)
    assert np.all((tr > 0) & (tr < 1)) and tr[0] > tr[1]
