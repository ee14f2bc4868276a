"""Observables from the transfer tallies (Sec. 6.1), on the host.

The transport library returns, per camera, the sums of W e^-tau_esc over all
next-event contributions binned in frequency and in image pixels, and the
escape spectrum.  This module turns them into the paper's observables:

* surface brightness per pixel (eq. SB), in erg s^-1 cm^-2 arcsec^-2;
* flux density f_lambda and line-of-sight bolometric flux;
* radial surface-brightness profiles, the enclosed light I(r) and the
  half-light radius R_1/2;
* the red-to-blue flux ratio F_r / F_b about line centre and the
  line-of-sight flux relative to the angle average, F / F_Omega
  (table model_bolometric_flux);
* the red damping wing of the Gunn-Peterson trough (eq. tauGP) and the IGM
  transmission it implies.

Frequencies are the library's x (Doppler widths at T_ref = 1e4 K, blue
positive), so the Doppler velocity is dv = -x v_th,ref and red means x < 0.
"""
import math

import numpy as np
from scipy import integrate

from . import galaxy, inputs

C_CMS = 2.99792458e10
C_KMS = 2.99792458e5
LAMBDA_ALPHA_CM = 1215.67e-8          # Lyman-alpha rest wavelength
ARCSEC_PER_RAD = 180.0 / math.pi * 3600.0
R_ALPHA = 2.0e-8                      # Lambda lambda_alpha / (4 pi c) (eq. tauGP)


# --------------------------------------------------------------------------- #
# Cosmological distances (flat universe, the model cosmology of Sec. 5.1)     #
# --------------------------------------------------------------------------- #
def hubble(z, h0=galaxy.H0_KMS_MPC, om=galaxy.OMEGA_M, ol=galaxy.OMEGA_L):
    """H(z) in km/s/Mpc for a flat (om + ol = 1) universe."""
    return h0 * math.sqrt(om * (1.0 + z) ** 3 + ol)


def luminosity_distance(z, h0=galaxy.H0_KMS_MPC, om=galaxy.OMEGA_M, ol=galaxy.OMEGA_L):
    """d_L = (1 + z) int_0^z c dz' / H(z') (cm)."""
    val, _ = integrate.quad(lambda zp: C_KMS / hubble(zp, h0, om, ol), 0.0, z,
                            epsabs=0.0, epsrel=1e-12, limit=200)
    return (1.0 + z) * val * inputs.MPC


def angular_diameter_distance(z, **kw):
    """d_A = d_L / (1 + z)^2 (cm)."""
    return luminosity_distance(z, **kw) / (1.0 + z) ** 2


# --------------------------------------------------------------------------- #
# Frequency bins                                                               #
# --------------------------------------------------------------------------- #
def dv_of_x(x):
    """Doppler velocity (km/s, red positive) of lab-frame x."""
    return -np.asarray(x, float) * inputs.VTH_REF


def bin_edges(x_min, x_max, n_bins):
    return np.linspace(x_min, x_max, n_bins + 1)


def rest_bin_widths(x_min, x_max, n_bins):
    """Rest-frame wavelength width of each frequency bin (cm)."""
    dv = np.abs(np.diff(dv_of_x(bin_edges(x_min, x_max, n_bins))))
    return LAMBDA_ALPHA_CM * dv / C_KMS


# --------------------------------------------------------------------------- #
# Surface brightness and flux (eq. SB and the text after it)                   #
# --------------------------------------------------------------------------- #
def sb_image(img, n_photons, l_lya, z, fov_cm):
    """Surface brightness per pixel (erg s^-1 cm^-2 arcsec^-2) from a camera
    image of summed W e^-tau: L / [4 pi N_ph (1+z)^4 206265^2 l_pix^2] times
    the pixel sum, l_pix the physical pixel size."""
    img = np.asarray(img, float)
    l_pix = fov_cm / img.shape[-1]
    return l_lya / (4.0 * math.pi * n_photons * (1.0 + z) ** 4 * ARCSEC_PER_RAD ** 2 *
                    l_pix ** 2) * img


def sb_image_direct(img, n_photons, l_lya, z, fov_cm):
    """The same from the defining form of eq. SB: L / N_ph / (4 pi d_L^2
    Omega_pix) with Omega_pix = (l_pix / d_A)^2 in arcsec^2."""
    img = np.asarray(img, float)
    l_pix = fov_cm / img.shape[-1]
    d_l = luminosity_distance(z)
    omega = (l_pix / angular_diameter_distance(z)) ** 2 * ARCSEC_PER_RAD ** 2
    return l_lya / n_photons / (4.0 * math.pi * d_l ** 2 * omega) * img


def flux_density(cam_spec, n_photons, l_lya, z, x_min, x_max):
    """f_lambda (erg s^-1 cm^-2 cm^-1, per observed wavelength) of a camera
    spectrum: L / (4 pi N_ph dlambda_obs d_L^2) times the bin sum, with
    dlambda_obs = (1+z) dlambda_bin."""
    spec = np.asarray(cam_spec, float)
    dlam_obs = (1.0 + z) * rest_bin_widths(x_min, x_max, spec.shape[-1])
    return l_lya / (4.0 * math.pi * n_photons * luminosity_distance(z) ** 2) * spec / dlam_obs


def line_flux(cam_spec, n_photons, l_lya, z):
    """Bolometric line-of-sight flux F = integral of f_lambda (erg s^-1 cm^-2)."""
    return l_lya * float(np.sum(cam_spec)) / (4.0 * math.pi * n_photons *
                                              luminosity_distance(z) ** 2)


def flux_ratio_to_average(cam_spec, n_photons, escaped_weight):
    """F / F_Omega: a camera's flux against the isotropic angle average.  The
    camera sums carry W normalised to a 4 pi mean of one, so for any job the
    angle average of cam_sum / N_ph equals the escaped weight / N_ph."""
    return (float(np.sum(cam_spec)) / n_photons) / (escaped_weight / n_photons)


def red_blue_ratio(spec, x_min, x_max):
    """F_r / F_b about line centre: weight at x < 0 (red) over x > 0 (blue);
    a bin containing x = 0 is split in proportion to its width on either side."""
    spec = np.asarray(spec, float)
    edges = bin_edges(x_min, x_max, spec.shape[-1])
    lo, hi = edges[:-1], edges[1:]
    red_share = np.clip((0.0 - lo) / (hi - lo), 0.0, 1.0)
    red = float(np.sum(spec * red_share))
    blue = float(np.sum(spec * (1.0 - red_share)))
    return red / blue if blue > 0 else math.inf


# --------------------------------------------------------------------------- #
# Radial profiles                                                              #
# --------------------------------------------------------------------------- #
def _pixel_radii(npix, fov):
    c = (np.arange(npix) + 0.5) / npix * fov - 0.5 * fov
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.hypot(X, Y)


def radial_profile(img, fov, n_rings=32, r_max=None):
    """Mean of the image in annuli about its centre: (ring centres, means)."""
    img = np.asarray(img, float)
    r = _pixel_radii(img.shape[-1], fov)
    r_max = 0.5 * fov if r_max is None else r_max
    edges = np.linspace(0.0, r_max, n_rings + 1)
    idx = np.digitize(r.ravel(), edges) - 1
    ok = (idx >= 0) & (idx < n_rings)
    sums = np.bincount(idx[ok], weights=img.ravel()[ok], minlength=n_rings)
    cnt = np.bincount(idx[ok], minlength=n_rings)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(cnt > 0, sums / np.maximum(cnt, 1), 0.0)
    return 0.5 * (edges[1:] + edges[:-1]), mean


def enclosed_light(img, fov):
    """I(r): the image's light within radius r about the centre, normalised to
    one; returns (radii sorted, cumulative fraction) over the pixels."""
    img = np.asarray(img, float)
    r = _pixel_radii(img.shape[-1], fov).ravel()
    w = img.ravel()
    order = np.argsort(r, kind="stable")
    cum = np.cumsum(w[order])
    return r[order], cum / cum[-1]


def half_light_radius(img, fov):
    """R_1/2: the radius enclosing half of the image's light."""
    r, frac = enclosed_light(img, fov)
    i = int(np.searchsorted(frac, 0.5))
    if i == 0:
        return float(r[0])
    f0, f1 = frac[i - 1], frac[i]
    t = 0.0 if f1 == f0 else (0.5 - f0) / (f1 - f0)
    return float(r[i - 1] + t * (r[i] - r[i - 1]))


# --------------------------------------------------------------------------- #
# IGM transmission (eq. tauGP)                                                 #
# --------------------------------------------------------------------------- #
def tau_gp_centre(z):
    """Gunn-Peterson optical depth at line centre, 7e5 ((1+z)/10)^3/2."""
    return 7.0e5 * ((1.0 + z) / 10.0) ** 1.5


def tau_gp_red(lambda_obs_cm, z_em, z_i, z_rei, r_alpha=R_ALPHA):
    """eq. tauGP: red damping wing of a neutral IGM between the edge of the
    source's H II region (z_i) and reionisation (z_rei), at observed
    wavelength lambda_obs (cm); x runs from x_rei = (1+z_rei) lambda_a /
    lambda_obs to x_i = (1+z_i) lambda_a / lambda_obs."""
    lam = np.atleast_1d(np.asarray(lambda_obs_cm, float))
    out = np.empty_like(lam)
    for k, lo in enumerate(lam):
        x_rei = (1.0 + z_rei) * LAMBDA_ALPHA_CM / lo
        x_i = (1.0 + z_i) * LAMBDA_ALPHA_CM / lo
        val, _ = integrate.quad(lambda x: x ** 4.5 / ((1.0 - x) ** 2 + r_alpha ** 2 * x ** 6),
                                x_rei, x_i, epsabs=0.0, epsrel=1e-10, limit=400,
                                points=[1.0] if x_rei < 1.0 < x_i else None)
        pre = tau_gp_centre(z_em) * r_alpha / math.pi
        out[k] = pre * (LAMBDA_ALPHA_CM * (1.0 + z_em) / lo) ** 1.5 * val
    return out if np.ndim(lambda_obs_cm) else float(out[0])


def igm_transmission(x, z_em, z_i, z_rei, r_alpha=R_ALPHA):
    """e^-tau_GP^red at the observed wavelengths of lab-frame x emitted at z_em."""
    lam_obs = LAMBDA_ALPHA_CM * (1.0 + z_em) * (1.0 + dv_of_x(x) / C_KMS)
    return np.exp(-np.asarray(tau_gp_red(lam_obs, z_em, z_i, z_rei, r_alpha)))
