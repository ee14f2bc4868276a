"""Idealised first-galaxy models of Sec. 5.1 as transfer inputs.

A model is a spherical hydrogen distribution with a flat core, an isothermal
r^-2 envelope and the neutral IGM outside (eq. nHprofile), normalised to a
total hydrogen mass through the chi parameter (eqs. MHtot, nH0, chi); an
"Early" or "Late" ionised region (a Stromgren sphere of radius r_core, plus for
"Late" a bipolar cone out to r_edge); a static or beta-law wind velocity field
(eq. wind); T = 1e4 K; mapped onto an octree over (-2 r_edge, 2 r_edge)^3 by the
Jeans, Sobolev and geometric refinement criteria of Sec. 5.1.4.  The source's
luminosity is only a normalisation of the tallies (the transfer is scale-free)
and is an argument of the observables.

Classification (table models): S/W (static / wind), E/L (early / late), 5-8
(M_H,tot = 1e5 ... 1e8 Msun); e.g. "WL7".

Like ``inputs``, this module only builds inputs: it holds none of the
transfer arithmetic.
"""
import math

import numpy as np

from . import inputs

# physical constants (cgs)
M_H = 1.6735575e-24          # g
M_SUN = 1.98847e33           # g
L_SUN = 3.828e33             # erg/s
G_NEWTON = 6.67430e-8
K_B = 1.380649e-16
PC = inputs.PC
KPC = inputs.KPC
MPC = inputs.MPC

# cosmology and composition used by the models (Sec. 5.1)
H0_KMS_MPC = 67.8
OMEGA_B = 0.0485
OMEGA_M = 0.307
OMEGA_L = 0.693
X_H = 0.75                   # hydrogen mass fraction
MU_GAS = 1.23                # mean molecular weight of primordial gas, in m_H

R_CORE = 10.0 * PC           # core radius
R_STAR = 1.0 * PC            # size of the central star cluster (wind base)
V_INF = 10.0                 # km/s, wind terminal velocity
THETA_OPEN = 30.0            # degrees, half-angle of the ionised cones ("Late")
N_JEANS = 64                 # cell width x N_J <= Jeans length
N_SOBOLEV = 32               # cell width x N_S <= Sobolev length
N_GEOM = 64                  # cell width x N_G <= r_edge (and r_core) where cut by it
N_CONE = 512                 # cell width x 512 <= r_edge where cut by the cone surface


def h0_per_s():
    return H0_KMS_MPC * 1.0e5 / MPC


def n_igm(z, x_h=X_H):
    """Background hydrogen number density rho_cr,0 x_h Omega_b (1+z)^3 / m_H
    (cm^-3), about 2e-4 ((1+z)/10)^3 with x_h = 0.75."""
    rho_cr = 3.0 * h0_per_s() ** 2 / (8.0 * math.pi * G_NEWTON)
    return rho_cr * x_h * OMEGA_B * (1.0 + z) ** 3 / M_H


def chi(m_h_tot_msun, z, r_core=R_CORE, x_h=X_H):
    """eq. chi: n_IGM^-1/3 / r_core (M_H,tot / 4 pi m_H)^1/3."""
    m = m_h_tot_msun * M_SUN
    return n_igm(z, x_h) ** (-1.0 / 3.0) / r_core * (m / (4.0 * math.pi * M_H)) ** (1.0 / 3.0)


def core_density(m_h_tot_msun, z, r_core=R_CORE, x_h=X_H):
    """Central density n_H,0 solving eq. MHtot exactly: with s = (n0/n_IGM)^1/2
    the mass condition reads s^3 - (2/3) s^2 = chi^3 (one real root above 2/3).
    Returns (n_H0, r_edge) with r_edge = r_core s."""
    c3 = chi(m_h_tot_msun, z, r_core, x_h) ** 3
    s = c3 ** (1.0 / 3.0) + 2.0 / 9.0                 # start near the root
    for _ in range(60):                               # Newton, monotone above 2/3
        f = s ** 3 - (2.0 / 3.0) * s ** 2 - c3
        s_new = s - f / (3.0 * s ** 2 - (4.0 / 3.0) * s)
        if abs(s_new - s) <= 1e-15 * s:
            s = s_new
            break
        s = s_new
    return n_igm(z, x_h) * s * s, r_core * s


def core_density_series(m_h_tot_msun, z, r_core=R_CORE, x_h=X_H):
    """eq. nH0: the large-mass expansion n_IGM (chi^2 + 4 chi / 9 + 4 / 27)."""
    c = chi(m_h_tot_msun, z, r_core, x_h)
    return n_igm(z, x_h) * (c * c + 4.0 * c / 9.0 + 4.0 / 27.0)


def total_mass_msun(n_h0, z, r_core=R_CORE, x_h=X_H):
    """eq. MHtot evaluated for a central density (the integral's closed form)."""
    ni = n_igm(z, x_h)
    return 4.0 * math.pi * M_H * n_h0 * r_core ** 3 * (math.sqrt(n_h0 / ni) - 2.0 / 3.0) / M_SUN


def jeans_length(n_h, T=1.0e4, x_h=X_H):
    """lambda_J = (15 k T / (4 pi G mu rho))^1/2 with rho = m_H n_H / x_h (cm)."""
    rho = M_H * np.asarray(n_h, float) / x_h
    with np.errstate(divide="ignore"):
        return np.sqrt(15.0 * K_B * T / (4.0 * math.pi * G_NEWTON * MU_GAS * M_H * rho))


def stromgren_radius(n_ion_per_s, n0, T=1.0e4):
    """eq. stromgren with alpha_B = 2.5e-13 T4^-3/4 cm^3/s (cm)."""
    alpha_b = 2.5e-13 * (T / 1.0e4) ** -0.75
    return (3.0 * n_ion_per_s / (4.0 * math.pi * n0 * n0 * alpha_b)) ** (1.0 / 3.0)


def wind_speed(r, v_inf=V_INF, r_star=R_STAR):
    """eq. wind: v_inf (1 - R_*/r)^1/2 outside R_*, zero inside (km/s)."""
    r = np.asarray(r, float)
    return np.where(r > r_star, v_inf * np.sqrt(np.clip(1.0 - r_star / np.maximum(r, r_star),
                                                        0.0, None)), 0.0)


def wind_gradient(r, v_inf=V_INF, r_star=R_STAR):
    """|dv/dr| of eq. wind (km/s per cm); infinite at R_*, zero inside."""
    r = np.asarray(r, float)
    out = np.zeros_like(r)
    m = r > r_star
    q = 1.0 - r_star / r[m]
    with np.errstate(divide="ignore"):
        out[m] = v_inf * r_star / (2.0 * r[m] ** 2 * np.sqrt(q))
    return out


class Model:
    """One idealised model: name like "WL7" or explicit parts."""

    def __init__(self, name="WL7", z=9.0, r_core=R_CORE, x_h=X_H, theta_open=THETA_OPEN,
                 v_inf=V_INF, r_star=R_STAR, T=1.0e4):
        name = name.upper()
        if len(name) != 3 or name[0] not in "SW" or name[1] not in "EL" or name[2] not in "5678":
            raise ValueError("model names are [S|W][E|L][5-8]")
        self.name = name
        self.wind = name[0] == "W"
        self.late = name[1] == "L"
        self.m_h_tot = 10.0 ** int(name[2])
        self.z = float(z)
        self.r_core = float(r_core)
        self.x_h = float(x_h)
        self.theta_open = float(theta_open)
        self.v_inf = float(v_inf)
        self.r_star = float(r_star)
        self.T = float(T)
        self.n_igm = n_igm(self.z, self.x_h)
        self.n_h0, self.r_edge = core_density(self.m_h_tot, self.z, self.r_core, self.x_h)
        self.r_s = self.r_core                # Stromgren sphere of radius r_core ("Early")

    # -- fields ----------------------------------------------------------- #
    def n_h(self, r):
        """eq. nHprofile: total hydrogen density (cm^-3)."""
        r = np.asarray(r, float)
        env = self.n_h0 * (np.maximum(r, self.r_core) / self.r_core) ** -2.0
        return np.where(r <= self.r_core, self.n_h0,
                        np.where(r < self.r_edge, env, self.n_igm))

    def ionised(self, pos):
        """True where the model has no neutral hydrogen: the Stromgren sphere,
        and for "Late" also the bipolar cone around z out to r_edge."""
        pos = np.asarray(pos, float)
        r = np.linalg.norm(pos, axis=-1)
        ion = r <= self.r_s
        if self.late:
            cos_t = math.cos(math.radians(self.theta_open))
            cone = (np.abs(pos[..., 2]) >= cos_t * r) & (r < self.r_edge)
            ion = ion | cone
        return ion

    def n_hi(self, pos):
        pos = np.asarray(pos, float)
        r = np.linalg.norm(pos, axis=-1)
        return np.where(self.ionised(pos), 0.0, self.n_h(r))

    def velocity(self, pos):
        """Bulk velocity (km/s, xyz): radial eq. wind for "W", zero for "S"."""
        pos = np.asarray(pos, float)
        if not self.wind:
            return np.zeros_like(pos)
        r = np.linalg.norm(pos, axis=-1)
        v = wind_speed(r, self.v_inf, self.r_star)
        with np.errstate(invalid="ignore", divide="ignore"):
            u = np.where(r[..., None] > 0, pos / np.maximum(r, 1e-300)[..., None], 0.0)
        return u * v[..., None]

    # -- refinement (Sec. 5.1.4) ------------------------------------------ #
    def refine(self, cen, w, n_j=N_JEANS, n_s=N_SOBOLEV, n_g=N_GEOM, n_c=N_CONE):
        """Which cells (centres cen, width w) violate a criterion: Jeans length
        at the densest point of the cell, Sobolev length at its steepest wind
        gradient, the r_edge and r_core spheres and (Late) the cone surface."""
        cen = np.asarray(cen, float)
        h = 0.5 * w
        # distance from the centre to the nearest and farthest point of the cell
        near = np.linalg.norm(np.maximum(np.abs(cen) - h, 0.0), axis=1)
        far = np.linalg.norm(np.abs(cen) + h, axis=1)
        split = w * n_j > jeans_length(self.n_h(near), self.T, self.x_h)
        if self.wind:
            vth = inputs.VTH_REF * math.sqrt(self.T / 1.0e4)
            grad = wind_gradient(np.maximum(near, self.r_star * (1.0 + 1e-12)), self.v_inf,
                                 self.r_star)
            with np.errstate(divide="ignore"):
                lam_s = np.where(grad > 0, vth / np.maximum(grad, 1e-300), np.inf)
            split |= (w * n_s > lam_s) & (far > self.r_star)
        for R in (self.r_edge, self.r_core):          # cut by the sphere of radius R
            split |= (near < R) & (far > R) & (w * n_g > R)
        if self.late:
            cos_t = math.cos(math.radians(self.theta_open))
            corners = cen[:, None, :] + h * np.array(
                [[(b & 1) * 2 - 1, ((b >> 1) & 1) * 2 - 1, ((b >> 2) & 1) * 2 - 1]
                 for b in range(8)], float)[None, :, :]
            f = np.abs(corners[..., 2]) - cos_t * np.linalg.norm(corners, axis=-1)
            apex = near <= 1e-9 * w                   # the cell touches the cone apex
            cut = (f.min(axis=1) < 0) & (f.max(axis=1) > 0) | apex
            split |= cut & (near < self.r_edge) & (w * n_c > self.r_edge)
        return split

    # -- transfer job --------------------------------------------------------#
    def workload(self, base_level=4, max_extra=6, n_photons=100_000, seed=1409448005,
                 factors=(N_JEANS, N_SOBOLEV, N_GEOM, N_CONE), n_bins=400, npix=128,
                 vmax_kms=400.0, max_nodes=8_000_000, f_nl=0.5):
        """Octree workload over (-2 r_edge, 2 r_edge)^3: `base_level` uniform
        levels, then up to `max_extra` more where a criterion (with the given
        factors N_J, N_S, N_G, N_cone) asks for it; a central point source
        with the intrinsic line profile (eq. init_freq); six axis cameras;
        local core-skipping with the non-local density threshold f_nl (Sec.
        3.2.4); recoil on."""
        L = 4.0 * self.r_edge
        box_min = np.full(3, -0.5 * L)
        nj, ns, ng, nc = factors
        tree = inputs.build_octree(box_min, L, base_level, max_extra,
                                   lambda c, w, lev: self.refine(c, w, nj, ns, ng, nc),
                                   max_nodes=max_nodes)
        if tree is None:
            raise ValueError("refinement exceeds max_nodes; lower the factors or levels")
        child, cen, width, level = tree
        grid = {"kind": 1, "box_min": box_min, "box_max": box_min + L, "child": child,
                "n_HI": self.n_hi(cen), "T": np.full(len(child), self.T),
                "v": self.velocity(cen), "k_dust": None, "albedo": 0.0, "escape_radius": 0.0,
                "level": level, "f_nl": float(f_nl)}
        xlo, xhi = inputs.velocity_window(vmax_kms)
        cams = inputs.AXIS_CAMERAS.copy()
        params = {"n_photons": int(n_photons), "seed": int(seed), "xcrit_mode": 2,
                  "atau0": 0.0, "recoil": 1, "isotropic": 0, "n_bins": int(n_bins),
                  "x_min": xlo, "x_max": xhi, "cam_dir": cams, "cam_nbins": int(n_bins),
                  "cam_xmin": xlo, "cam_xmax": xhi, "cam_npix": int(npix), "cam_fov": float(L),
                  "tau_peel_max": 50.0}
        source = {"kind": 0, "pos": np.zeros((1, 3)), "freq_mode": 1}
        return {"name": f"galaxy_{self.name}", "grid": grid, "source": source,
                "params": params, "leaves": int((child < 0).sum()), "model": self,
                "centres": cen, "widths": width}
