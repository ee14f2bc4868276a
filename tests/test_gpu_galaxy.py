"""Transfer through the idealised first-galaxy models of Sec. 5.1 on the GPU.

Parity: FP64 histories through a Late wind model (bipolar cavity, beta-law
wind, octree from the refinement criteria, six axis cameras) match the
oracle's photon by photon to a per-photon event cap.  Physics: the trends the
paper reports for these models (Sec. 6.2, table model_bolometric_flux) appear
in the observables computed from the tallies: static spectra are symmetric,
winds give several times more red than blue flux, and Late models are brighter
face-on (z) than edge-on.  These are trends, not the printed values: the grids
here are much coarser than the paper's refinement factors.
"""
import numpy as np
import pytest

import oracle
from paper_1409_4480_amd import colt
from paper_1409_4480_amd import galaxy as gx
from paper_1409_4480_amd import observables as ob
from tests.test_gpu_parity import compare_records, measured_flip, oracle_grid, say

pytestmark = pytest.mark.gpu

COARSE = dict(base_level=3, max_extra=4, factors=(8, 4, 8, 64))


def run_models(names, n_photons, precision=colt.FP32_BULK):
    """The models' jobs in one launch (their long histories overlap)."""
    wls = [gx.Model(name).workload(n_photons=n_photons, npix=64, **COARSE) for name in names]
    grids = [colt.Grid(wl["grid"]) for wl in wls]
    jobs = [colt.Job(g, wl["source"], wl["params"], precision=precision)
            for g, wl in zip(grids, wls)]
    say(f"[gpu] galaxy models {names}: {[wl['leaves'] for wl in wls]} leaves, "
        f"{n_photons} photons each, precision {precision}")
    try:
        colt.transport_all(jobs)
        return wls, [j.tally() for j in jobs]
    finally:
        for j in jobs:
            j.release()
        for g in grids:
            g.release()


def test_galaxy_fp64_histories_match_the_oracle():
    n, cap = 128, 2000
    wl = gx.Model("WL5").workload(n_photons=n, npix=32, **COARSE)
    wl["params"]["max_events"] = cap
    say(f"[gpu] galaxy WL5 parity: {wl['leaves']} leaves, {n} photons, cap {cap}")
    g = colt.run(wl, precision=colt.FP64, record=True, max_events=cap)
    r = oracle.run(oracle_grid(wl["grid"]), wl["source"], wl["params"], records=True)
    size = wl["grid"]["box_max"][0] - wl["grid"]["box_min"][0]
    compare_records(g, r, size, peel=True, flip=measured_flip(wl))
    assert g["counters"]["escaped"] + g["counters"]["capped"] == n


def test_galaxy_observables_follow_the_paper_trends():
    # ~1e6 scatterings per photon: a few hundred waves take as long as one, so
    # the run is sized for the statistics
    n = 16_000
    out = {}
    names = ("SE5", "SL5", "WL5")
    for name, wl, res in zip(names, *run_models(names, n)):
        c = res["counters"]
        assert c["emitted"] == n == c["escaped"]            # no dust: every photon escapes
        p = wl["params"]
        # cameras: +x, -x, +y, -y, +z, -z (edge-on: x, y; face-on: z)
        spec = res["cam_spec"].reshape(6, -1)
        ratio = [ob.flux_ratio_to_average(spec[i], n, c["escaped"]) for i in range(6)]
        img = res["cam_img"].reshape(6, p["cam_npix"], p["cam_npix"])
        out[name] = {
            "face": 0.5 * (ratio[4] + ratio[5]), "edge": 0.25 * sum(ratio[:4]),
            "red_blue": ob.red_blue_ratio(res["spectrum"][1:-1], p["x_min"], p["x_max"]),
            "red_blue_edge": ob.red_blue_ratio(spec[:4].sum(axis=0), p["cam_xmin"],
                                               p["cam_xmax"]),
            "r_half_edge": np.mean([ob.half_light_radius(img[i], p["cam_fov"])
                                    for i in range(4)]) / gx.PC,
            "r_half_face": np.mean([ob.half_light_radius(img[i], p["cam_fov"])
                                    for i in range(4, 6)]) / gx.PC}
        say(f"    {name}: {out[name]}")
    # a spherical model: every axis camera sees the angle-averaged flux
    assert out["SE5"]["face"] == pytest.approx(1.0, abs=0.1)
    assert out["SE5"]["edge"] == pytest.approx(1.0, abs=0.1)
    # static spectra are symmetric about line centre; the wind reddens them (the
    # paper's WL5 edge-on view has F_r / F_b = 6.36)
    tol = 8.0 / np.sqrt(n)                 # 4 sigma of a symmetric red/blue split
    assert out["SE5"]["red_blue"] == pytest.approx(1.0, abs=tol)
    assert out["SL5"]["red_blue"] == pytest.approx(1.0, abs=tol)
    assert out["WL5"]["red_blue"] > 3.0 and out["WL5"]["red_blue_edge"] > 3.0
    # Late models: brighter face-on than edge-on (table model_bolometric_flux)
    for name in ("SL5", "WL5"):
        assert out[name]["face"] > 1.3 and out[name]["edge"] < 0.95
