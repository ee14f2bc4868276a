"""Host-side logic of the serving layer that needs no GPU: the admission
estimate and the latency summary."""
import numpy as np

from paper_1409_4480_amd import inputs, serving


def test_footprint_grows_with_what_a_job_holds():
    small = inputs.static_sphere(n=16, tau0=1e4, n_photons=1000, seed=1)
    big = inputs.static_sphere(n=32, tau0=1e4, n_photons=1000, seed=1)
    base = serving.footprint(small)
    # cells: every record of both precisions per cell
    assert serving.footprint(big) - base == serving.CELL_BYTES * (32 ** 3 - 16 ** 3)
    # per-photon records: final x, counts, position and one peel sum per camera
    assert serving.footprint(small, record=True) - base == 32 * 1000
    cams = inputs.static_sphere(n=16, tau0=1e4, n_photons=1000, seed=1,
                                cameras=np.eye(3), cam_nbins=50, cam_npix=8)
    extra = serving.footprint(cams) - serving.footprint(small)
    assert extra == 8 * 3 * (50 + 8 * 8)


def test_summary_percentiles_and_rate():
    lat = np.linspace(0.01, 1.0, 100)
    results = [{"latency_s": float(t), "counters": {"scat_hi": 10}} for t in lat]
    s = serving.summarize(results, makespan=2.0)
    assert s["jobs"] == 100 and s["scatterings"] == 1000
    assert abs(s["p50_ms"] - 1e3 * np.percentile(lat, 50)) < 1e-9
    assert abs(s["p99_ms"] - 1e3 * np.percentile(lat, 99)) < 1e-9
    assert s["p99_ms"] > s["p50_ms"] and s["scatterings_per_s"] == 500.0
