"""Host-side logic of the serving layer that needs no GPU: the admission
estimate and the latency summary."""
import numpy as np

from paper_1409_4480_amd import inputs, serving


def up(n):
    """An allocation of the library: whole 256-byte blocks, at least one."""
    return max((n + 255) // 256 * 256, 256)


def test_footprint_grows_with_what_a_job_holds():
    n = 1000
    small = inputs.static_sphere(n=16, tau0=1e4, n_photons=n, seed=1)
    big = inputs.static_sphere(n=32, tau0=1e4, n_photons=n, seed=1)
    base = serving.footprint(small)
    # cells: every record of both precisions per cell
    assert serving.footprint(big) - base == serving.CELL_BYTES * (32 ** 3 - 16 ** 3)
    # per-photon records: final x, counts, status, position, peel sums (none)
    assert serving.footprint(small, record=True) - base == \
        up(8 * n) + 2 * up(4 * n) + up(24 * n) + up(0)
    # cameras: their table, spectra and images, and the next-event task buffer
    # of at least 2^20 slots (64 bytes each in FP32-bulk)
    cams = inputs.static_sphere(n=16, tau0=1e4, n_photons=n, seed=1,
                                cameras=np.eye(3), cam_nbins=50, cam_npix=8)
    extra = serving.footprint(cams) - serving.footprint(small)
    tallies = up(96 * 3) - up(96) + up(8 * 3 * 50) - up(8) + up(8 * 3 * 64) - up(8)
    assert extra == tallies + 64 * (1 << 20)
    # a job's suspended-photon store holds at most one record per photon
    one = inputs.static_sphere(n=16, tau0=1e4, n_photons=1, seed=1)
    assert base - serving.footprint(one) == 2 * (up(128 * n) - up(128))


def test_summary_percentiles_and_rate():
    lat = np.linspace(0.01, 1.0, 100)
    results = [{"latency_s": float(t), "counters": {"scat_hi": 10}} for t in lat]
    s = serving.summarize(results, makespan=2.0)
    assert s["jobs"] == 100 and s["scatterings"] == 1000
    assert abs(s["p50_ms"] - 1e3 * np.percentile(lat, 50)) < 1e-9
    assert abs(s["p99_ms"] - 1e3 * np.percentile(lat, 99)) < 1e-9
    assert s["p99_ms"] > s["p50_ms"] and s["scatterings_per_s"] == 500.0


def test_line_depth_ranks_jobs_by_their_optical_depth():
    """The split server's ranking proxy is proportional to the line-centre
    optical depth tau0 of a uniform sphere, whatever the grid resolution, and
    falls as 1/sqrt(T) at fixed column density."""
    r = [serving.line_depth(inputs.static_sphere(n=n, tau0=t, n_photons=10)) / t
         for n, t in ((16, 1e4), (32, 1e6), (48, 3e7), (16, 1e8))]
    assert np.allclose(r, r[0], rtol=1e-12)
    a = inputs.static_sphere(n=16, tau0=1e6, n_photons=10)
    b = {"grid": dict(a["grid"], T=4.0 * np.asarray(a["grid"]["T"]))}
    assert np.isclose(serving.line_depth(b), 0.5 * serving.line_depth(a), rtol=1e-12)
