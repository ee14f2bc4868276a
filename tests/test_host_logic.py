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
    optical depth tau0 of a uniform sphere, whatever the grid resolution, with
    the same constant for a slab (whose tau0 is across its thin direction),
    and falls as 1/sqrt(T) at fixed column density."""
    r = [serving.line_depth(inputs.static_sphere(n=n, tau0=t, n_photons=10)) / t
         for n, t in ((16, 1e4), (32, 1e6), (48, 3e7), (16, 1e8))]
    r += [serving.line_depth(inputs.slab(tau0=t, n_photons=10)) / t for t in (1e5, 1e7)]
    assert np.allclose(r, r[0], rtol=1e-12)
    a = inputs.static_sphere(n=16, tau0=1e6, n_photons=10)
    b = {"grid": dict(a["grid"], T=4.0 * np.asarray(a["grid"]["T"]))}
    assert np.isclose(serving.line_depth(b), 0.5 * serving.line_depth(a), rtol=1e-12)


class _Stub:
    def __init__(self, tier):
        self.tier = tier


def test_split_epochs_keep_long_history_jobs_apart():
    """Slot 0 runs the short-history tier only while any short job is
    active; the long-history slot runs its own tier, else short jobs; a taken
    slot is skipped; without the split an epoch takes every ready job."""
    srv = serving.Server(budget_bytes=1 << 30, depth=2)
    s0, s1, l0, l1 = _Stub(0), _Stub(0), _Stub(1), _Stub(1)
    act = [s0, s1, l0, l1]
    assert srv._next_epoch([s0, l0, l1], act, set()) == (0, [s0])
    assert srv._next_epoch([s0, l0, l1], act, {0}) == (1, [l0, l1])
    assert srv._next_epoch([s0, s1], act, {0}) == (1, [s0, s1])
    # short jobs active but none ready: slot 0 waits, the long jobs take slot 1
    assert srv._next_epoch([l0], act, set()) == (1, [l0])
    assert srv._next_epoch([l0], act, {1}) == (None, [])
    # no short job active at all: slot 0 takes the long-history jobs too
    assert srv._next_epoch([l0, l1], [l0, l1], {1}) == (0, [l0, l1])
    fair = serving.Server(budget_bytes=1 << 30, depth=2, split=False)
    assert fair._next_epoch([s0, l0], act, {0}) == (1, [s0, l0])


def test_tiers_follow_the_rank_among_admitted_jobs():
    srv = serving.Server(budget_bytes=1 << 30, depth=2)
    depths = []
    tiers = []
    for d in (5.0, 1.0, 9.0, 3.0, 7.0, 2.0):
        depths.append(d)
        tiers.append(srv._tier_of(d, depths))
    # the first job is alone (tier 0); later ones are heavy from the median up
    assert tiers == [0, 0, 1, 0, 1, 0]
    three = serving.Server(budget_bytes=1 << 30, depth=3)
    ds = [float(i) for i in range(9)]
    assert [three._tier_of(d, ds) for d in ds] == [0, 0, 0, 1, 1, 1, 2, 2, 2]
