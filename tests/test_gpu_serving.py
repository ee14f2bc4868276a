"""Serving: continuous batching of uneven jobs gives each job the result it
gets alone (FP64 and FP32-bulk photon records bit for bit), admission by memory budget
queues jobs without changing results, and latencies are reported."""
import numpy as np
import pytest

from paper_1409_4480_amd import colt, inputs, serving
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu


def small_stream(n=6, seed=3):
    jobs = inputs.job_stream(n_jobs=n, seed=seed, n_range=(16, 32), tau_range=(1e3, 1e5),
                             ph_range=(300, 3000))
    for k, wl in enumerate(jobs):
        wl["arrival"] = 0.02 * k
    return jobs


@pytest.mark.parametrize("prec,split", [(colt.FP64, False), (colt.FP32_BULK, False),
                                        (colt.FP64, True)])
def test_each_job_same_alone_and_in_the_mix(prec, split):
    """Every job's records are the same bit for bit when served in a mix of
    epochs (the multi-job kernel, slices of uneven jobs, with or without the
    long-history jobs kept apart) as when run alone (in FP32-bulk, the one-job
    kernel compiled for its grid kind)."""
    jobs = small_stream()
    say(f"[gpu] serving mix of {len(jobs)} jobs, precision {prec}, split {split}")
    srv = serving.Server(epoch_photons=2048, min_quota=256, precision=prec, record=True,
                         split=split)
    mixed = srv.run(jobs, realtime=False)
    assert srv.max_active == len(jobs) and srv.epochs > 1
    for wl, m in zip(jobs, mixed):
        alone = colt.run(wl, precision=prec, record=True)
        for k in ("x", "nscat", "status", "pos"):
            assert np.array_equal(alone["records"][k], m["records"][k]), (wl["name"], k)
        assert np.array_equal(alone["spectrum"], m["spectrum"])
        for k in ("emitted", "escaped", "scat_hi", "upar_tries", "crossings"):
            assert alone["counters"][k] == m["counters"][k]


@pytest.mark.parametrize("prec", [colt.FP64, colt.FP32_BULK])
def test_tail_rule_epochs_give_each_job_its_own_results(prec):
    """Epochs under the tail rule (every wave with fewer than 64 live photons
    suspends them once the epoch's queue is drained; the epochs are large
    enough for the rule to apply: every job has more than the 16384 photons a
    launch needs for it) resume the suspended photons in later epochs, and
    each job still gets the records it gets alone."""
    jobs = inputs.job_stream(n_jobs=3, seed=12, n_range=(16, 32), tau_range=(1e4, 1e5),
                             ph_range=(17000, 30000))
    say(f"[gpu] serving with the tail rule, {len(jobs)} jobs, precision {prec}")
    srv = serving.Server(epoch_photons=1 << 16, min_quota=8192, precision=prec, record=True,
                         tail_live=64)
    mixed = srv.run(jobs, realtime=False)
    say(f"    {srv.epochs} epochs")
    assert srv.epochs > len(jobs)
    for wl, m in zip(jobs, mixed):
        alone = colt.run(wl, precision=prec, record=True)
        for k in ("x", "nscat", "status", "pos"):
            assert np.array_equal(alone["records"][k], m["records"][k]), (wl["name"], k)
        assert np.array_equal(alone["spectrum"], m["spectrum"])
        for k in ("emitted", "escaped", "scat_hi", "upar_tries", "crossings"):
            assert alone["counters"][k] == m["counters"][k]


@pytest.mark.parametrize("prec", [colt.FP64, colt.FP32_BULK])
def test_bounded_epochs_stop_and_resume_bit_for_bit(prec):
    """With a time bound of zero every epoch is asked to stop as soon as the
    host sees it running: photons in flight are suspended and resumed in later
    epochs, and every job still gets the records it gets alone."""
    jobs = small_stream(n=5, seed=9)
    say(f"[gpu] serving with bounded epochs, {len(jobs)} jobs, precision {prec}")
    free = serving.Server(epoch_photons=2048, min_quota=256, precision=prec, record=True)
    free.run(jobs, realtime=False)
    srv = serving.Server(epoch_photons=2048, min_quota=256, precision=prec, record=True,
                         epoch_ms=0.0)
    mixed = srv.run(jobs, realtime=False)
    say(f"    epochs {srv.epochs} ({srv.stopped} asked to stop), unbounded {free.epochs}")
    assert srv.stopped > 0 and srv.epochs > free.epochs
    for wl, m in zip(jobs, mixed):
        alone = colt.run(wl, precision=prec, record=True)
        for k in ("x", "nscat", "status", "pos"):
            assert np.array_equal(alone["records"][k], m["records"][k]), (wl["name"], k)
        assert np.array_equal(alone["spectrum"], m["spectrum"])
        for k in ("emitted", "escaped", "scat_hi", "upar_tries", "crossings"):
            assert alone["counters"][k] == m["counters"][k]


def test_admission_footprint_bounds_the_device_bytes():
    """The server admits by an estimate made before anything is allocated; it
    must not undercount what the library then holds for the grid and the job
    (records on, with and without cameras, Cartesian and octree)."""
    cases = small_stream(n=4, seed=6)
    cases.append(inputs.halo(n=32, n_photons=500, seed=7))
    cases.append(inputs.nfw_octree(base_level=3, max_extra=2, leaves_target=(500, 4000),
                                   turb_n=32, n_photons=300, seed=8, npix=64))
    for wl in cases:
        g = colt.Grid(wl["grid"])
        j = colt.Job(g, wl["source"], wl["params"], precision=colt.FP32_BULK, record=True)
        try:
            held = g.nbytes + j.nbytes
            est = serving.footprint(wl, record=True)
            say(f"    {wl.get('name', '?')}: estimate {est} B, held {held} B")
            assert est >= held, (wl.get("name"), est, held)
        finally:
            j.release()
            g.release()


def test_memory_budget_queues_jobs_without_changing_results():
    jobs = small_stream(n=5, seed=4)
    biggest = max(serving.footprint(wl, record=True) for wl in jobs)
    srv = serving.Server(budget_bytes=int(1.2 * biggest), epoch_photons=4096, min_quota=512,
                         precision=colt.FP64, record=True)
    out = srv.run(jobs, realtime=False)
    assert srv.max_active < len(jobs) and srv.max_used <= srv.budget
    for wl, o in zip(jobs, out):
        assert o["counters"]["emitted"] == wl["params"]["n_photons"]
        alone = colt.run(wl, precision=colt.FP64, record=True)
        assert np.array_equal(alone["records"]["nscat"], o["records"]["nscat"])
    with pytest.raises(colt.ColtError):
        serving.Server(budget_bytes=biggest // 4).run(jobs[:1])


def test_realtime_arrivals_report_latency():
    jobs = small_stream(n=8, seed=5)
    srv = serving.Server(epoch_photons=8192, min_quota=512)
    out = srv.run(jobs, realtime=True)
    s = serving.summarize(out, srv.makespan)
    assert all(o["latency_s"] >= o["queue_s"] >= 0 for o in out)
    assert all(o["finished_s"] >= wl["arrival"] for o, wl in zip(out, jobs))
    assert s["p99_ms"] >= s["p50_ms"] > 0
    assert s["scatterings"] == sum(o["counters"]["scat_hi"] for o in out)


def test_autotuner_picks_and_caches_a_launch_shape(tmp_path):
    from paper_1409_4480_amd import autotune
    wl = inputs.dusty_sphere(n=16, tau0=1e5, n_photons=1)
    cache = str(tmp_path / "tune.json")
    space = [(256, 1), (128, 2), (64, 4), (256, 2, 4)]
    r = autotune.tune(wl, space=space, photons=20_000, cache_path=cache)
    shapes = {(e[0], e[1], e[2] if len(e) > 2 else 0) for e in space}
    assert not r["cached"] and (r["block"], r["blocks_per_cu"], r["march_min"]) in shapes
    assert len(r["table"]) == 4 and all(e["scatterings_per_s"] > 0 for e in r["table"])
    r2 = autotune.tune(wl, space=space, photons=20_000, cache_path=cache)
    assert r2["cached"] and r2["block"] == r["block"] and r2["march_min"] == r["march_min"]


def test_graph_replays_match_eager_transport():
    """A captured epoch replayed four times walks two jobs through their
    photons; after every replay (with unrelated eager work in between) the
    processed photons equal an eager run's, bit for bit."""
    import torch
    wl1 = inputs.static_sphere(n=8, tau0=5e3, n_photons=700, seed=1, isotropic=False)
    wl2 = inputs.dusty_sphere(n=8, tau0=1e5, n_photons=333, seed=2)
    ref1 = colt.run(wl1, record=True)["records"]
    ref2 = colt.run(wl2, record=True)["records"]
    other = inputs.static_sphere(n=8, tau0=1e3, n_photons=100, seed=3)
    g1, g2 = colt.Grid(wl1["grid"]), colt.Grid(wl2["grid"])
    j1 = colt.Job(g1, wl1["source"], wl1["params"], record=True)
    j2 = colt.Job(g2, wl2["source"], wl2["params"], record=True)
    graph = colt.Graph([j1, j2], photons_per_job=250)
    for rep in range(4):
        say(f"[gpu] graph replay {rep}")
        graph.launch()
        colt.run(other)                               # eager work between replays
        torch.cuda.synchronize()
        for j, ref, n in ((j1, ref1, 700), (j2, ref2, 333)):
            done = min(n, 250 * (rep + 1))
            assert j.status()[0] == done
            out = j.tally()
            assert out["counters"]["emitted"] == done
            for k in ("x", "nscat", "status", "pos"):
                assert np.array_equal(out["records"][k][:done], ref[k][:done]), (rep, k)
    graph.release()
    for h in (j1, j2, g1, g2):
        h.release()


def test_graph_of_one_fp32_job_matches_eager_transport():
    """A one-job FP32 graph (the job passed to the kernel by value at capture)
    replayed three times equals one eager launch of the whole job."""
    import torch
    wl = inputs.dusty_sphere(n=8, tau0=1e5, n_photons=900, seed=21)
    ref = colt.run(wl, precision=colt.FP32_BULK, record=True)
    g = colt.Grid(wl["grid"])
    j = colt.Job(g, wl["source"], wl["params"], precision=colt.FP32_BULK, record=True)
    graph = colt.Graph([j], photons_per_job=300)
    try:
        for rep in range(3):
            say(f"[gpu] one-job FP32 graph replay {rep}")
            graph.launch()
            torch.cuda.synchronize()
            assert j.status()[0] == 300 * (rep + 1)
        out = j.tally()
        for k in ("x", "nscat", "status", "pos"):
            assert np.array_equal(out["records"][k], ref["records"][k]), k
        assert np.array_equal(out["spectrum"], ref["spectrum"])
        assert out["counters"]["scat_hi"] == ref["counters"]["scat_hi"]
    finally:
        graph.release()
        j.release()
        g.release()
