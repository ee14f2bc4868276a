"""The measurement script's host logic on the CPU: the CPU-baseline leg on a
small time budget, and profile figures reported only for the kernel sources
they were taken on."""
import bench


def test_cpu_baseline_reports_the_oracle_on_a_bounded_sample():
    r = bench.cpu_baseline(1_000_000, budget_s=0.5)
    assert r["kind"] == "oracle" and r["unit"] == "scatterings/s"
    assert r["value"] > 0 and r["photons_per_s"] > 0 and 1 <= r["cores"] <= 16
    assert "photons 0.." in r["sample"]


def test_profile_figures_only_for_the_sources_they_were_taken_on(monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: bench.PROFILE["sources_sha256"])
    assert bench.profile_figures() is bench.PROFILE
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.profile_figures() is None


def test_algorithmic_ops_follow_the_per_event_model():
    c = {"scat_hi": 1000, "upar_tries": 3000, "crossings": 500, "peel_crossings": 200}
    # 3 candidates per scattering: 335 + 83 * 3 lane-ops each, 34 per crossing
    assert bench.algorithmic_ops(c) == 1000 * (335 + 83 * 3) + 700 * 34
