"""Throughput benchmark of the Lyman-alpha transport hot path on one MI355X.

Workload (one step): the dusty uniform sphere -- 64^3 Cartesian grid, line-
centre radial optical depth tau0 = 1e7 at T = 1e4 K, grey dust tau_d = 1 with
albedo 0.32, global core-skipping from a*tau0 = 4702, anisotropic scattering,
500-bin escape spectrum, 1e6 photons from a central point source.  Each step
transports one full job (fresh seed) with the gas already resident in HBM and
reads its tallies back.  Consecutive steps are queued on eight streams in turn
(--streams), each launched on half of the device's workgroup slots
(--pipe-blocks-per-cu 2), so two or more steps run side by side and the
long-lived last photons of one step share the device with the bulk of the next (optionally, with --tail-live and --launches, waves left
with few live photons once a step's photons are all handed out pass them on
to the step's next launch, packed into full waves).  All steps complete
inside the timed region.  The
headline value is in FP32-bulk mode (FP32 Voigt/sampling/directions, FP64
position, optical depth and tallies); the same steps in all-FP64 mode are
reported beside it.  The roofline figures use the transport kernel's own
duration, measured on steps run one at a time in the same run.

Prints one JSON line.  Only one GPU is supported.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lyα scatterings/sec on 1 MI355X (mixed vs FP64 plain); p50/p99 job latency"
VALU_PEAK = 256 * 4 * 16 * 2.4e9      # lane-ops/s: 256 CUs x 4 SIMD16 x 2.4 GHz

# Algorithmic VALU lane-ops per unit of work, as the hot-path scope table
# derives them for this method (non-packed lane-op slots; transcendentals and
# 32-bit integer multiplies at quarter rate, i.e. four slots):
#   one H I scattering with n u_par candidates: (8 + 3 (n - 1)) uniforms of ~25
#   integer ops (Philox4x32-10), (10 + 2 n) transcendentals of 4 slots, ~150
#   FP32 and ~20 FP64 flops, i.e. 335 + 83 n (about 500 for core scatterings,
#   1100 for 3 <= |x| < 9);
#   one cell crossing, of the transport or of a next-event march: one H(a,x)
#   (~15 flops and an exp) and ~15 FP64 ops, i.e. 34.
def ops_per_scattering(n_iter):
    return 335.0 + 83.0 * n_iter


OPS_PER_CROSSING = 34.0


def algorithmic_ops(c):
    """Lane-ops of a launch from its event counters."""
    n_iter = c["upar_tries"] / max(c["scat_hi"], 1)
    return (c["scat_hi"] * ops_per_scattering(n_iter) +
            (c["crossings"] + c["peel_crossings"]) * OPS_PER_CROSSING)


# Figures of the FP32-bulk transport kernel on this workload from rocprofv3
# counters of the committed profile (profiles/k_transport_fp32_dusty_sphere_64.md),
# per launch:
# HBM bytes per launch from FETCH_SIZE and WRITE_SIZE scaled by a plain-copy
# calibration, and the VALU lane-instructions the hardware executed
# (SQ_INSTS_VALU x 64 x lane use) with the kernel time of that run.  They hold
# for the kernel sources they were taken on; for other sources they are null.
KERNEL_SOURCES = ("colt_kernels.hip", "colt_device.h", "colt_internal.h")
PROFILE = {"sources_sha256": "1bd05505aaf266e6e15e4c6019badf7ce981370ad12493eb0017ba83373715dd",
           "fetch_bytes": 51033707.0, "write_bytes": 45274587.0,
           "valu_lane_instructions": 311809032934.0, "kernel_ms": 21.286}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1409_4480_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_figures():
    if PROFILE["sources_sha256"] and PROFILE["sources_sha256"] == kernel_sources_sha256():
        return PROFILE
    return None


def workload(n_photons, seed):
    from paper_1409_4480_amd import inputs
    return inputs.dusty_sphere(n=64, tau0=1.0e7, n_photons=n_photons, seed=seed)


def cpu_baseline(n_photons_full, budget_s=15.0):
    """The CPU oracle on a bounded sample of the same workload: the first
    photons of a job, sized to about `budget_s` seconds after a calibration."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    wl = workload(n_photons_full, 1409448002)
    n_cal = 2000
    t = time.perf_counter()
    r = oracle.run(wl["grid"], wl["source"], wl["params"], id_begin=0, id_end=n_cal,
                   threads=threads)
    dt = time.perf_counter() - t
    n = int(min(n_photons_full, max(n_cal, n_cal * budget_s / max(dt, 1e-3))))
    t = time.perf_counter()
    r = oracle.run(wl["grid"], wl["source"], wl["params"], id_begin=0, id_end=n,
                   threads=threads)
    dt = time.perf_counter() - t
    scat = r["counters"]["scat_hi"]
    return {"value": scat / dt, "unit": "scatterings/s", "cores": threads, "kind": "oracle",
            "sample": f"photons 0..{n - 1} of the 1e6-photon job ({scat} scatterings, "
                      f"{dt:.1f} s, FP64 scalar C)",
            "photons_per_s": n / dt}


def serve_section(n_jobs, scaled=False):
    """The serving stream: n_jobs uniform or Hubble-expanding spheres (grid
    32^3-128^3, tau0 log-uniform in 1e4-1e8, 1e4-1e6 photons log-uniform,
    global core-skipping, recoil), FP32-bulk, the long-history jobs in epochs of
    their own.  Capacity with every job arrived at once; then Poisson arrivals
    at 0.8 of that capacity with p50/p99 latency (arrival to tallies on the
    host); against one job at a time in
    plain FP64, timed on a sample of jobs spread over the stream's range of
    scatterings per job (it would take over an hour for all 512).  scaled:
    the smaller stream of 32^3-64^3 grids, tau0 1e4-1e5, 1e4-5e4 photons."""
    import numpy as np
    import torch

    from paper_1409_4480_amd import colt, inputs, serving

    if scaled:
        stream = inputs.job_stream(n_jobs=n_jobs, seed=5, n_range=(32, 64),
                                   tau_range=(1.0e4, 1.0e5), ph_range=(1.0e4, 5.0e4))
        epoch, quota = 1 << 20, 8192
        cfg = {"grid": "32^3-64^3", "tau0": "1e4-1e5", "photons": "1e4-5e4"}
    else:
        stream = inputs.job_stream(n_jobs=n_jobs, seed=5)
        epoch, quota = 1 << 22, 65536
        cfg = {"grid": "32^3-128^3", "tau0": "1e4-1e8", "photons": "1e4-1e6"}
    srv = serving.Server(epoch_photons=epoch, min_quota=quota)
    out = srv.run(stream, realtime=False)
    batched = serving.summarize(out, srv.makespan)
    batched["epochs"] = srv.epochs
    print(f"# serving: capacity {batched['scatterings_per_s']:.3e} scatterings/s over "
          f"{srv.makespan:.1f} s", file=sys.stderr, flush=True)
    rate = 0.8 * n_jobs / srv.makespan
    rng = np.random.default_rng(5)
    t = 0.0
    for wl in stream:
        t += rng.exponential(1.0 / rate)
        wl["arrival"] = t
    srv = serving.Server(epoch_photons=epoch, min_quota=quota)
    out2 = srv.run(stream, realtime=True)
    poisson = serving.summarize(out2, srv.makespan)
    print(f"# serving: Poisson p50/p99 {poisson['p50_ms']:.0f}/{poisson['p99_ms']:.0f} ms",
          file=sys.stderr, flush=True)
    # one job at a time, FP64: a sample across the stream's job sizes (the
    # FP32 run's scatterings per job, from small to large)
    scat_job = np.array([o["counters"]["scat_hi"] for o in out], float)
    order = np.argsort(scat_job)
    picks = order[np.linspace(0, len(order) - 1, 12).round().astype(int)]
    picks = [int(i) for i in picks if scat_job[i] <= 2e9][:10]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scat = 0
    for i in picks:
        r = colt.run(stream[i], precision=colt.FP64)
        scat += r["counters"]["scat_hi"]
    serial = time.perf_counter() - t0
    serial_rate = scat / serial
    return {"config": dict(cfg, jobs=n_jobs, precision="FP32-bulk", epoch_photons=epoch,
                           scaled=scaled, split=srv.split, tail_live=srv.tail_live),
            "batched": batched,
            "poisson": dict(poisson, rate_jobs_per_s=rate, offered_load=0.8,
                            offered_scatterings_per_s=rate * poisson["scatterings"] / n_jobs,
                            epochs=srv.epochs,
                            note="offered: the arrival rate times the mean scatterings per "
                                 "job; a run that sustains less than it was offered fell "
                                 "behind its arrivals and its latencies include the backlog"),
            "serial_fp64": {"scatterings_per_s": serial_rate, "sample_jobs": len(picks),
                            "sample_scatterings": scat, "sample_s": serial,
                            "sample": "jobs spread over the stream's scatterings per job "
                                      "(up to 2e9), each alone, FP64"},
            "speedup_batched_vs_serial_fp64": batched["scatterings_per_s"] / serial_rate}


def precision_errors(grid, wl):
    """FP32-bulk against FP64 on the same job (same seed), per result: escape
    fraction, mean and mean |x| of the escaped photons, mean scatterings per
    photon -- each as the difference and its Monte-Carlo standard error --
    and the escape spectra's two-sample chi^2 and x KS p-values.  The two
    modes draw different histories from the same streams, so agreement is
    statistical."""
    import numpy as np
    from scipy import stats as sst

    from paper_1409_4480_amd import colt

    out = {}
    for prec in (colt.FP32_BULK, colt.FP64):
        job = colt.Job(grid, wl["source"], wl["params"], precision=prec, record=True)
        colt.transport([job])
        out[prec] = job.tally(wait=True)
        job.release()
    a, b = out[colt.FP32_BULK], out[colt.FP64]
    n = wl["params"]["n_photons"]
    res = {}
    fa, fb = a["counters"]["escaped"] / n, b["counters"]["escaped"] / n
    res["escape_fraction"] = {"fp32": fa, "fp64": fb, "diff": fa - fb,
                              "sigma": math.sqrt((fa * (1 - fa) + fb * (1 - fb)) / n)}
    xa = a["records"]["x"][a["records"]["status"] == 1]
    xb = b["records"]["x"][b["records"]["status"] == 1]
    for name, fa_, fb_ in (("mean_x", xa, xb), ("mean_abs_x", np.abs(xa), np.abs(xb))):
        res[name] = {"fp32": float(fa_.mean()), "fp64": float(fb_.mean()),
                     "diff": float(fa_.mean() - fb_.mean()),
                     "sigma": float(math.sqrt(fa_.var() / len(fa_) + fb_.var() / len(fb_)))}
    na, nb = a["records"]["nscat"], b["records"]["nscat"]
    res["mean_scatterings"] = {"fp32": float(na.mean()), "fp64": float(nb.mean()),
                               "diff": float(na.mean() - nb.mean()),
                               "sigma": float(math.sqrt((na.var() + nb.var()) / n))}
    ha, hb = a["spectrum"], b["spectrum"]
    keep = (ha + hb) >= 10
    table = np.vstack([ha[keep], hb[keep]])
    res["spectrum_chi2_p"] = float(sst.chi2_contingency(table)[1])
    res["escaped_x_ks_p"] = float(sst.ks_2samp(xa, xb).pvalue)
    return res


PROGRESS_TOKEN = 9


def timed_job(grid, wl, precision, cap=0, progress=None):
    """Runs one job to completion (as many launches as its next-event task
    buffer needs) and returns its counters, the wall time between device
    synchronisations and the launch count.  With `progress` (a name), a host
    thread also sets a stop word every 20 s, so no launch runs longer than
    that (the stopped photons resume exactly in the next launch), and a
    progress line is printed between launches."""
    import threading

    import torch

    from paper_1409_4480_amd import colt
    job = colt.Job(grid, wl["source"], wl["params"], precision=precision, max_events=cap)
    torch.cuda.synchronize()
    t = time.perf_counter()
    if progress is None:
        n = colt.transport_all([job])
    else:
        done = threading.Event()

        def tick():
            while not done.wait(20.0):
                colt.stop_set(PROGRESS_TOKEN, True)
        th = threading.Thread(target=tick, daemon=True)
        th.start()
        n, last = 0, t
        try:
            while not job.complete:
                colt.stop_set(PROGRESS_TOKEN, False)
                colt.transport([job], stop_token=PROGRESS_TOKEN)
                n += 1
                torch.cuda.synchronize()
                now = time.perf_counter()
                if now - last > 15.0:
                    nxt, n_susp, _ = job.pending()
                    print(f"#   {progress}: {now - t:.0f} s, {n} launches, {nxt} photons "
                          f"started, {n_susp} in flight", file=sys.stderr, flush=True)
                    last = now
        finally:
            done.set()
            th.join()
            colt.stop_set(PROGRESS_TOKEN, False)
    c = job.tally(wait=True)["counters"]
    dt = time.perf_counter() - t
    job.release()
    return c, dt, n


def workload_figures(c, dt, n, extra):
    ops = algorithmic_ops(c)
    return dict({"scatterings_per_s": c["scat_hi"] / dt, "ms": dt * 1e3, "launches": n,
                 "photons": c["emitted"], "photons_per_s": c["emitted"] / dt,
                 "scatterings_per_photon": c["scat_hi"] / max(c["emitted"], 1),
                 "peels_per_scattering": c["peels"] / max(c["scat_hi"], 1),
                 "peel_crossings_per_s": c["peel_crossings"] / dt,
                 "upar_tries_per_scattering": c["upar_tries"] / max(c["scat_hi"], 1),
                 "valu_frac_algorithmic": ops / dt / VALU_PEAK,
                 "precision": "FP32-bulk"}, **extra)


def workloads_section(n_photons=262144, cap=2000, only=None):
    """Throughput of the other workloads, FP32-bulk, all kernels of every
    launch timed between device synchronisations: the 128^3 first-galaxy halo
    (8 cameras, 256^2 images, 1000 bins), the ~2e6-leaf NFW octree (4 cameras,
    512^2 images, non-local core-skipping estimate at set-up) and an idealised
    first-galaxy model (WL7 on an octree, six axis cameras), a full pool of
    photons each followed for its first `cap` events (the steady state of jobs
    whose full histories run to ~1e6 scatterings per photon), and the static
    slab at tau0 = 1e7 run to completion."""
    import numpy as np
    import torch

    from paper_1409_4480_amd import colt, galaxy, inputs

    cases = [("halo_128cube_8cams", lambda: inputs.halo(n_photons=n_photons), cap),
             ("nfw_octree_2e6_leaves_4cams", lambda: inputs.nfw_octree(n_photons=n_photons), cap),
             ("galaxy_WL7_octree_6cams",
              lambda: galaxy.Model("WL7").workload(n_photons=n_photons, npix=128, base_level=4,
                                                   max_extra=5, factors=(16, 8, 16, 128)), cap),
             ("slab_tau1e7", lambda: inputs.slab(tau0=1.0e7, n_photons=n_photons), 0)]
    if only:
        cases = [c for c in cases if c[0] == only]
        if not cases:
            raise SystemExit(f"no workload named {only!r}")
    out = {}
    for name, make, ev_cap in cases:
        wl = make()
        if ev_cap:
            wl["params"]["max_events"] = ev_cap
        torch.cuda.synchronize()
        t = time.perf_counter()
        grid = colt.Grid(wl["grid"])
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t) * 1e3
        for rep in range(2):                      # the first run warms up
            c, dt, n = timed_job(grid, wl, colt.FP32_BULK, ev_cap)
        grid.release()
        n_cells = int(np.asarray(wl["grid"]["n_HI"]).size)
        out[name] = workload_figures(c, dt, n, {"events_cap": ev_cap or None,
                                                "grid_nodes": n_cells, "grid_setup_ms": setup_ms})
        print(f"# {name}: {out[name]['scatterings_per_s']:.3e} scatterings/s", file=sys.stderr,
              flush=True)
    return out


def full_histories_section(n_photons, only=None):
    """The halo (128^3, its configuration: local and non-local core-skipping,
    8 cameras) and the NFW octree (~2e6 leaves, 4 cameras) followed to the end
    of every history, on a subsample: the job's first n_photons photon ids (the
    same photons as in the 1e7-photon jobs; 1e6 by default).  Their histories
    are heavy-tailed (~7.6e5 scatterings per halo photon on average, 4.2e4 per
    octree photon, a few far more), so the last photons run nearly alone for
    tens of seconds and the run's time includes that tail."""
    from paper_1409_4480_amd import colt, inputs

    out = {}
    cases = (("halo_128cube_8cams_full", lambda: inputs.halo(n_photons=n_photons)),
             ("nfw_octree_2e6_leaves_4cams_full", lambda: inputs.nfw_octree(n_photons=n_photons)))
    if only:
        cases = [c for c in cases if c[0] == only]
        if not cases:
            raise SystemExit(f"no full-history workload named {only!r}")
    for name, make in cases:
        wl = make()
        grid = colt.Grid(wl["grid"])
        c, dt, n = timed_job(grid, wl, colt.FP32_BULK, progress=name)
        grid.release()
        sample = ("the whole 1e7-photon job" if n_photons == 10_000_000 else
                  f"photon ids 0..{n_photons - 1} of the 1e7-photon job")
        out[name] = workload_figures(c, dt, n, {"sample": sample + ", full histories"})
        print(f"# {name}: {dt:.1f} s, {out[name]['scatterings_per_photon']:.3g} scatterings "
              f"per photon", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=int, default=1_000_000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--streams", type=int, default=8,
                    help="streams the steps are queued on in turn (1: one step at a time)")
    ap.add_argument("--pipe-blocks-per-cu", type=int, default=2,
                    help="resident workgroups per CU of each pipelined step's launch (2: a "
                         "step takes half of the device, so two or more run side by side; "
                         "0: the kernel's limit)")
    ap.add_argument("--tail-live", type=int, default=0,
                    help="pipelined steps: once a step's photons are all handed out, waves "
                         "with fewer live photons hand them to the next of its launches "
                         "(0: off, the default: measured slower on this workload)")
    ap.add_argument("--launches", type=int, default=1,
                    help="launch sequences queued per pipelined step")
    ap.add_argument("--batch", type=int, default=4,
                    help="jobs of the workload fused in one launch for the batched figure "
                         "(0 or 1 skips it)")
    ap.add_argument("--no-cams", action="store_true",
                    help="skip the other workloads (cameras, octrees, galaxy model, slab)")
    ap.add_argument("--serve-jobs", type=int, default=512,
                    help="jobs in the serving stream (0 skips the serving section)")
    ap.add_argument("--serve-scaled", action="store_true",
                    help="serve the smaller stream (32^3-64^3, tau0 <= 1e5, <= 5e4 photons)")
    ap.add_argument("--full-photons", type=int, default=1_000_000,
                    help="photons of the halo and octree followed to the end of their "
                         "histories (0 skips)")
    ap.add_argument("--only-workload", default=None,
                    help="only run this entry of the workloads section (e.g. halo_128cube_8cams) "
                         "and print its figures")
    ap.add_argument("--only-full", default=None,
                    help="only follow this full-history workload (e.g. "
                         "nfw_octree_2e6_leaves_4cams_full) for --full-photons photons")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the transport "
              "shards by photon ranges across GPUs, which is not implemented here.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1409_4480_amd import colt

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = 256 * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return
    if args.only_workload:
        print(json.dumps(workloads_section(only=args.only_workload)))
        return
    if args.only_full:
        print(json.dumps(full_histories_section(args.full_photons, only=args.only_full)))
        return
    stream = torch.cuda.current_stream()
    wl = workload(args.photons, 1409448002)
    t0 = time.perf_counter()
    grid = colt.Grid(wl["grid"])
    torch.cuda.synchronize()
    grid_setup_ms = (time.perf_counter() - t0) * 1e3

    def run_steps(precision, n_steps, seed0, streams=args.streams):
        """n_steps jobs of the workload (seeds seed0, seed0 + 1, ...), each one
        step; with several streams consecutive steps are queued on them in
        turn, so a step's bulk overlaps the previous step's tail.  Every step's
        launches are bracketed by HIP events on its own stream (its kernel
        time); tallies are read back once each step is complete."""
        import ctypes
        jobs = [colt.Job(grid, wl["source"], dict(wl["params"], seed=seed0 + i),
                         precision=precision) for i in range(n_steps)]
        sts = [torch.cuda.Stream() for _ in range(max(1, streams))]
        for st in sts:          # every stream has its hardware queue before the clock starts
            with torch.cuda.stream(st):
                torch.ones(1, device="cuda").add_(1.0)
        torch.cuda.synchronize()
        marks = []
        t_start = time.perf_counter()
        for i, j in enumerate(jobs):
            st = sts[i % len(sts)]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            colt.transport([j], block=args.block, blocks_per_cu=args.pipe_blocks_per_cu,
                           stream=ctypes.c_void_p(st.cuda_stream), tail_live=args.tail_live,
                           launches=args.launches)
            e1.record(st)
            marks.append((e0, e1))
        counters = []
        for i, j in enumerate(jobs):
            j.tally(wait=True)
            if not j.complete:      # the tail needed more launches than were queued
                colt.transport_all([j], tail_live=args.tail_live,
                                   stream=ctypes.c_void_p(sts[i % len(sts)].cuda_stream))
            counters.append(j.tally(wait=True)["counters"])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kern = [e0.elapsed_time(e1) for e0, e1 in marks]
        for j in jobs:
            j.release()
        return elapsed, kern, counters

    def steps_alone(precision, n_steps, seed0):
        """Steps run one at a time: the latency of a step (launch to tallies on
        the host) and the transport kernel's own duration (HIP events around
        it on its stream), with its counters."""
        lat, kern, cnt = [], [], []
        for i in range(n_steps):
            j = colt.Job(grid, wl["source"], dict(wl["params"], seed=seed0 + i),
                         precision=precision)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            colt.transport([j], block=args.block, blocks_per_cu=args.blocks_per_cu,
                           time_kernel=True)
            cnt.append(j.tally(wait=True)["counters"])
            lat.append((time.perf_counter() - ts) * 1e3)
            kern.append(colt.last_kernel_ms())
            j.release()
        return lat, kern, cnt

    # warm-up, then the timed steps (FP32-bulk headline)
    if args.warmup:
        run_steps(colt.FP32_BULK, args.warmup, 7000)
    el, span, cnt = run_steps(colt.FP32_BULK, args.steps, 1409448002)
    lat, kern, cnt1 = steps_alone(colt.FP32_BULK, 5, 8000)
    scat = sum(c["scat_hi"] for c in cnt)
    photons = sum(c["emitted"] for c in cnt)
    value = scat / el
    kern_avg_ms = float(np.mean(kern))
    ops = np.mean([algorithmic_ops(c) for c in cnt1])
    achieved = ops / (kern_avg_ms * 1e-3)
    prof = profile_figures()
    measured = None
    if prof:
        lanes = prof["valu_lane_instructions"]
        measured = {"valu_lane_instructions": lanes, "kernel_ms": prof["kernel_ms"],
                    "achieved": lanes / (prof["kernel_ms"] * 1e-3) / 1e12,
                    "frac": lanes / (prof["kernel_ms"] * 1e-3) / VALU_PEAK,
                    "source": "rocprofv3 counters, profiles/k_transport_fp32_dusty_sphere_64.md"}
    result = {
        "metric": METRIC, "value": value, "unit": "scatterings/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "dusty_sphere_64cube_tau1e7", "grid": "64^3 Cartesian",
                   "tau0": 1.0e7, "T_K": 1.0e4, "tau_dust": 1.0, "albedo": 0.32,
                   "core_skip": "global x_crit(a tau0=4702)=3.35", "photons_per_step": args.photons,
                   "spectrum_bins": 500, "precision": "FP32-bulk"},
        "photons_per_s": photons / el,
        "streams": args.streams, "pipelined_blocks_per_cu": args.pipe_blocks_per_cu,
        "tail_live": args.tail_live, "launches_per_step": args.launches,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "of": "one step alone, launch to tallies on the host"},
        "per_step": {"scatterings": scat / args.steps,
                     "escaped_fraction": sum(c["escaped"] for c in cnt) / photons,
                     "upar_tries_per_scattering": sum(c["upar_tries"] for c in cnt) / max(scat, 1),
                     "crossings": sum(c["crossings"] for c in cnt) / args.steps,
                     "loop_passes": sum(c["passes"] for c in cnt) / args.steps,
                     "upar_rounds_per_pass": sum(c["upar_rounds"] for c in cnt) /
                     max(sum(c["passes"] for c in cnt), 1),
                     # FP32 lanes evaluate two candidates per round
                     "upar_candidate_lane_use": sum(c["upar_tries"] for c in cnt) /
                     max(128 * sum(c["upar_rounds"] for c in cnt), 1)},
        "grid_setup_ms": grid_setup_ms,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK,
                     "traffic": (prof["fetch_bytes"] + prof["write_bytes"]) if prof else None,
                     "kernel": "k_transport<float>", "kernel_ms": kern_avg_ms,
                     "kernel_ms_note": "the transport kernel's own duration: HIP events around "
                                       "it on its stream, for 5 steps run one at a time in this "
                                       "run (pipelined steps overlap, so their spans include "
                                       "time shared with the next step)",
                     "pipelined_span_ms": float(np.mean(span)),
                     "timed_region": {
                         "ops": float(sum(algorithmic_ops(c) for c in cnt)),
                         "elapsed_ms": el * 1e3,
                         "achieved": sum(algorithmic_ops(c) for c in cnt) / el / 1e12,
                         "frac": sum(algorithmic_ops(c) for c in cnt) / el / VALU_PEAK,
                         "note": "all the timed steps' algorithmic lane-ops over the timed "
                                 "region's wall time (the steps overlap on the device)"},
                     "ops_per_launch": ops,
                     "ops_model": "335 + 83 n lane-ops per H I scattering (n u_par candidates), "
                                  "34 per cell crossing",
                     "measured": measured},
    }
    # the same steps fused: args.steps jobs of the workload in one persistent
    # launch (per-job queues), so that one job's long-lived last photons share
    # the device with the others' bulk
    if args.batch > 1:
        jobs = [colt.Job(grid, wl["source"], dict(wl["params"], seed=1409448002 + i),
                         precision=colt.FP32_BULK) for i in range(args.batch)]
        torch.cuda.synchronize()
        tb = time.perf_counter()
        colt.transport(jobs, block=args.block, blocks_per_cu=args.blocks_per_cu,
                       time_kernel=True)
        outs = [j.tally(wait=True) for j in jobs]
        elb = time.perf_counter() - tb
        scat_b = sum(o["counters"]["scat_hi"] for o in outs)
        for j in jobs:
            j.release()
        result["batched_steps"] = {"jobs": args.batch, "value": scat_b / elb,
                                   "unit": "scatterings/s", "ms": elb * 1e3,
                                   "kernel_ms": colt.last_kernel_ms(),
                                   "note": "the jobs of as many steps in one launch"}
    if not args.no_fp64:
        el64, span64, cnt64 = run_steps(colt.FP64, args.steps, 1409448002)
        lat64, kern64, _ = steps_alone(colt.FP64, 3, 8000)
        scat64 = sum(c["scat_hi"] for c in cnt64)
        result["fp64_plain"] = {
            "value": scat64 / el64, "unit": "scatterings/s",
            "ms_per_step": el64 / args.steps * 1e3, "kernel_ms": float(np.mean(kern64)),
            "latency_ms": {"p50": float(np.percentile(lat64, 50)),
                           "p99": float(np.percentile(lat64, 99))},
            "escaped_fraction": sum(c["escaped"] for c in cnt64) /
            sum(c["emitted"] for c in cnt64)}
        result["speedup_mixed_vs_fp64"] = value / (scat64 / el64)
        result["fp32_vs_fp64"] = precision_errors(grid, wl)
    grid.release()
    if not args.no_cams:
        result["workloads"] = workloads_section()
    if args.full_photons > 0:
        result["full_histories"] = full_histories_section(args.full_photons)
    if args.serve_jobs > 0:
        result["serving"] = serve_section(args.serve_jobs, scaled=args.serve_scaled)
        result["latency_ms"] = {"p50": result["serving"]["poisson"]["p50_ms"],
                                "p99": result["serving"]["poisson"]["p99_ms"],
                                "of": "serving stream jobs (arrival to tallies on host)"}
        result["per_step"]["step_latency_ms"] = {"p50": float(np.percentile(lat, 50)),
                                                 "p99": float(np.percentile(lat, 99))}
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args.photons)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
