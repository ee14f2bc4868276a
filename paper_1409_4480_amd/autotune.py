"""Launch-shape autotuner for the transport kernel.

Sweeps workgroup size, resident workgroups per CU (the photon-pool depth) and
the march threshold (a wave keeps stepping its flights while at least this
many of its lanes are in flight; the rest resume after the wave's scatterings)
on a calibration slice of a workload, keeps the fastest by scatterings per
second, and caches the choice per (device, workload class) in a JSON file.
"""
import json
import os
import time

from . import colt

# (block, workgroups per CU[, march threshold]); a threshold of 0 is the library's
# default (16)
DEFAULT_SPACE = [(256, 1), (256, 2), (256, 3), (256, 4), (128, 2), (128, 4), (128, 6),
                 (64, 4), (64, 8), (256, 4, 8), (256, 4, 32)]


def device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def tune(workload, precision=colt.FP32_BULK, space=None, photons=200_000, cache_path=None,
         workload_class=None, repeats=1):
    """Returns {"block", "blocks_per_cu", "march_min", "scatterings_per_s",
    "table"} for the fastest launch shape on `photons` photons of the workload."""
    import torch
    space = list(space or DEFAULT_SPACE)
    cls = workload_class or workload.get("name", "workload")
    key = f"{device_key()}|{cls}|p{precision}"
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return dict(cache[key], cached=True)
    params = dict(workload["params"], n_photons=int(photons))
    grid = colt.Grid(workload["grid"])
    table = []
    try:
        for entry in space:
            block, per_cu = entry[0], entry[1]
            march_min = entry[2] if len(entry) > 2 else 0
            best = 0.0
            for r in range(repeats + 1):          # the first run warms up
                job = colt.Job(grid, workload["source"], dict(params, seed=params["seed"] + r),
                               precision=precision)
                torch.cuda.synchronize()
                t = time.perf_counter()
                colt.transport([job], block=block, blocks_per_cu=per_cu, march_min=march_min)
                out = job.tally(wait=True)
                dt = time.perf_counter() - t
                job.release()
                if r > 0 or repeats == 0:
                    best = max(best, out["counters"]["scat_hi"] / dt)
            table.append({"block": block, "blocks_per_cu": per_cu, "march_min": march_min,
                          "scatterings_per_s": best})
    finally:
        grid.release()
    top = max(table, key=lambda e: e["scatterings_per_s"])
    result = {"block": top["block"], "blocks_per_cu": top["blocks_per_cu"],
              "march_min": top["march_min"], "scatterings_per_s": top["scatterings_per_s"],
              "table": table}
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = result
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(result, cached=False)
