"""Continuous-batching server for transfer jobs on one GPU.

Jobs (workload dictionaries from ``inputs``, each with an arrival time in
seconds) are admitted in arrival order while their device footprint fits the
memory budget; every admitted job keeps its grid and tallies resident.  The
server then runs epochs: one persistent transport launch over the next slice
of photons of active jobs (``colt_transport`` with ``photons_per_job``), so
jobs that arrive while others are running join at the next epoch and share
the device with them.  Up to ``depth`` epochs are in flight on separate
streams, so an epoch's last long-lived photons share the device with the next
epoch instead of holding it alone (a job's slices cover disjoint photon ids and
its tallies are atomic, so overlapping epochs are safe).  An epoch ends with
its longest photon histories, so jobs whose histories are long (high optical
depth) run in epochs of their own, apart from the others.  A job's latency
runs from its arrival to its tallies being on the host.

Scheduling only: all transport work happens in the HIP library.
"""
import ctypes
import time
from collections import deque

import numpy as np

from . import colt

# per cell: line records (FP64 64 B, FP32 32 B), scattering-only records
# (g, non-local and Jeans a tau: FP64 32 B, FP32 16 B) and n_HI
CELL_BYTES = 64 + 32 + 32 + 16 + 8


def footprint(wl, record=False, precision=colt.FP32_BULK):
    """Device bytes a job will hold: its grid's records (estimated here) and
    the job's own memory (as the library computes it: tallies, records,
    suspend arrays, next-event task buffer)."""
    g = wl["grid"]
    n_cells = int(np.asarray(g["n_HI"]).size)
    n = CELL_BYTES * n_cells
    if g.get("child") is not None:                     # child table, base table, six
        n += (4 + 24 + 32) * n_cells + 4 * 128 ** 3     # links per leaf (again beside the
                                                        # FP32 record, filling its line)
    n += colt.job_footprint(wl["source"], wl["params"], precision, record)
    return n + (64 << 10)


_EPOCH_TOKEN0 = 40                     # stop tokens of bounded epochs: 40 .. 40 + depth - 1


class _Active:
    __slots__ = ("wl", "grid", "job", "arrival", "admitted", "bytes", "index", "tier")


def line_depth(wl):
    """A proxy, for ranking jobs only, of how long a job's photon histories
    run: the largest n_HI / sqrt(T) of its cells (the line-centre opacity
    scales so) times the distance from the domain's centre to its nearest
    face (half its narrowest extent)."""
    g = wl["grid"]
    n = np.asarray(g["n_HI"], float)
    t = np.asarray(g["T"], float)
    width = float(np.min(np.asarray(g["box_max"], float) - np.asarray(g["box_min"], float)))
    return float(np.max(n / np.sqrt(t))) * 0.5 * width


class Server:
    """Admits jobs by HBM footprint and runs them in shared epochs.

    budget_bytes    device memory the server may hold (None: 90 % of free HBM)
    epoch_photons   photons per epoch, split evenly over the epoch's jobs
    min_quota       smallest per-job slice of an epoch
    depth           epochs in flight at once, each on a stream of its own
    epoch_ms        None, or a time after which a running epoch is asked to stop:
                    its photons in flight are suspended and resume, bit for bit,
                    in a later epoch, so the jobs whose photons are done leave
                    without waiting for the longest histories of the others
                    (a job is then in one epoch at a time)
    split           (default) keep jobs with long photon histories out of the
                    epochs of jobs with short ones (False: every epoch takes
                    every active job): each job falls in one of `depth`
                    tiers by the rank of its line_depth among the jobs admitted
                    so far, and stream slot k runs epochs of tier k (or, when
                    it has nothing ready, of the nearest lighter tier; when no
                    job of tier k or lighter is active, of the nearest heavier
                    one), so a short job's epoch does not last as long as the
                    longest histories of the mix
    tail_live       the transport's tail rule for every epoch (0: off): once
                    an epoch's photons are all handed out, a wave holding fewer
                    than this many live photons suspends them, and they resume
                    in the job's next epoch beside fresh work, so an epoch does
                    not wait for its longest histories (a job is then in one
                    epoch at a time)
    """

    def __init__(self, budget_bytes=None, epoch_photons=1 << 20, min_quota=8192,
                 precision=colt.FP32_BULK, record=False, block=0, blocks_per_cu=0, depth=2,
                 epoch_ms=None, split=True, tail_live=16):
        import torch
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.9 * free)
        self.budget = int(budget_bytes)
        self.epoch_photons = int(epoch_photons)
        self.min_quota = int(min_quota)
        self.precision = precision
        self.record = record
        self.block = block
        self.blocks_per_cu = blocks_per_cu
        self.depth = max(1, int(depth))
        if epoch_ms is not None and self.depth > 64 - _EPOCH_TOKEN0:
            raise ValueError("bounded epochs take one stop token each: "
                             f"depth <= {64 - _EPOCH_TOKEN0}")
        self.epoch_ms = epoch_ms
        self.split = bool(split) and self.depth > 1
        if not 0 <= int(tail_live) <= 64:
            raise ValueError("tail_live is a number of lanes, 0..64")
        self.tail_live = int(tail_live)
        self._torch = torch

    def _tier_of(self, d, depths):
        """The tier of a job whose line_depth is d among the line_depths of
        the jobs admitted so far (d included)."""
        below = sum(1 for x in depths if x < d)
        return min(self.depth - 1, below * self.depth // len(depths))

    def _next_epoch(self, ready, active, taken):
        """The stream slot and the jobs of the next epoch, or (None, []): the
        first free slot that has jobs to run.  Without the split that is every
        ready job; with it, slot k takes tier k, else the nearest lighter tier
        with ready jobs, else (only when no job of tier k or lighter is active
        at all) the nearest heavier one."""
        for k in range(self.depth):
            if k in taken:
                continue
            if not self.split:
                return k, ready
            for tier in range(k, -1, -1):
                cand = [a for a in ready if a.tier == tier]
                if cand:
                    return k, cand
            if not any(a.tier <= k for a in active):
                for tier in range(k + 1, self.depth):
                    cand = [a for a in ready if a.tier == tier]
                    if cand:
                        return k, cand
        return None, []

    def run(self, workloads, realtime=True, on_done=None):
        """Serves the jobs; returns one result dict per job, in input order.

        With realtime=False every job is taken as arrived at time 0.  on_done,
        if given, is called as on_done(index, result) as each job finishes.  If
        a launch or on_done raises, the epochs in flight are waited for and
        every job and grid the server holds is released before the error
        propagates.
        """
        order = sorted(range(len(workloads)),
                       key=lambda i: workloads[i].get("arrival", 0.0) if realtime else 0.0)
        pending = deque(order)
        for i in order:
            if footprint(workloads[i], self.record, self.precision) > self.budget:
                raise colt.ColtError(f"job {i} needs more than the memory budget")
        torch = self._torch
        streams = [torch.cuda.Stream() for _ in range(self.depth)]
        results = [None] * len(workloads)
        active = []
        inflight = deque()             # [event, ids of the jobs, stream slot, start, stop asked]
        bounded = self.epoch_ms is not None
        may_stop = bounded or self.tail_live > 0
        used = 0
        epochs = 0
        depths = []
        self.stopped = 0
        self.max_active = 0
        self.max_used = 0
        t0 = time.perf_counter()
        try:
            while pending or active:
                now = time.perf_counter() - t0
                while pending:
                    i = pending[0]
                    wl = workloads[i]
                    arrival = wl.get("arrival", 0.0) if realtime else 0.0
                    need = footprint(wl, self.record, self.precision)
                    if arrival > now or used + need > self.budget:
                        break
                    pending.popleft()
                    a = _Active()
                    a.wl, a.arrival, a.admitted, a.bytes, a.index = wl, arrival, now, need, i
                    a.tier = 0
                    if self.split:
                        depths.append(line_depth(wl))
                        a.tier = self._tier_of(depths[-1], depths)
                    a.grid = colt.Grid(wl["grid"])
                    try:
                        a.job = colt.Job(a.grid, wl["source"], wl["params"],
                                         precision=self.precision, record=self.record)
                    except BaseException:
                        a.grid.release()
                        raise
                    used += need
                    self.max_used = max(self.max_used, used)
                    active.append(a)
                self.max_active = max(self.max_active, len(active))
                busy = set()
                for x in inflight:
                    busy |= x[1]
                # a job whose launches may have stopped is asked only when idle (its
                # status waits for its launches)
                ready = [a for a in active if not (may_stop and id(a) in busy)
                         and a.job.status()[0] < a.job.status()[1]]
                slot = None
                if ready and len(inflight) < self.depth:
                    slot, ready = self._next_epoch(ready, active, {x[2] for x in inflight})
                if slot is not None:
                    quota = max(self.min_quota, self.epoch_photons // len(ready))
                    st = streams[slot]
                    st.wait_stream(torch.cuda.current_stream())     # the jobs' uploads
                    token = 0
                    if bounded:
                        token = _EPOCH_TOKEN0 + slot
                        colt.stop_set(token, False)
                    colt.transport([a.job for a in ready], photons_per_job=quota, block=self.block,
                                   blocks_per_cu=self.blocks_per_cu,
                                   stream=ctypes.c_void_p(st.cuda_stream), stop_token=token,
                                   tail_live=self.tail_live)
                    ev = torch.cuda.Event()
                    ev.record(st)
                    inflight.append([ev, {id(a) for a in ready}, slot, time.perf_counter(), False])
                    epochs += 1
                    continue
                if inflight:
                    # wait for an epoch to end, or for the next arrival to admit it;
                    # a bounded epoch past its time is asked to stop
                    while not any(x[0].query() for x in inflight):
                        if bounded:
                            tnow = time.perf_counter()
                            for x in inflight:
                                if not x[4] and (tnow - x[3]) * 1e3 > self.epoch_ms:
                                    colt.stop_set(_EPOCH_TOKEN0 + x[2], True)
                                    x[4] = True
                                    self.stopped += 1
                        if realtime and pending and time.perf_counter() - t0 >= \
                                workloads[pending[0]].get("arrival", 0.0):
                            break
                        time.sleep(2e-4)
                    inflight = deque(x for x in inflight if not x[0].query())
                elif not active:
                    nxt = workloads[pending[0]].get("arrival", 0.0)
                    time.sleep(max(0.0, min(nxt - (time.perf_counter() - t0), 0.05)))
                    continue
                busy = set()
                for x in inflight:
                    busy |= x[1]
                still = []
                for a in active:
                    if id(a) in busy:
                        still.append(a)
                        continue
                    launched, total = a.job.status()
                    if launched < total:
                        still.append(a)
                        continue
                    out = a.job.tally(wait=True)
                    done = time.perf_counter() - t0
                    out["latency_s"] = done - a.arrival
                    out["queue_s"] = a.admitted - a.arrival
                    out["finished_s"] = done
                    results[a.index] = out
                    if on_done is not None:
                        on_done(a.index, out)
                    a.job.release()
                    a.grid.release()
                    used -= a.bytes
                active = still
        except BaseException:
            # wait for the epochs in flight, then give back every job and grid the
            # server holds, before the error goes on to the caller
            for x in inflight:
                x[0].synchronize()
            for a in active:
                a.job.release()
                a.grid.release()
            raise
        self.epochs = epochs
        self.makespan = time.perf_counter() - t0
        return results


def summarize(results, makespan):
    lat = np.array([r["latency_s"] for r in results])
    scat = sum(r["counters"]["scat_hi"] for r in results)
    return {"jobs": len(results), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "makespan_s": makespan,
            "scatterings": scat, "scatterings_per_s": scat / makespan}
