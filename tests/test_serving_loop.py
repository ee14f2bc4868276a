"""The serving loop on the CPU, with the library and the device replaced by
fakes: every job is served to completion exactly once, results come back in
input order, the memory budget holds, a job whose launches may stop (tail rule
or time bound) is in one epoch at a time and its suspended photons are taken
again, and with the split no launch mixes tiers."""
import itertools

import pytest

from paper_1409_4480_amd import inputs, serving


class _Launch:
    def __init__(self, jobs):
        self.jobs = jobs
        self.done = False

    def finish(self):
        if not self.done:
            self.done = True
            for j in self.jobs:
                j.inflight -= 1


class _Stream:
    ids = itertools.count(1)

    def __init__(self):
        self.cuda_stream = next(self.ids)
        self.last = None

    def wait_stream(self, other):
        pass


class _Event:
    def __init__(self):
        self.polls = 0
        self.launch = None

    def record(self, stream):
        self.launch = stream.last

    def query(self):
        self.polls += 1
        if self.polls >= 3 and self.launch is not None:
            self.launch.finish()
        return self.polls >= 3

    def synchronize(self):
        self.polls = max(self.polls, 3)
        if self.launch is not None:
            self.launch.finish()


class _Cuda:
    Stream = _Stream
    Event = _Event

    @staticmethod
    def current_stream():
        return _Stream()


class _Grid:
    def __init__(self, desc):
        self.desc = desc
        self.released = False

    def release(self):
        self.released = True


class _Job:
    def __init__(self, grid, source, params, precision=None, record=False):
        self.grid = grid
        self.total = int(params["n_photons"])
        self.seed = int(params["seed"])
        self.taken = 0          # photons handed to launches, suspended ones included
        self.susp = 0
        self.inflight = 0
        self.released = False
        self.tallied = 0

    def status(self):
        return self.taken - self.susp, self.total

    def tally(self, wait=True):
        assert self.inflight == 0 and self.susp == 0 and self.taken == self.total
        self.tallied += 1
        return {"counters": {"emitted": self.total, "scat_hi": 7 * self.total},
                "seed": self.seed}

    def release(self):
        self.released = True


class _Lib:
    """The library calls the server makes, recording every launch."""

    def __init__(self):
        self.fail_at = None
        self.launches = []
        self.jobs = []
        self.tier_of = {}
        self.stop = {}
        self.resumed = 0

    def transport(self, jobs, photons_per_job=0, stream=None, stop_token=0, tail_live=0,
                  **kw):
        if self.fail_at is not None and len(self.launches) == self.fail_at:
            raise serving.colt.ColtError("launch failed")
        may_stop = tail_live > 0 or stop_token != 0
        for j in jobs:
            assert not j.released
            assert not (may_stop and j.inflight), "a job in two epochs whose launches may stop"
            new = min(photons_per_job or j.total, j.total - j.taken)
            resumed, j.susp = j.susp, 0
            self.resumed += resumed
            j.taken += new
            # the tail rule leaves some of the launch's photons suspended
            if tail_live > 0 and new + resumed >= 4:
                j.susp = 2
            j.inflight += 1
        if jobs:
            tiers = {self.tier_of.get(j.seed) for j in jobs}
            self.launches.append((tuple(j.seed for j in jobs), tiers))
        return _Launch(jobs)

    def stop_set(self, token, value=True):
        self.stop[token] = value


@pytest.fixture
def fake(monkeypatch):
    lib = _Lib()
    monkeypatch.setattr(serving.colt, "Grid", _Grid)

    def job(*a, **k):
        lib.jobs.append(_Job(*a, **k))
        return lib.jobs[-1]
    monkeypatch.setattr(serving.colt, "Job", job)
    monkeypatch.setattr(serving.colt, "stop_set", lib.stop_set)

    def transport(jobs, stream=None, **kw):
        launch = lib.transport(jobs, stream=stream, **kw)
        _streams_by_handle[stream.value].last = launch
    monkeypatch.setattr(serving.colt, "transport", transport)
    return lib


_streams_by_handle = {}


class _TrackedStream(_Stream):
    def __init__(self):
        super().__init__()
        _streams_by_handle[self.cuda_stream] = self


class _TrackedCuda(_Cuda):
    Stream = _TrackedStream


class _TrackedTorch:
    cuda = _TrackedCuda


def _server(**kw):
    srv = serving.Server(budget_bytes=kw.pop("budget_bytes", 1 << 40), **kw)
    srv._torch = _TrackedTorch
    return srv


def _stream(n=12, seed=21):
    return inputs.job_stream(n_jobs=n, seed=seed, n_range=(16, 24), tau_range=(1e3, 1e7),
                             ph_range=(50, 5000))


@pytest.mark.parametrize("split,tail,bound", [(False, 0, None), (True, 0, None),
                                              (True, 16, None), (False, 16, None),
                                              (True, 0, 0.0)])
def test_every_job_is_served_once_in_input_order(fake, split, tail, bound):
    jobs = _stream()
    done = []
    srv = _server(epoch_photons=4000, min_quota=100, split=split, tail_live=tail,
                  epoch_ms=bound)
    out = srv.run(jobs, realtime=False, on_done=lambda i, r: done.append(i))
    assert sorted(done) == list(range(len(jobs)))
    for wl, r in zip(jobs, out):
        assert r["seed"] == wl["params"]["seed"]
        assert r["counters"]["emitted"] == wl["params"]["n_photons"]
        assert r["latency_s"] >= 0.0 and r["queue_s"] >= 0.0
    assert srv.epochs == len(fake.launches) and srv.epochs > 1
    assert srv.max_active == len(jobs)
    assert len(fake.jobs) == len(jobs)
    assert all(j.released and j.grid.released and j.tallied == 1 for j in fake.jobs)
    if tail:
        assert fake.resumed > 0
    if bound is not None:
        assert srv.stopped > 0 and any(fake.stop.values())


def test_split_launches_never_mix_tiers(fake):
    jobs = _stream(n=16, seed=22)
    srv = _server(epoch_photons=4000, min_quota=100)
    depths = []
    for wl in jobs:                     # admission order is input order here
        depths.append(serving.line_depth(wl))
        fake.tier_of[wl["params"]["seed"]] = srv._tier_of(depths[-1], depths)
    assert set(fake.tier_of.values()) == {0, 1}
    srv.run(jobs, realtime=False)
    assert all(len(tiers) == 1 for _, tiers in fake.launches)
    assert {t for _, tiers in fake.launches for t in tiers} == {0, 1}


def test_budget_admits_jobs_in_turn(fake):
    jobs = _stream(n=8, seed=23)
    sizes = [serving.footprint(wl) for wl in jobs]
    srv = _server(budget_bytes=int(1.5 * max(sizes)), epoch_photons=4000, min_quota=100)
    out = srv.run(jobs, realtime=False)
    assert srv.max_used <= srv.budget and srv.max_active < len(jobs)
    assert [r["seed"] for r in out] == [wl["params"]["seed"] for wl in jobs]
    fat = dict(jobs[0])
    with pytest.raises(serving.colt.ColtError):
        _server(budget_bytes=sizes[0] // 2).run([fat], realtime=False)


@pytest.mark.parametrize("where", ["launch", "on_done"])
def test_an_error_releases_everything_the_server_holds(fake, where):
    """A failed launch, or a caller's callback that raises, ends the run with
    that error after the epochs in flight have finished and every job and grid
    has been released."""
    jobs = _stream(n=10, seed=24)
    srv = _server(epoch_photons=4000, min_quota=100, tail_live=16)

    def done(i, r):
        if where == "on_done":
            raise KeyError("caller")
    if where == "launch":
        fake.fail_at = 3
    with pytest.raises(serving.colt.ColtError if where == "launch" else KeyError):
        srv.run(jobs, realtime=False, on_done=done)
    assert fake.jobs and all(j.released and j.grid.released for j in fake.jobs)
    assert all(j.inflight == 0 for j in fake.jobs)
