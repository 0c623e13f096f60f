"""Scheduling logic of the serving loop on the CPU: admission by memory,
continuous batching over lanes, per-stream ordering, failure isolation,
drain, latency statistics and the Poisson trace.  A fake executor stands in
for the device (completion after a simulated service time)."""
import numpy as np
import pytest

from paper_1910_01997_amd.serve import (Executor, MemoryPool, Request, Server, latency_stats,
                                        poisson_arrivals)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    def __init__(self, clock, lanes=2, service=1.0, sizes=None, fail_streams=(), fail_launch=()):
        self.clock = clock
        self.lanes = lanes
        self.service = service
        self.sizes = sizes or {}
        self.fail_streams = set(fail_streams)
        self.fail_launch = set(fail_launch)
        self.log = []            # (event, time, lane, [rids])
        self.inflight_streams = set()

    def request_bytes(self, req):
        return self.sizes.get(req.stream, 100)

    def launch(self, lane, batch):
        if any(r.stream in self.fail_launch for r in batch):
            raise RuntimeError("device refused")
        for r in batch:
            assert r.stream not in self.inflight_streams, "two requests of one stream in flight"
            self.inflight_streams.add(r.stream)
        self.log.append(("launch", self.clock(), lane, [r.rid for r in batch]))
        return {"end": self.clock() + self.service, "batch": batch, "lane": lane}

    def poll(self, h):
        return self.clock() >= h["end"]

    def finish(self, h):
        for r in h["batch"]:
            self.inflight_streams.discard(r.stream)
        self.log.append(("finish", self.clock(), h["lane"], [r.rid for r in h["batch"]]))
        return ["boom" if r.stream in self.fail_streams else None for r in h["batch"]]


def _run(server, clock, arrivals, step=0.25, horizon=100.0):
    arrivals = sorted(arrivals)
    i = 0
    while clock.t < horizon:
        while i < len(arrivals) and arrivals[i][0] <= clock.t:
            t, s = arrivals[i]
            server.submit(Request(stream=s, arrival=t, frame_index=0))
            i += 1
        server.tick()
        if i == len(arrivals) and server.idle():
            break
        clock.t += step
    return server.completed


def test_memory_pool_never_exceeds_budget():
    p = MemoryPool(1024)
    a = p.try_take(600)                 # 768 bytes with the 256-byte alignment
    assert a == 0
    assert p.try_take(500) is None      # 512 more do not fit
    p.give(a, 600)
    assert p.used == 0
    assert p.try_take(1024) == 0
    with pytest.raises(ValueError):
        p.try_take(1025)


def test_memory_pool_first_fit_and_merging():
    p = MemoryPool(4 * 256)
    offs = [p.try_take(256) for _ in range(4)]
    assert offs == [0, 256, 512, 768] and p.try_take(1) is None
    p.give(256, 256)
    p.give(768, 256)
    # two free regions of 256, not adjacent: 512 does not fit
    assert p.try_take(512) is None
    p.give(512, 256)                    # merges 256..1024 into one region
    assert p.try_take(768) == 256
    assert p.used == 1024 and p.peak == 1024


def test_admission_waits_for_memory_and_is_fifo():
    clock = FakeClock()
    ex = FakeExecutor(clock, lanes=4, service=1.0, sizes={s: 256 for s in range(10)})
    srv = Server(ex, pool_bytes=3 * 256 + 100, clock=clock)
    done = _run(srv, clock, [(0.0, s) for s in range(6)])
    assert len(done) == 6 and all(r.error is None for r in done)
    assert srv.pool.peak <= 3 * 256
    assert srv.pool.used == 0
    # only three requests fit at once: the later ones were admitted after a completion
    adm = sorted(done, key=lambda r: r.rid)
    assert max(r.admitted for r in adm[:3]) == 0.0
    assert min(r.admitted for r in adm[3:]) >= 1.0
    # admission order follows arrival order
    assert [r.rid for r in sorted(done, key=lambda r: (r.admitted, r.rid))] == [1, 2, 3, 4, 5, 6]


def test_a_request_waiting_for_its_stream_holds_no_memory():
    """Stream 0 sends three requests at once; stream 1's request, arriving
    after them, is admitted beside stream 0's first one instead of queueing
    behind requests that could not run anyway."""
    clock = FakeClock()
    ex = FakeExecutor(clock, lanes=2, service=1.0, sizes={0: 256, 1: 256})
    srv = Server(ex, pool_bytes=2 * 256, clock=clock)
    done = _run(srv, clock, [(0.0, 0), (0.0, 0), (0.0, 0), (0.1, 1)])
    by_rid = {r.rid: r for r in done}
    assert by_rid[4].stream == 1 and by_rid[4].admitted < 0.5
    assert by_rid[2].admitted >= 1.0 and by_rid[3].admitted >= 2.0
    assert srv.pool.peak <= 2 * 256


def test_requests_larger_than_the_pool_are_refused_at_submission():
    clock = FakeClock()
    ex = FakeExecutor(clock, sizes={0: 2048})
    srv = Server(ex, pool_bytes=1024, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(Request(stream=0, arrival=0.0, frame_index=0))
    assert srv.idle()


def test_continuous_batching_uses_free_lanes_without_waiting_for_the_batch():
    clock = FakeClock()
    ex = FakeExecutor(clock, lanes=2, service=2.0)
    srv = Server(ex, pool_bytes=10 ** 9, clock=clock)
    # two requests at t=0 go out together; three arriving at t=0.5 use the
    # second lane at once instead of waiting for the first batch
    done = _run(srv, clock, [(0.0, 0), (0.0, 1), (0.5, 2), (0.5, 3), (0.5, 4)])
    launches = [e for e in ex.log if e[0] == "launch"]
    assert launches[0][1] == 0.0 and sorted(launches[0][3]) == [1, 2]
    assert launches[1][1] == 0.5 and sorted(launches[1][3]) == [3, 4, 5]
    assert launches[1][2] != launches[0][2]
    assert len(done) == 5


def test_one_stream_never_has_two_requests_in_flight_and_keeps_order():
    clock = FakeClock()
    ex = FakeExecutor(clock, lanes=3, service=1.0)
    srv = Server(ex, pool_bytes=10 ** 9, clock=clock)
    arr = [(0.0, 7), (0.0, 7), (0.1, 7), (0.1, 2), (0.2, 7)]
    done = _run(srv, clock, arr)
    mine = sorted([r for r in done if r.stream == 7], key=lambda r: r.done)
    assert [r.rid for r in mine] == sorted(r.rid for r in mine)
    # each of stream 7's requests starts after the previous one finished
    for a, b in zip(mine, mine[1:]):
        assert b.launched >= a.done


def test_failures_are_isolated_and_release_memory():
    clock = FakeClock()
    ex = FakeExecutor(clock, lanes=2, service=1.0, fail_streams={3}, fail_launch={5})
    srv = Server(ex, pool_bytes=10 ** 9, clock=clock)
    done = _run(srv, clock, [(0.0, s) for s in range(4)] + [(2.0, 5), (2.0, 6)])
    by = {r.stream: r for r in done}
    assert by[3].error == "boom"
    assert by[5].error.startswith("launch failed")
    # stream 6 was in the refused launch batch too; everything else succeeded
    assert all(by[s].error is None for s in (0, 1, 2))
    assert srv.pool.used == 0 and srv.idle()
    stats = latency_stats(done)
    assert stats["errors"] == sum(1 for r in done if r.error)


def test_max_batch_caps_a_launch():
    clock = FakeClock()
    ex = FakeExecutor(clock, lanes=1, service=1.0)
    srv = Server(ex, pool_bytes=10 ** 9, max_batch=3, clock=clock)
    _run(srv, clock, [(0.0, s) for s in range(7)])
    sizes = [len(e[3]) for e in ex.log if e[0] == "launch"]
    assert sizes == [3, 3, 1]


def test_latency_statistics():
    rs = []
    for i, lat in enumerate([1.0, 2.0, 3.0, 4.0, 100.0]):
        r = Request(stream=0, arrival=float(i), frame_index=0)
        r.done = r.arrival + lat / 1e3
        rs.append(r)
    st = latency_stats(rs)
    assert st["count"] == 5
    assert st["p50_ms"] == pytest.approx(3.0)
    assert st["max_ms"] == pytest.approx(100.0)


def test_poisson_trace_rate_and_determinism():
    a = poisson_arrivals(200.0, 20.0, 32, seed=599, frames_per_stream=4)
    b = poisson_arrivals(200.0, 20.0, 32, seed=599, frames_per_stream=4)
    assert a == b
    assert 3700 < len(a) < 4300
    gaps = np.diff([t for t, _, _ in a])
    assert np.mean(gaps) == pytest.approx(1 / 200.0, rel=0.05)
    streams = np.bincount([s for _, s, _ in a], minlength=32)
    assert streams.min() > 80
    assert all(0 <= f < 4 for _, _, f in a)


def test_snapshot_archive_round_trip(tmp_path):
    """Stream snapshots go to .npz and back exactly, dtypes included, with no
    pickled objects in the archive."""
    from paper_1910_01997_amd.serve import load_snapshot, save_snapshot
    rng = np.random.default_rng(3)
    snap = {"state_inv_depth": rng.random(12, dtype=np.float32),
            "state_flags": rng.integers(0, 1 << 30, 12).astype(np.int32),
            "kf_image": rng.random((4, 6)).astype(np.float16),
            "nbr_images": rng.integers(0, 256, (3, 4, 6)).astype(np.uint8),
            "R": rng.random((3, 3, 3)), "t": rng.random((3, 3)),
            "oldest": np.array(2, np.int64), "first": np.array(False)}
    p = tmp_path / "s.npz"
    save_snapshot(p, snap)
    back = load_snapshot(p)
    assert back.keys() == snap.keys()
    for k in snap:
        assert back[k].dtype == snap[k].dtype and np.array_equal(back[k], snap[k]), k
