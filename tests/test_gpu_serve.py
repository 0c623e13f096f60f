"""Serving on the GPU: a request's result is the same alone and in the mix
(bitwise, same plan), responses carry the device state, and a short trace
completes with admission binding."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from scenegen import stream_specs

pytestmark = pytest.mark.gpu


def _specs():
    # six streams of the serving workload, reduced to 320x240 / 640x480 for speed
    out = []
    for i, sp in enumerate(stream_specs(6)):
        W, H = ((320, 240), (640, 480))[i % 2]
        out.append(dataclasses.replace(sp, width=W, height=H))
    return out


def test_alone_equals_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import serve
    from paper_1910_01997_amd import surfgn as sg
    specs = _specs()
    results = {}
    for mode in ("mix", "alone"):
        ctx = sg.Context(0)
        streams = serve.make_streams(ctx, specs, extra=2)
        ex = serve.HipExecutor(streams, lanes=2, iters=8)
        srv = serve.Server(ex, pool_bytes=1 << 30, max_batch=32 if mode == "mix" else 1)
        for s in range(len(specs)):
            srv.submit(serve.Request(stream=s, arrival=srv.clock(), frame_index=1))
            if mode == "alone":
                srv.drain()
        srv.drain()
        assert all(r.error is None for r in srv.completed)
        if mode == "mix":
            assert max(srv.batches) > 1
        else:
            assert max(srv.batches) == 1
        results[mode] = {r.stream: (r.result[0].numpy().copy(), r.result[1].numpy().copy())
                         for r in srv.completed}
        # the response holds the device state
        for r in srv.completed:
            dk = streams[r.stream].dk
            assert np.array_equal(r.result[1][0].numpy(), dk.state.inv_depth.cpu().numpy())
        for c in ex.ctxs:
            c.close()
        ctx.close()
    for s in range(len(specs)):
        assert np.array_equal(results["mix"][s][0], results["alone"][s][0]), f"depth of stream {s}"
        assert np.array_equal(results["mix"][s][1], results["alone"][s][1]), f"surfels of stream {s}"


def test_short_trace_with_binding_admission():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import serve
    specs = _specs()
    res = serve.serving_benchmark(specs=specs, rate=300.0, duration=1.5, warmup=0.2,
                                  pool_bytes=6 << 20, iters=8)
    for mode in ("served", "plain"):
        st = res[mode]
        assert st["count"] > 50 and st["errors"] == 0
        assert st["pool_peak_mb"] <= 6.0 + 1e-9
        assert st["p99_ms"] >= st["p50_ms"] > 0


def test_snapshot_resume_equals_uninterrupted(tmp_path):
    """Checkpoint / resume: a stream snapshot written to .npz after its first
    request and loaded into freshly built streams gives, for the next
    requests, bitwise the responses of the uninterrupted run."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import serve
    from paper_1910_01997_amd import surfgn as sg
    specs = _specs()[:2]

    def run(streams, frames):
        ex = serve.HipExecutor(streams, lanes=1, iters=6)
        srv = serve.Server(ex, pool_bytes=1 << 30, max_batch=1)
        out = {}
        for f in frames:
            for s in range(len(streams)):
                srv.submit(serve.Request(stream=s, arrival=srv.clock(), frame_index=f))
                srv.drain()
        assert all(r.error is None for r in srv.completed)
        for r in srv.completed:
            out[(r.stream, r.frame_index)] = (r.result[0].numpy().copy(), r.result[1].numpy().copy())
        for c in ex.ctxs:
            c.close()
        return out

    print("case snapshot after one request, resume two more", flush=True)
    ctx = sg.Context(0)
    streams = serve.make_streams(ctx, specs, extra=3)
    run(streams, [0])
    paths = []
    for s, cs in enumerate(streams):
        paths.append(tmp_path / f"stream{s}.npz")
        serve.save_snapshot(paths[-1], cs.snapshot())
    uninterrupted = run(streams, [1, 2])
    ctx.close()

    ctx2 = sg.Context(0)
    fresh = serve.make_streams(ctx2, specs, extra=3)
    for cs, p in zip(fresh, paths):
        cs.restore(serve.load_snapshot(p))
    resumed = run(fresh, [1, 2])
    assert uninterrupted.keys() == resumed.keys()
    for k in uninterrupted:
        assert np.array_equal(uninterrupted[k][0], resumed[k][0]), f"depth {k}"
        assert np.array_equal(uninterrupted[k][1], resumed[k][1]), f"surfels {k}"
    # a snapshot of another shape is refused and changes nothing
    before = fresh[0].snapshot()
    with pytest.raises(ValueError):
        fresh[0].restore(serve.load_snapshot(paths[1]))
    after = fresh[0].snapshot()
    assert all(np.array_equal(before[k], after[k]) for k in before)
    ctx2.close()
