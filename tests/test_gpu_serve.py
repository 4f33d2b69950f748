"""Serving loop on the GPU: requests that overlap on the device give exactly the results they
give when run alone, and every request of a short trace completes."""

import numpy as np
import pytest

from gpu_util import needs_gpu, note

pytestmark = [pytest.mark.gpu, needs_gpu]


def _reqs():
    from paper_1103_6031_amd.serve import Request
    c = lambda n, o: ((n,) * 3, (o,) * 3)        # noqa: E731
    return [Request(0, 0.0, 32, [], 1, 1.0),
            Request(1, 0.0, 32, [c(32, 8)], 2, 1.02),
            Request(2, 0.0, 64, [c(32, 24)], 2, 0.97),
            Request(3, 0.0, 64, [c(64, 16), c(32, 8)], 1, 1.01),
            Request(4, 0.0, 32, [c(32, 8), c(32, 8)], 2, 0.99),
            Request(5, 0.0, 64, [], 2, 1.03),
            Request(6, 0.0, 48, [c(32, 16)], 1, 1.04),
            # the largest shape of the serving trace: a 256^3 base with 128^3, 96^3 and 64^3 patches
            Request(7, 0.0, 256, [c(128, 96), c(96, 40), c(64, 32)], 2, 0.98)]


def test_alone_equals_mix():
    from paper_1103_6031_amd import serve
    reqs = _reqs()
    ids = [r.id for r in reqs]
    fields = serve.device_fields(serve.host_fields(reqs, workers=1))
    note("serve: %d requests in a burst over 3 slots" % len(reqs))
    mix = serve.GpuExecutor(fields, 3, keep=ids)
    srv = serve.Server(mix, lambda r: serve.footprint_bytes(r), slots=3, budget_bytes=12 << 30)
    recs = srv.run(reqs)
    assert all(r.error is None for r in recs.values()), [r.error for r in recs.values()]
    assert srv.peak_inflight >= 2
    note("serve: the same requests one at a time")
    alone = serve.GpuExecutor(fields, 1, keep=ids)
    for r in reqs:
        alone(r, 0)
    for i in ids:
        a, b = mix.outputs[i], alone.outputs[i]
        assert len(a) == len(b)
        for x, y in zip(a, b):
            for s, t in zip(x, y):
                assert np.array_equal(s.numpy(), t.numpy()), i


def test_short_trace_completes():
    from paper_1103_6031_amd import serve
    reqs = serve.trace(count=12, rate=40.0)
    note("serve: 12-request trace")
    summary, recs, _ = serve.serve_trace(reqs, slots=4, budget_gb=8.0, workers=1)
    assert summary["failed"] == 0
    assert summary["p99_ms"] >= summary["p50_ms"] > 0
    assert all(r.done >= r.admitted >= r.arrival for r in recs.values())
