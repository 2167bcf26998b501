"""Host-side checks of the request stream and the latency summary (no GPU)."""
import math

import numpy as np
import pytest

from paper_2101_04550_amd import serving as SV


def test_stream_is_seeded_and_shaped():
    a = SV.make_stream(400, rate=50.0, share_3d=0.1)
    b = SV.make_stream(400, rate=50.0, share_3d=0.1)
    assert [(r.kind, r.n, r.steps, r.storage, r.arrival) for r in a] == \
           [(r.kind, r.n, r.steps, r.storage, r.arrival) for r in b]
    arrivals = np.array([r.arrival for r in a])
    assert np.all(np.diff(arrivals) > 0)
    # Poisson process at 50 / s: mean gap 0.02 s
    assert abs(np.diff(arrivals).mean() - 0.02) < 0.004
    share = sum(r.kind == "hit" for r in a) / len(a)
    assert 0.05 < share < 0.16
    for r in a:
        assert 200 <= r.steps <= 5000
        assert r.storage in ("f32", "f16")
        assert r.T in (1 / 3, 0.5)
        assert 0.0 < r.omega < 2.0
        if r.lam[0] == 2.0:
            assert r.n[0] * 2 == r.n[1]   # stretched boxes keep the physical square / cube
        # positivity of the rest weight: T < lambda_min^2
        assert r.T < min(r.lam) ** 2


def test_summary_statistics():
    res = {i: SV.Result(i, 0.1 * i, 0.1 * i, 0.1 * i + 0.5 + 0.01 * i, 100, 64 * 64, 0.0, 0.0, 1.0, "")
           for i in range(100)}
    s = SV.summarize(res, 20.0)
    assert s["requests"] == 100
    assert math.isclose(s["solves_per_s"], 5.0)
    assert math.isclose(s["p50_latency_s"], 0.5 + 0.01 * 49.5, rel_tol=1e-9)
    assert s["p99_latency_s"] <= 0.5 + 0.99 + 1e-9
    assert math.isclose(s["sustained_glups"], 100 * 64 * 64 * 100 / 20.0 / 1e9)
