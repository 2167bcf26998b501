"""Continuous batching: requests that arrive while others run are admitted as
memory and slots free up, and every served result is bitwise the solo result."""
import numpy as np
import pytest

import inputs as I
import oracle as O
from gpu_helpers import MEASURED, rel_l2
from paper_2101_04550_amd import elbm as E
from paper_2101_04550_amd import serving as SV

pytestmark = pytest.mark.gpu


def small_stream():
    """12 mixed requests arriving within 50 ms: D2Q9 waves / shear layers and
    D3Q27 turbulence boxes, cubic and stretched, FP32 and FP16."""
    reqs = []
    specs = [
        ("shear", (64, 64), (1.0, 1.0), 1 / 3, 1.8, 120, "f32"),
        ("dsl", (64, 128), (2.0, 1.0), 0.5, 1.97, 80, "f16"),
        ("hit", (32, 32, 32), (1.0, 1.0, 1.0), 0.5, 1.9, 60, "f32"),
        ("shear", (128, 128), (1.0, 1.0), 0.5, 1.8, 200, "f16"),
        ("hit", (24, 48, 48), (2.0, 1.0, 1.0), 1 / 3, 1.7, 90, "f16"),
        ("dsl", (256, 256), (1.0, 1.0), 1 / 3, 1.96, 40, "f32"),
        ("shear", (32, 64), (2.0, 1.0), 1 / 3, 1.8, 150, "f32"),
        ("hit", (48, 48, 48), (1.0, 1.0, 1.0), 0.5, 1.95, 130, "f32"),
        ("dsl", (128, 128), (1.0, 1.0), 0.5, 1.97, 55, "f16"),
        ("shear", (64, 64), (1.0, 1.0), 0.5, 1.8, 33, "f16"),
        ("hit", (32, 32, 32), (1.0, 1.0, 1.0), 1 / 3, 1.8, 171, "f16"),
        ("dsl", (32, 64), (2.0, 1.0), 1 / 3, 1.9, 99, "f32"),
    ]
    for rid, (kind, n, lam, T, om, steps, st) in enumerate(specs):
        uadv = (0.1, 0.0) if kind == "shear" else None
        reqs.append(SV.Request(rid, kind, n, lam, T, om, steps, st, 0.004 * rid, u_adv=uadv))
    for r in reqs:
        if r.kind == "shear":
            f = I.shear_wave_axis(r.n, U0=0.0, A=0.01, lam=r.lam)
        elif r.kind == "dsl":
            f = I.double_shear_layer(r.n, lam=r.lam)
        else:
            N = r.n[1]
            f = I.hit_field(N, k0=4.0, urms=0.05, seed_offset=30 + r.rid)
            if r.n[0] != N:
                f = I.Field(f.rho[:, :, ::2].copy(), f.u[:, :, :, ::2].copy(), r.n, r.lam)
        r.rho, r.u = np.ascontiguousarray(f.rho), np.ascontiguousarray(f.u)
    return reqs


def solo_checksum(r):
    lat = E.Lattice(r.params())
    lat.init(r.rho, r.u)
    lat.step(r.steps)
    cs = SV.state_checksum(lat)
    lat.close()
    return cs


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_results_equal_solo_under_queueing(use_graph):
    reqs = small_stream()
    sizes = [E.query_bytes(r.params()) for r in reqs]
    budget = 3 * max(sizes)  # only a few lattices fit at once: later arrivals queue
    srv = SV.Server(budget, max_slots=4, quantum=37, use_graph=use_graph, checksums=True)
    res = srv.run(reqs)
    srv.close()
    assert sorted(res) == [r.rid for r in reqs]
    assert srv.peak_used <= budget
    assert srv.peak_slots <= 4
    assert srv.rounds > 3
    for r in reqs:
        got = res[r.rid]
        assert got.finished >= got.admitted >= r.arrival - 1e-9
        assert got.steps == r.steps
        assert got.checksum == solo_checksum(r), r.rid
        assert np.isfinite(got.ke) and got.min_rho > 0


def test_served_results_match_oracle():
    """Served results against the FP64 oracle, not only against solo GPU runs:
    an FP32 shear wave (advected reference), an FP32 turbulence box and an
    FP16 shear wave, each run by the oracle from the request's own fields.
    Velocity rel-L2 per component within 1e-5 (FP32) and 1e-3 (FP16)."""
    reqs = small_stream()
    srv = SV.Server(3 * max(E.query_bytes(r.params()) for r in reqs), max_slots=4, quantum=37, keep_fields=True)
    res = srv.run(reqs)
    srv.close()
    for rid in (0, 2, 9):
        r = reqs[rid]
        p = O.Params(n=r.n, lam=r.lam, T=r.T, omega=r.omega)
        fo = O.run(O.init_state(r.rho, r.u, p, u_adv=r.u_adv), p, r.steps)
        _, uo = O.velocity(fo, p)
        gate = 1e-5 if r.storage == "f32" else 1e-3
        for a in range(p.D):
            if np.abs(uo[a]).max() == 0.0:
                continue
            e = rel_l2(res[rid].u[a], uo[a])
            MEASURED.append(dict(test="served_vs_oracle", case=f"{r.kind} {r.n} {r.steps} steps", storage=r.storage,
                                 component=f"u{a}", measured=e, target=gate, bound=gate))
            assert e <= gate, (rid, a, e)


def test_stream_statistics_on_gpu():
    reqs = small_stream()
    srv = SV.Server(1 << 34, max_slots=16, quantum=50)
    res = srv.run(reqs)
    srv.close()
    s = SV.summarize(res, srv.makespan)
    assert s["requests"] == len(reqs)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert s["solves_per_s"] > 0 and s["sustained_glups"] > 0


def test_admission_overlaps_the_running_round():
    """A request admitted while a round runs uploads on its own stream: the
    admission returns while the round is still on the GPU, in a fraction of
    the round's time (host timing)."""
    import time

    import torch

    big = SV.Request(0, "hit", (192, 192, 192), (1.0, 1.0, 1.0), 0.5, 1.9, 400, "f32", 0.0)
    f = I.hit_field(192, k0=4.0, urms=0.05, seed_offset=40)
    big.rho, big.u = np.ascontiguousarray(f.rho), np.ascontiguousarray(f.u)
    small = small_stream()[:3]
    srv = SV.Server(1 << 34, max_slots=8, quantum=400)
    a_big = srv._admit(big, 0.0)
    warm = srv._admit(small[0], 0.0)  # first admission pays one-time costs
    srv._release(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.batch.run([a_big.lat], [400], use_graph=True)
    round_end = torch.cuda.Event()
    round_end.record(torch.cuda.current_stream())  # the caller's stream waits for the round
    t1 = time.perf_counter()
    joined = [srv._admit(r, 0.0) for r in small[1:]]
    t2 = time.perf_counter()
    still_running = not round_end.query()
    round_end.synchronize()
    t3 = time.perf_counter()
    MEASURED.append(dict(test="admission_overlap", case="192^3 round of 400 steps", storage="f32",
                         component="host_s", measured=t2 - t1, target=None, bound=0.5 * (t3 - t0)))
    for a in joined + [a_big]:
        srv._release(a)
    srv.close()
    assert still_running, (t2 - t1, t3 - t0)
    assert t2 - t1 < 0.5 * (t3 - t0), (t2 - t1, t3 - t0)
