"""Batched fused launches: every lattice advances bitwise exactly as alone,
whatever the mix, with and without HIP-graph replay."""
import numpy as np
import pytest

import inputs as I
import oracle as O
from gpu_helpers import MEASURED, dev_rel_l2, lattice_from_field, lib
from storage_rounding import round_state

pytestmark = pytest.mark.gpu


def _mix():
    """(oracle params, field, storage) of lattices of different classes and sizes."""
    out = []
    p = O.Params(n=(64, 64), T=1 / 3, omega=1.8)
    out.append((p, I.shear_wave_axis((64, 64), U0=0.1, A=0.01), "f32"))
    p = O.Params(n=(128, 256), lam=(2.0, 1.0), T=0.5, omega=1.97)
    out.append((p, I.double_shear_layer((128, 256), lam=(2.0, 1.0)), "f16"))
    p = O.Params(n=(32, 32, 32), T=0.5, omega=1.7)
    out.append((p, I.hit_field(32, k0=4.0, urms=0.05, seed_offset=11), "f32"))
    p = O.Params(n=(40, 24, 24), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, walls=(False, True, False),
                 force=(1e-5, 0.0, 0.0))
    out.append((p, I.channel_field((40, 24, 24), (2.0, 1.0, 1.0)), "f16"))
    p = O.Params(n=(48, 48, 48), T=1 / 3, omega=1.5)
    out.append((p, I.hit_field(48, k0=4.0, urms=0.05, seed_offset=12), "bf16"))
    p = O.Params(n=(96, 64, 40), T=0.5, omega=1.6)
    out.append((p, I.uniform((96, 64, 40), u0=(0.02, 0.0, -0.01)), "f32"))
    # LDS-staged kernel class (16-bit, periodic, n_x % 64 == 0, n_y % 16 == 0):
    # two lattices in one table, and the forced variant
    p = O.Params(n=(64, 32, 24), T=0.5, omega=1.85)
    out.append((p, I.channel_field((64, 32, 24), (1.0, 1.0, 1.0), seed_offset=13), "f16"))
    p = O.Params(n=(128, 16, 12), lam=(2.0, 1.0, 1.0), T=0.4, omega=1.6)
    out.append((p, I.uniform((128, 16, 12), u0=(0.01, -0.02, 0.005)), "f16"))
    p = O.Params(n=(64, 16, 20), T=1 / 3, omega=1.3, force=(1e-4, -2e-4, 5e-5))
    out.append((p, I.uniform((64, 16, 20), u0=(0.0, 0.01, 0.0)), "bf16"))
    # the staged class again, n_y = 24: its last tile row overhangs the periodic
    # y axis (the tile variant chosen per tile, behind other lattices' tiles)
    p = O.Params(n=(64, 24, 10), lam=(1.0, 1.5, 1.0), T=0.5, omega=1.75)
    out.append((p, I.channel_field((64, 24, 10), (1.0, 1.5, 1.0), seed_offset=14), "f16"))
    return out


def _make(mix):
    return [lattice_from_field(p, fld, st) for p, fld, st in mix]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_alone_bitwise(use_graph):
    E = lib()
    mix = _mix()
    steps = [7, 12, 3, 12, 9, 1, 5, 12, 8, 6]
    alone = _make(mix)
    for lat, k in zip(alone, steps):
        lat.step(k)
    ref = [lat.populations() for lat in alone]
    batched = _make(mix)
    b = E.Batch(len(batched))
    b.run(batched, steps, use_graph=use_graph)
    for lat, k, r in zip(batched, steps, ref):
        assert lat.step_count == k
        assert np.array_equal(lat.populations(), r)
    b.close()


def test_batch_matches_oracle():
    """Every lattice of a graph-replayed batched run against the FP64 oracle run
    from the same stored initial state: the population deviations f - w within
    1e-5 (FP32 storage), or, for 16-bit storage, the oracle's state rounded to
    the format after every step as the library stores it, within 1e-3 (FP16)
    and 1e-2 (BF16)."""
    E = lib()
    mix = _mix()
    steps = [7, 12, 3, 12, 9, 1, 5, 12, 8, 6]
    lats = _make(mix)
    f0 = [lat.populations() for lat in lats]
    b = E.Batch(len(lats))
    b.run(lats, steps, use_graph=True)
    b.close()
    gate = {"f32": 1e-5, "f16": 1e-3, "bf16": 1e-2}
    for (p, _, st), lat, k, f in zip(mix, lats, steps, f0):
        w = O.reference_weights(p).reshape((-1,) + (1,) * p.D)
        for _ in range(k):
            f = O.step(f, p)
            if st != "f32":
                f = round_state(f, w, st)
        e = dev_rel_l2(lat.populations(), f, p)
        MEASURED.append(dict(test="batch_vs_oracle", case=f"{p.n} {st} {k} steps", storage=st,
                             component="f-w", measured=e, target=gate[st], bound=gate[st]))
        assert e <= gate[st], (p.n, st, k, e)


def test_graph_reuse_across_mixes_and_continuation():
    """One captured graph serves different mixes of the same size class; a batch
    run followed by solo steps continues the same trajectory."""
    E = lib()
    mix = _mix()
    total = [20] * 10
    alone = _make(mix)
    for lat, k in zip(alone, total):
        lat.step(k)
    ref = [lat.populations() for lat in alone]
    lats = _make(mix)
    b = E.Batch(len(lats))
    # three rounds of at most 8 steps; lattices drop in and out of the mix
    b.run(lats, [8, 8, 0, 8, 3, 8, 8, 0, 5, 8], use_graph=True)
    b.run(lats, [8, 5, 8, 8, 8, 8, 8, 8, 8, 4], use_graph=True)
    done = [lat.step_count for lat in lats]
    b.run(lats[::-1], [min(8, 20 - d) for d in done[::-1]], use_graph=True)
    for lat in lats:
        rest = 20 - lat.step_count
        lat.step(rest)
    for lat, r in zip(lats, ref):
        assert lat.step_count == 20
        assert np.array_equal(lat.populations(), r)
    b.close()


def test_batch_rejects_bad_input():
    E = lib()
    mix = _mix()[:2]
    lats = _make(mix)
    b = E.Batch(2)
    with pytest.raises(E.ElbmError):
        b.run([lats[0], lats[0]], [1, 1])
    with pytest.raises(E.ElbmError):
        b.run(lats + lats[:1], [1, 1, 1])
    with pytest.raises(E.ElbmError):
        b.run(lats, [1, -1])
    b.close()
