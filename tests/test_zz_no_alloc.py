"""elbm_batch_run_static (the batched run for callers that cannot allocate)
against elbm_batch_run, through the C ABI: the same lattices advance bitwise
alike, on two calls in a row (the second with fewer, smaller lattices and
fewer steps), and a call leaves the device's free memory unchanged."""
import numpy as np
import pytest

import inputs as I
import oracle as O
from gpu_helpers import lattice_from_field, lib

pytestmark = pytest.mark.gpu


def _mix():
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
    p = O.Params(n=(64, 32, 24), T=0.5, omega=1.85)
    out.append((p, I.channel_field((64, 32, 24), (1.0, 1.0, 1.0), seed_offset=13), "f16"))
    p = O.Params(n=(128, 48, 32), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.95, walls=(False, True, False),
                 force=(2e-6, 0.0, 0.0))
    out.append((p, I.channel_field((128, 48, 32), (2.0, 1.0, 1.0), seed_offset=14), "bf16"))
    return out


def _make(mix):
    return [lattice_from_field(p, fld, st) for p, fld, st in mix]


def test_static_batch_equals_batch_on_two_calls():
    import torch

    E = lib()
    mix = _mix()
    ref = _make(mix)
    got = _make(mix)
    b = E.Batch(len(ref))
    first = [7, 12, 3, 12, 5, 9]
    b.run(ref, first, use_graph=False)
    E.batch_run_static(got, first)
    torch.cuda.synchronize()
    for r, g in zip(ref, got):
        assert g.step_count == r.step_count
        assert np.array_equal(g.populations(), r.populations())
    # second call: fewer and smaller lattices (the table shrinks), fewer steps;
    # the tables of the first call must not leak into it
    sub = [0, 2, 3]
    second = [4, 6, 2]
    b.run([ref[k] for k in sub], second, use_graph=False)
    free0 = torch.cuda.mem_get_info()[0]
    E.batch_run_static([got[k] for k in sub], second)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for k in range(len(mix)):
        assert got[k].step_count == ref[k].step_count
        assert np.array_equal(got[k].populations(), ref[k].populations()), k
    b.close()


def test_static_batch_rejects_more_than_its_tables_hold():
    E = lib()
    lat = _make(_mix()[:1])[0]
    too_many = [lat] * (E.STATIC_MAX_LATTICES + 1)
    with pytest.raises(E.ElbmError) as ei:
        E.batch_run_static(too_many, [1] * len(too_many))
    assert ei.value.status == E.EINVAL
    assert "at most" in str(ei.value)
    with pytest.raises(E.ElbmError):
        E.batch_run_static([lat, lat], [1, 1])
    assert lat.step_count == 0
