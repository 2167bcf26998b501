"""Full-size parity in the launch configuration bench.py times: one step of the
256^3 turbulence lattice and of the 384x192x192 stretched channel, checked at
sampled nodes that the oracle updates one by one (oracle.step_node) from the
GPU's own input state. Samples include tile, chunk and wall boundaries."""
import numpy as np
import pytest

import inputs as I
import oracle as O
from gpu_helpers import lattice_from_field

pytestmark = pytest.mark.gpu


def _nodes(n, special, count, seed):
    g = np.random.default_rng(seed)
    pts = set()
    for x in special[0]:
        for y in special[1]:
            for z in special[2]:
                pts.add((z % n[2], y % n[1], x % n[0]))
    for _ in range(count):
        pts.add(tuple(int(g.integers(0, m)) for m in (n[2], n[1], n[0])))
    return sorted(pts)


def _check(lat, p, nodes, tol_abs, tol_rel):
    f0 = lat.populations()
    lat.step(1)
    f1 = lat.populations()
    w = O.reference_weights(p).reshape(-1)
    worst = 0.0
    for idx in nodes:
        o = O.step_node(f0, p, idx)
        g = f1[(slice(None),) + idx]
        err = np.abs(g - o)
        assert (err <= tol_abs + tol_rel * np.abs(o - w)).all(), (idx, err.max())
        worst = max(worst, float(err.max()))
    return worst


@pytest.mark.parametrize("storage,tol_abs,tol_rel", [("f32", 2e-7, 0.0), ("f16", 1e-7, 2.0 ** -10)])
def test_hit_256_cube_one_step_sampled(storage, tol_abs, tol_rel):
    n = (256, 256, 256)
    fld = I.hit_field(256, k0=4.0, urms=0.05)
    p = O.Params(n=n, T=0.5, omega=1.892885)
    lat = lattice_from_field(p, fld, storage)
    special = ([0, 1, 63, 64, 127, 128, 255], [0, 7, 8, 255], [0, 31, 32, 33, 255])
    nodes = _nodes(n, special, 120, seed=3)
    _check(lat, p, nodes, tol_abs, tol_rel)


@pytest.mark.parametrize("storage,tol_abs,tol_rel,kernel", [("f32", 2e-7, 0.0, "register"),
                                                           ("f16", 1e-7, 2.0 ** -10, "staged")])
def test_channel_full_size_one_step_sampled(storage, tol_abs, tol_rel, kernel):
    """384 x 192 x 192 channel (walls in y, Re_tau = 180 force): FP32 takes the
    register-pull kernel, FP16 the LDS-staged kernel with walls and force --
    the two kernels of the bench's channel workload, in its launch shape."""
    n, lam = (384, 192, 192), (2.0, 1.0, 1.0)
    omega = 1.976785
    nu = (1 / omega - 0.5) * 0.5
    g = 180.0 ** 2 * nu ** 2 / 96.0 ** 3
    fld = I.channel_field(n, lam)
    p = O.Params(n=n, lam=lam, T=0.5, omega=omega, walls=(False, True, False), force=(g, 0.0, 0.0))
    lat = lattice_from_field(p, fld, storage)
    assert lat.kernel_info()["kernel"] == kernel
    special = ([0, 63, 64, 383], [0, 1, 7, 8, 15, 16, 190, 191], [0, 23, 24, 27, 28, 191])
    nodes = _nodes(n, special, 120, seed=4)
    _check(lat, p, nodes, tol_abs, tol_rel)
