"""Grad's-approximation walls on D3Q27 channels on the GPU (elbm_faces_* on a
D3Q27 FP32 lattice with one ghost row below and one above the fluid)
against the oracle of oracle/elbm_walls3d.py."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import MEASURED, lib
from oracle import elbm_walls3d as OW

pytestmark = pytest.mark.gpu

CASES = {
    # the benchmark channel's lattice, force along x, the upper wall moving
    "channel_force": dict(n=(24, 10, 12), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, force=(1e-5, 0.0, 0.0),
                          wall_u=(0.0, 0.02)),
    # cubic, resting walls, ragged extents
    "cubic_ragged": dict(n=(13, 7, 5), lam=(1.0, 1.0, 1.0), T=1 / 3, omega=1.2, wall_u=(0.0, 0.0)),
    # Sec. 3.5's stretched lattice with the multi-relaxation-time collision
    "stretched_mrt": dict(n=(16, 9, 8), lam=(1.4, 1.0, 2.0), T=0.55, omega=1.6, wall_u=(-0.01, 0.015),
                          rates=(1.2, 1.5)),
    # 16-bit storage: FP16 on the LDS-staged kernel (n_x = 64; 22 storage rows,
    # so the last tile row overhangs the periodic y axis), BF16 on the
    # register-pull kernel
    "f16_staged": dict(n=(64, 20, 6), lam=(1.4, 1.0, 1.0), T=0.55, omega=1.6, force=(1e-5, 0.0, 0.0),
                       wall_u=(0.0, 0.02), storage="f16"),
    "bf16_register": dict(n=(24, 10, 12), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, force=(1e-5, 0.0, 0.0),
                          wall_u=(0.0, 0.02), storage="bf16"),
}
# bound on the rel-L2 of the deviations after 20 steps (see test_walls_match_oracle)
BOUND = {"f32": 1e-5, "f16": 2e-3, "bf16": 1.6e-2}


def setup(case, seed=3):
    E = lib()
    c = CASES[case]
    n, lam, T, omega = c["n"], c["lam"], c["T"], c["omega"]
    force = c.get("force", (0.0, 0.0, 0.0))
    rates = c.get("rates")
    p = O.Params(n=n, lam=lam, T=T, omega=omega, walls=(False, True, False), force=force)
    g = np.random.default_rng(seed)
    nx, ny, nz = n
    rho = 1.0 + 0.01 * g.standard_normal((nz, ny, nx))
    u = 0.03 * g.standard_normal((3, nz, ny, nx))
    u[0] += 0.05
    f0 = O.equilibrium(rho, u, T, lam, p.c) * (1.0 + 0.001 * g.standard_normal((27, nz, ny, nx)))
    w = O.equilibrium(np.ones(()), np.zeros(3), T, lam, p.c)
    S = np.empty((27, nz, ny + 2, nx))
    S[:] = w.reshape(27, 1, 1, 1)
    S[:, :, 1:ny + 1, :] = f0
    kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
    lat = E.Lattice(E.make_params((nx, ny + 2, nz), lam=lam, T=T, omega=omega, force=force,
                                  storage=c.get("storage", "f32"), **kw))
    lat.set_populations(S)
    walls = E.Faces(lat, ["periodic", "periodic", "wall", "wall"], wall_velocity=(0.0, 0.0) + tuple(c["wall_u"]))
    return p, f0, w, lat, walls, c["wall_u"], rates


@pytest.mark.parametrize("case", sorted(CASES))
def test_walls_match_oracle(case):
    """20 steps from a seeded non-equilibrium state: fluid populations within
    1e-5 rel-L2 of their deviations and 1e-6 absolute with FP32 storage. With
    16-bit storage every stored deviation is rounded each step, by at most
    its unit roundoff u (2^-11 FP16, 2^-8 BF16) and u / sqrt(3) rms; with
    omega near 2, which damps the non-equilibrium part little, 20 such
    roundings add up like a random walk to about sqrt(20 / 3) u = 1.3e-3
    (FP16) and 1.0e-2 (BF16) of the deviations: bounds 2e-3 and 1.6e-2. The
    initial state is the stored (rounded) one on both sides."""
    p, f, w, lat, walls, wall_u, rates = setup(case)
    storage = CASES[case].get("storage", "f32")
    if storage != "f32":
        f = lat.populations()[:, :, 1:p.n[1] + 1, :]  # the rounded initial state
        assert lat.kernel_info()["kernel"] == ("staged" if storage == "f16" else "register")
    steps = 20
    walls.step(steps)
    g = lat.populations()[:, :, 1:p.n[1] + 1, :]
    f = OW.run(f, p, steps, wall_u=wall_u, rates=rates)
    W = w.reshape(27, 1, 1, 1)
    e = float(np.linalg.norm((g - f).ravel()) / np.linalg.norm((f - W).ravel()))
    MEASURED.append(dict(test="walls3d_vs_oracle", case=case, storage=storage, component="dev_rel_l2", measured=e,
                         target=BOUND[storage], bound=BOUND[storage]))
    assert e <= BOUND[storage], e
    if storage == "f32":
        assert np.abs(g - f).max() <= 1e-6
    walls.close()
    lat.close()


def test_couette_between_grad_walls_3d():
    """Steady plane Couette flow between a resting and a moving Grad wall on
    the D3Q27 lattice: the straight line through the halfway walls to 1e-5
    of the wall speed, no spanwise or normal velocity."""
    E = lib()
    nx, ny, nz, uw = 4, 16, 4, 0.02
    lat = E.Lattice(E.make_params((nx, ny + 2, nz), T=1 / 3, omega=1.2))
    lat.init(np.ones((nz, ny + 2, nx)), np.zeros((3, nz, ny + 2, nx)))
    walls = E.Faces(lat, ["periodic", "periodic", "wall", "wall"], wall_velocity=(0.0, 0.0, 0.0, uw))
    walls.step(4000)
    _, u = lat.fields()
    y = np.arange(ny) + 0.5
    prof = u[0][0, 1:ny + 1, 0]
    err = float(np.abs(prof - uw * y / ny).max() / uw)
    MEASURED.append(dict(test="walls3d_couette", case=f"{ny} rows", storage="f32", component="max_err/uw",
                         measured=err, target=1e-5, bound=1e-5))
    assert err < 1e-5, err
    assert np.abs(u[1][:, 1:ny + 1]).max() < 1e-4 * uw
    assert np.abs(u[2][:, 1:ny + 1]).max() < 1e-4 * uw
    walls.close()
    lat.close()


def test_walls3d_reject_unsupported_lattices():
    E = lib()
    lat16 = E.Lattice(E.make_params((8, 8, 8), T=1 / 3, omega=1.2, storage="f16", u_adv=(0.05, 0.0, 0.0)))
    with pytest.raises(E.ElbmError) as ei:  # walls need the rest reference
        E.Faces(lat16, ["periodic", "periodic", "wall", "wall"])
    assert ei.value.status == E.EUNSUPPORTED
    latw = E.Lattice(E.make_params((8, 8, 8), T=1 / 3, omega=1.2, walls=(False, True, False)))
    with pytest.raises(E.ElbmError) as ei:
        E.Faces(latw, ["periodic", "periodic", "wall", "wall"])
    assert ei.value.status == E.EINVAL
    lat = E.Lattice(E.make_params((8, 8, 8), T=1 / 3, omega=1.2))
    with pytest.raises(E.ElbmError) as ei:  # only the y faces take walls
        E.Faces(lat, ["wall", "wall", "periodic", "periodic"])
    assert ei.value.status == E.EUNSUPPORTED
    with pytest.raises(E.ElbmError) as ei:  # one kind per face
        E.Faces(lat, ["periodic", "periodic", ["wall"] * 8, "wall"])
    assert ei.value.status == E.EUNSUPPORTED
    for L in (lat16, latw, lat):
        L.close()
