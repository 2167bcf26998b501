"""Open boundaries on the GPU (elbm_faces_*, D2Q9; FP32, and FP16 / BF16
storage on the flat plate's faces) against the
open-boundary oracle (oracle/elbm_faces.py): Grad's-approximation walls
(resting and moving), symmetry planes, inlets, outlets and their corners, on
cubic and stretched lattices, with and without a body force."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import MEASURED, lib
from oracle import elbm_faces as OF

pytestmark = pytest.mark.gpu

PLATE_BOTTOM = [OF.SYMMETRY] * 3 + [OF.WALL] * 9
CASES = {
    # the flat plate's faces (Sec. 3.4) on a small stretched box
    "plate": dict(n=(12, 9), lam=(2.0, 1.0), T=1 / 3, omega=1.7,
                  kinds=[OF.INLET, OF.OUTLET, PLATE_BOTTOM, OF.SYMMETRY], inlet=(0.05, 0.0)),
    # channel between a resting and a moving wall, force along x, periodic x
    "channel_force": dict(n=(10, 8), lam=(1.0, 1.0), T=1 / 3, omega=1.5,
                          kinds=[OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.WALL], wall=(0, 0, 0.0, 0.02),
                          force=(1e-5, 0.0)),
    # oblique inflow through a stretched box, periodic y
    "inlet_outlet": dict(n=(11, 7), lam=(1.4, 1.0), T=0.5, omega=1.6,
                         kinds=[OF.INLET, OF.OUTLET, OF.PERIODIC, OF.PERIODIC], inlet=(0.04, 0.01)),
    # walls normal to x (one moving along y) on a y-stretched lattice
    "x_walls": dict(n=(9, 10), lam=(1.0, 1.4), T=1 / 3, omega=1.6,
                    kinds=[OF.WALL, OF.SYMMETRY, OF.PERIODIC, OF.PERIODIC], wall=(0.01, 0, 0, 0)),
}


def setup(case, seed=1, rates=None, storage="f32"):
    E = lib()
    c = CASES[case]
    n, lam, T, omega = c["n"], c["lam"], c["T"], c["omega"]
    force = c.get("force", (0.0, 0.0))
    inlet = c.get("inlet", (0.0, 0.0))
    wall = c.get("wall", (0.0, 0.0, 0.0, 0.0))
    p = O.Params(n=n, lam=lam, T=T, omega=omega, force=force)
    fc = OF.Faces(n, c["kinds"], wall_velocity=wall, inlet_velocity=(inlet,) * 4)
    o = [0 if fc.periodic(a) else 1 for a in range(2)]
    N = (n[0] + 2 * o[0], n[1] + 2 * o[1])
    g = np.random.default_rng(seed)
    rho = 1 + 0.01 * g.standard_normal((n[1], n[0]))
    u = 0.03 * g.standard_normal((2, n[1], n[0]))
    u[0] += 0.05
    f0 = O.equilibrium(rho, u, T, lam, p.c) * (1 + 0.001 * g.standard_normal((9, n[1], n[0])))
    w = O.equilibrium(np.ones(()), np.zeros(2), T, lam, p.c)
    S = np.empty((9, N[1], N[0]))
    S[:] = w.reshape(9, 1, 1)
    S[:, o[1]:o[1] + n[1], o[0]:o[0] + n[0]] = f0
    kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
    lat = E.Lattice(E.make_params(N, lam=lam, T=T, omega=omega, force=force, storage=storage, **kw))
    lat.set_populations(S)
    faces = E.Faces(lat, [fc.node_kind[F].tolist() if not fc.periodic(F // 2) else "periodic" for F in range(4)],
                    wall_velocity=wall, inlet_velocity=(inlet,) * 4)
    return p, fc, o, f0, w, lat, faces


@pytest.mark.parametrize("case", sorted(CASES))
def test_faces_match_oracle(case):
    """30 steps from a seeded non-equilibrium state: interior populations
    within 1e-5 rel-L2 of their deviations (FP32 storage and arithmetic)."""
    p, fc, o, f, w, lat, faces = setup(case)
    steps = 30
    faces.step(steps)
    g = lat.populations()[:, o[1]:o[1] + p.n[1], o[0]:o[0] + p.n[0]]
    for _ in range(steps):
        f = OF.step_open(f, p, fc)
    W = w.reshape(9, 1, 1)
    e = float(np.linalg.norm((g - f).ravel()) / np.linalg.norm((f - W).ravel()))
    MEASURED.append(dict(test="faces_vs_oracle", case=case, storage="f32", component="dev_rel_l2", measured=e,
                         target=1e-5, bound=1e-5))
    assert e <= 1e-5, e
    assert np.abs(g - f).max() <= 1e-6
    faces.close()
    lat.close()


@pytest.mark.parametrize("case,rates", [("plate", (1.2, 1.5)), ("channel_force", (1.9, 1.1)),
                                        ("x_walls", (1.6, 1.0)), ("inlet_outlet", (1.0, 1.3))])
def test_faces_with_the_mrt_collision_match_oracle(case, rates):
    """The same faces under the multi-relaxation-time collision (the Grad
    wall's stress trace at omega_bulk): 30 steps within 1e-5 rel-L2 of the
    oracle's deviations."""
    p, fc, o, f, w, lat, faces = setup(case, rates=rates)
    steps = 30
    faces.step(steps)
    g = lat.populations()[:, o[1]:o[1] + p.n[1], o[0]:o[0] + p.n[0]]
    f = OF.run_open(f, p, fc, steps, rates=rates)
    W = w.reshape(9, 1, 1)
    e = float(np.linalg.norm((g - f).ravel()) / np.linalg.norm((f - W).ravel()))
    MEASURED.append(dict(test="faces_mrt_vs_oracle", case=case, storage="f32", component="dev_rel_l2", measured=e,
                         target=1e-5, bound=1e-5))
    assert e <= 1e-5, e
    assert np.abs(g - f).max() <= 1e-6
    faces.close()
    lat.close()


def test_couette_between_grad_walls_on_gpu():
    """Steady plane Couette flow between a resting and a moving Grad wall:
    the straight line through the halfway walls to 1e-5 of the wall speed."""
    E = lib()
    nx, ny, uw = 4, 16, 0.02
    lat = E.Lattice(E.make_params((nx, ny + 2), T=1 / 3, omega=1.2))
    lat.init(np.ones((ny + 2, nx)), np.zeros((2, ny + 2, nx)))
    faces = E.Faces(lat, ["periodic", "periodic", "wall", "wall"], wall_velocity=(0, 0, 0.0, uw))
    faces.step(4000)
    _, u = lat.fields()
    y = np.arange(ny) + 0.5
    prof = u[0][1:ny + 1, 0]
    err = float(np.abs(prof - uw * y / ny).max() / uw)
    MEASURED.append(dict(test="faces_couette", case=f"{ny} rows", storage="f32", component="max_err/uw",
                         measured=err, target=1e-5, bound=1e-5))
    assert err < 1e-5, err
    assert np.abs(u[1][1:ny + 1]).max() < 1e-6 * uw * 100
    faces.close()
    lat.close()


@pytest.mark.parametrize("storage,bound", [("f16", 2e-3), ("bf16", 1.6e-2)])
@pytest.mark.parametrize("case", ["plate", "channel_force"])
def test_faces_with_16_bit_storage_match_oracle(case, storage, bound):
    """The face kernels read the stored 16-bit deviations exactly and round
    what they write once: 20 steps from the stored (rounded) initial state
    against the FP64 oracle, deviations rel-L2 within the bound of 20
    roundings at the format's unit roundoff u (2^-11 FP16, 2^-8 BF16, u /
    sqrt(3) rms each, adding up to about sqrt(20 / 3) u: 1.3e-3 / 1.0e-2)."""
    p, fc, o, _, w, lat, faces = setup(case, storage=storage)
    f = lat.populations()[:, o[1]:o[1] + p.n[1], o[0]:o[0] + p.n[0]]
    steps = 20
    faces.step(steps)
    g = lat.populations()[:, o[1]:o[1] + p.n[1], o[0]:o[0] + p.n[0]]
    for _ in range(steps):
        f = OF.step_open(f, p, fc)
    W = w.reshape(9, 1, 1)
    e = float(np.linalg.norm((g - f).ravel()) / np.linalg.norm((f - W).ravel()))
    MEASURED.append(dict(test="faces_vs_oracle", case=case, storage=storage, component="dev_rel_l2", measured=e,
                         target=bound, bound=bound))
    assert e <= bound, e
    faces.close()
    lat.close()


def test_faces_reject_unsupported_lattices():
    E = lib()
    lat16 = E.Lattice(E.make_params((8, 8), T=1 / 3, omega=1.2, storage="f16", u_adv=(0.05, 0.0)))
    with pytest.raises(E.ElbmError) as ei:  # faces need the rest reference
        E.Faces(lat16, ["inlet", "outlet", "wall", "wall"])
    assert ei.value.status == E.EUNSUPPORTED
    latw = E.Lattice(E.make_params((8, 8), T=1 / 3, omega=1.2, walls=(False, True)))
    with pytest.raises(E.ElbmError) as ei:
        E.Faces(latw, ["periodic", "periodic", "wall", "wall"])
    assert ei.value.status == E.EINVAL
    lat = E.Lattice(E.make_params((8, 8), T=1 / 3, omega=1.2))
    with pytest.raises(E.ElbmError) as ei:  # a corner whose x face is a wall
        E.Faces(lat, ["wall", "outlet", "wall", "symmetry"])
    assert ei.value.status == E.EUNSUPPORTED
    with pytest.raises(E.ElbmError) as ei:  # periodic on one face of an axis only
        E.Faces(lat, ["periodic", "outlet", "wall", "wall"])
    assert ei.value.status == E.EINVAL
    for L in (lat16, latw, lat):
        L.close()
