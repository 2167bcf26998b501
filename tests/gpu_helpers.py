"""Helpers shared by the GPU tests: build a lattice through the C ABI from the
same seeded inputs the oracle gets, and compare the two."""
import numpy as np

import inputs as I
import oracle as O


def lib():
    from paper_2101_04550_amd import elbm as E

    return E


def params_for(p: "O.Params", storage="f32", u_adv=None, diag_every=0, diag_capacity=0, mode_k=None,
               mode_dir=None):
    E = lib()
    return E.make_params(p.n, lam=p.lam, T=p.T, omega=p.omega, u_adv=u_adv, force=p.force, walls=p.walls,
                         storage=storage, extended=p.extended, diag_every=diag_every,
                         diag_capacity=diag_capacity, mode_k=mode_k, mode_dir=mode_dir)


def lattice_from_field(p, fld, storage="f32", u_adv=None, **kw):
    """GPU lattice initialised with f^eq(rho, u + u_adv); the oracle gets the same."""
    E = lib()
    lat = E.Lattice(params_for(p, storage, u_adv=u_adv, mode_k=fld.mode_k, mode_dir=fld.mode_dir, **kw))
    lat.init(fld.rho, fld.u)
    return lat


def oracle_init(p, fld, u_adv=None):
    return O.init_state(fld.rho, fld.u, p, u_adv=u_adv)


def random_state(p, seed, amp=0.03, noise=0.01):
    """Seeded non-equilibrium populations: equilibrium of a random smooth-ish
    field times (1 + noise), so every term of the collision is exercised."""
    g = I.rng(1000 + seed)
    grid = tuple(reversed(p.n))
    rho = 1.0 + 0.02 * g.standard_normal(grid)
    u = amp * g.standard_normal((p.D,) + grid)
    f = O.equilibrium(rho, u, p.T, p.lam, p.c)
    return f * (1.0 + noise * g.standard_normal(f.shape))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev_rel_l2(fg, fo, p, u_ref=None):
    """rel-L2 of population deviations from the reference weights."""
    w = O.reference_weights(p, u_ref).reshape((-1,) + (1,) * p.D)
    return rel_l2(fg - w, fo - w)


# ---- parity bounds from the storage floors, and a record of what was measured ----

_FLOORS = None
MEASURED = []  # dicts written to $ELBM_PARITY_JSON at the end of the session (tests/conftest.py)
FLOOR_MARGIN = 1.5


def floors():
    global _FLOORS
    if _FLOORS is None:
        import os
        import sys

        sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
        import make_storage_floors as MSF

        _FLOORS = MSF.load()
    return _FLOORS


def bound(case, storage, comp, gate):
    """Parity bound of one velocity component: the target `gate` where the
    storage floor (tests/golden/storage_floors.txt) lies at least a factor
    FLOOR_MARGIN below it, otherwise FLOOR_MARGIN times the floor (the format
    alone then misses the target; the bound says how close to the floor the
    kernel stays)."""
    fl = floors()[(case, storage, f"u{comp}")]
    return gate if FLOOR_MARGIN * fl <= gate else FLOOR_MARGIN * fl


def check_fields(test, case, storage, u, uo, gates):
    """Asserts rel-L2(u_a) within bound(case, storage, a, gates[a]) for every
    component and records measured value, floor, target and bound."""
    errs = []
    for a in range(len(gates)):
        e = rel_l2(u[a], uo[a])
        b = bound(case, storage, a, gates[a])
        MEASURED.append(dict(test=test, case=case, storage=storage, component=f"u{a}", measured=e,
                             floor=floors()[(case, storage, f"u{a}")], target=gates[a], bound=b))
        errs.append((a, e, b))
    for a, e, b in errs:
        assert e <= b, (test, case, storage, a, e, b)
