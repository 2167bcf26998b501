"""C-ABI host checks that need no GPU: the library loads, exports every symbol
include/elbm.h declares, validates parameters and computes the footprint."""
import math

import pytest

from paper_2101_04550_amd import elbm as E


def test_every_declared_symbol_is_exported():
    declared = E.header_functions()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(E._lib, n)]
    assert missing == []


def test_abi_version_and_status_strings():
    assert E._lib.elbm_abi_version() == E.ABI_VERSION
    names = [E._lib.elbm_status_string(s).decode() for s in range(6)]
    assert names == ["ELBM_OK", "ELBM_EINVAL", "ELBM_EUNSUPPORTED", "ELBM_ENOMEM", "ELBM_EDEVICE", "ELBM_EUNSTABLE"]
    assert E._lib.elbm_status_string(99).decode() == "ELBM_UNKNOWN"


@pytest.mark.parametrize("kw,msg", [
    (dict(omega=2.0), "omega"),
    (dict(omega=0.0), "omega"),
    (dict(T=0.0), "T must"),
    (dict(T=0.5, lam=(0.5, 1.0)), "rest weight"),   # Psi_0 = 1 - T/lam^2 < 0
    (dict(n=(2, 64)), "periodic axis"),
    (dict(n=(64, 1), walls=(False, True)), "bounce-back axis"),
    (dict(lam=(0.0, 1.0)), "lambda"),
    (dict(storage=7), "storage"),
    (dict(diag_every=5, diag_capacity=0), "diag_capacity"),
])
def test_validation_rejects(kw, msg):
    args = dict(n=(64, 64), T=1 / 3, omega=1.5)
    args.update(kw)
    p = E.make_params(**args)
    assert E.validate(p) == E.EINVAL
    assert msg in E._lib.elbm_last_error().decode()
    with pytest.raises(E.ElbmError):
        E.query_bytes(p)


@pytest.mark.parametrize("D", [2, 3])
def test_walls_with_advection_reference_are_unsupported(D):
    """A bounced population stored as a deviation from w(u_adv) would need the
    correction w_opp - w_i, which the kernels do not apply: walls need u_adv = 0."""
    n = (16, 16, 8)[:D]
    walls = (False, True, False)[:D]
    ok = E.make_params(n, T=0.5, omega=1.5, walls=walls)
    assert E.validate(ok) == E.OK
    bad = E.make_params(n, T=0.5, omega=1.5, walls=walls, u_adv=(0.05,) + (0.0,) * (D - 1))
    assert E.validate(bad) == E.EUNSUPPORTED
    assert "u_adv" in E._lib.elbm_last_error().decode()
    # periodic lattices keep the advected reference
    assert E.validate(E.make_params(n, T=0.5, omega=1.5, u_adv=(0.05,) + (0.0,) * (D - 1))) == E.OK


def test_mrt_collision_validation():
    """The multi-relaxation-time collision: D2Q9 and D3Q27, rates in (0, 2),
    and a collision code the library knows."""
    assert E.validate(E.make_params((32, 16), T=0.5, omega=1.6, omega_bulk=1.1, omega_ghost=1.3)) == E.OK
    assert E.validate(E.make_params((8, 8, 8), T=0.5, omega=1.6, omega_bulk=1.1)) == E.OK
    assert E.validate(E.make_params((8, 8, 8), T=0.5, omega=1.6, omega_ghost=2.0)) == E.EINVAL
    for ob, og in ((0.0, 1.0), (1.0, 2.0), (-0.5, 1.0), (1.0, float("nan"))):
        assert E.validate(E.make_params((32, 16), T=0.5, omega=1.6, omega_bulk=ob, omega_ghost=og)) == E.EINVAL
        assert "omega_bulk" in E._lib.elbm_last_error().decode()
    p = E.make_params((32, 16), T=0.5, omega=1.6)
    p.collision = 7
    assert E.validate(p) == E.EINVAL
    # the LBGK default leaves both extra rates unused
    p = E.make_params((32, 16), T=0.5, omega=1.6)
    assert p.collision == E.COLLISION_BGK
    p.omega_bulk = 5.0
    assert E.validate(p) == E.OK


def test_validation_rejects_bad_lattice_shapes():
    p = E.make_params((8, 8, 8), T=0.5, omega=1.0)
    p.lattice = 15
    assert E.validate(p) == E.EINVAL
    p = E.make_params((8, 8), T=0.5, omega=1.0)
    p.n[2] = 4
    assert E.validate(p) == E.EINVAL
    p = E.make_params((8, 8), T=0.5, omega=1.0)
    p.abi_version = 99
    assert E.validate(p) == E.EINVAL
    p = E.make_params((2048, 2048, 1024), T=0.5, omega=1.0)
    assert E.validate(p) == E.EINVAL  # more than 2^31 - 1 nodes


@pytest.mark.parametrize("n,storage,ok", [((6400, 6400, 3), "f32", False), ((6400, 6400, 3), "f16", True),
                                          ((1 << 27, 8), "f32", False), ((1 << 26, 8), "f16", True)])
def test_validation_bounds_one_plane_slab(n, storage, ok):
    # the Q direction arrays of one plane across the slowest axis must be
    # addressable with 32-bit byte offsets
    p = E.make_params(n, T=0.5, omega=1.0, storage=storage)
    if ok:
        assert E.validate(p) == E.OK
    else:
        assert E.validate(p) == E.EINVAL
        assert "per plane" in E._lib.elbm_last_error().decode()


@pytest.mark.parametrize("n,storage,es", [((64, 64), "f32", 4), ((256, 256, 256), "f32", 4),
                                          ((384, 192, 192), "f16", 2), ((100, 77), "bf16", 2)])
def test_footprint_covers_two_population_buffers(n, storage, es):
    p = E.make_params(n, T=1 / 3, omega=1.5, storage=storage)
    b = E.query_bytes(p)
    Q = 9 if len(n) == 2 else 27
    N = math.prod(n)
    pops = 2 * Q * N * es
    assert b >= pops
    # padding and fixed scratch (descriptor, two sets of 1024 partial records
    # of 16 doubles, one record) stay small
    assert b - pops < 2 * Q * 256 * es + 2 * 4096 + 256 * 1024 + 1024 * 16 * 8
    # sampled diagnostics add the history (capacity * 16 doubles), the staged
    # velocity of a sample step (3 N floats) and the mode factors (2 doubles
    # per node of each axis)
    p2 = E.make_params(n, T=1 / 3, omega=1.5, storage=storage, diag_every=10, diag_capacity=1000)
    extra = 1000 * 16 * 8 + 3 * N * 4 + 2 * sum(n) * 8
    assert extra <= E.query_bytes(p2) - b < extra + 4 * 256


def test_last_error_is_thread_local():
    import threading

    E.validate(E.make_params((64, 64), T=1 / 3, omega=3.0))
    seen = {}

    def other():
        seen["msg"] = E._lib.elbm_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == ""
    assert "omega" in E._lib.elbm_last_error().decode()


def test_probe_library_exports_its_header():
    """The bandwidth probe (libelbm_probe.so) exports every function its header
    declares, and sizes its buffers as the step's plane slabs (no GPU)."""
    import ctypes as C
    import os
    import re

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(root, "include", "elbm_probe.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(elbm_probe_[a-z0-9_]+)\s*\(", txt)))
    lib = C.CDLL(os.path.join(root, "paper_2101_04550_amd", "libelbm_probe.so"))
    assert names and all(hasattr(lib, n) for n in names)
    lib.elbm_probe_bytes.argtypes = [C.c_int32] * 4 + [C.POINTER(C.c_size_t)]
    nb = C.c_size_t(0)
    assert lib.elbm_probe_bytes(4, 256, 256, 256, C.byref(nb)) == 0
    assert nb.value == 256 * 27 * 65536 * 4
    assert lib.elbm_probe_bytes(3, 256, 256, 256, C.byref(nb)) == 1
