"""Python binding of the libelbm C ABI (include/elbm.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels. PyTorch provides
device memory (a uint8 CUDA/HIP tensor per lattice) and the stream. If the
library has not been built, importing this module raises ImportError; no
CPU fallback exists.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

# torch must be loaded first: it brings the HIP runtime its tensors and streams
# belong to, and libelbm must bind to that same runtime instance (a second
# libamdhip64 in the process would not see the device).
import torch  # noqa: F401

_PKG = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_PKG)
LIB_PATH = os.path.join(_PKG, "libelbm.so")
HEADER = os.path.join(_ROOT, "include", "elbm.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_04550_amd.build`")

_lib = C.CDLL(LIB_PATH)

ABI_VERSION = 2
OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, EUNSTABLE = range(6)
BC_PERIODIC, BC_BOUNCEBACK = 0, 1
COLLISION_BGK, COLLISION_MRT = 0, 1
STORE_F32, STORE_F16, STORE_BF16 = 0, 1, 2
STORAGE_NAMES = {"f32": STORE_F32, "f16": STORE_F16, "bf16": STORE_BF16}


class ElbmParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("lattice", C.c_int32),
        ("n", C.c_int64 * 3),
        ("lambda_", C.c_double * 3),
        ("T", C.c_double),
        ("omega", C.c_double),
        ("u_adv", C.c_double * 3),
        ("force", C.c_double * 3),
        ("bc", C.c_int32 * 3),
        ("storage", C.c_int32),
        ("extended", C.c_int32),
        ("diag_every", C.c_int32),
        ("diag_capacity", C.c_int32),
        ("collision", C.c_int32),
        ("mode_k", C.c_double * 3),
        ("mode_dir", C.c_double * 3),
        ("omega_bulk", C.c_double),
        ("omega_ghost", C.c_double),
    ]


class ElbmKernelInfo(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32),
        ("block_threads", C.c_int32),
        ("tile", C.c_int32 * 3),
        ("blocks_per_cu", C.c_int32),
        ("tiles", C.c_int64),
    ]


class ElbmDiag(C.Structure):
    _fields_ = [
        ("step", C.c_int64),
        ("mass", C.c_double),
        ("mom", C.c_double * 3),
        ("ke", C.c_double),
        ("enstrophy", C.c_double),
        ("mode_re", C.c_double),
        ("mode_im", C.c_double),
        ("max_uperp", C.c_double),
        ("min_rho", C.c_double),
        ("nan_count", C.c_int64),
    ]

    def as_dict(self):
        return {
            "step": int(self.step), "mass": self.mass, "mom": tuple(self.mom), "ke": self.ke,
            "enstrophy": self.enstrophy, "mode": complex(self.mode_re, self.mode_im),
            "max_uperp": self.max_uperp, "min_rho": self.min_rho, "nan_count": int(self.nan_count),
        }


FACE_PERIODIC, FACE_SYMMETRY, FACE_WALL, FACE_INLET, FACE_OUTLET = range(5)
FACE_NAMES = {"periodic": FACE_PERIODIC, "symmetry": FACE_SYMMETRY, "wall": FACE_WALL, "inlet": FACE_INLET,
              "outlet": FACE_OUTLET}


class ElbmFacesParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("kind", C.c_int32 * 4),
        ("node_kind", C.POINTER(C.c_int8) * 4),
        ("wall_velocity", C.c_double * 4),
        ("inlet_velocity", (C.c_double * 2) * 4),
        ("outlet_density", C.c_double * 4),
    ]


_P = C.POINTER
_sigs = {
    "elbm_abi_version": (C.c_uint32, []),
    "elbm_status_string": (C.c_char_p, [C.c_int32]),
    "elbm_last_error": (C.c_char_p, []),
    "elbm_validate": (C.c_int32, [_P(ElbmParams)]),
    "elbm_query_bytes": (C.c_int32, [_P(ElbmParams), _P(C.c_size_t)]),
    "elbm_create": (C.c_int32, [_P(ElbmParams), C.c_void_p, C.c_size_t, C.c_void_p, _P(C.c_void_p)]),
    "elbm_init": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "elbm_step": (C.c_int32, [C.c_void_p, C.c_int64]),
    "elbm_step_count": (C.c_int64, [C.c_void_p]),
    "elbm_kernel": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "elbm_fields": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "elbm_populations": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "elbm_set_populations": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "elbm_diag": (C.c_int32, [C.c_void_p, _P(ElbmDiag)]),
    "elbm_diag_history": (C.c_int32, [C.c_void_p, _P(ElbmDiag), C.c_int32, _P(C.c_int32)]),
    "elbm_checkpoint_bytes": (C.c_int32, [C.c_void_p, _P(C.c_size_t)]),
    "elbm_save": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "elbm_load": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "elbm_sync": (C.c_int32, [C.c_void_p]),
    "elbm_destroy": (C.c_int32, [C.c_void_p]),
    "elbm_batch_create": (C.c_int32, [C.c_int32, C.c_void_p, _P(C.c_void_p)]),
    "elbm_batch_run": (C.c_int32, [C.c_void_p, _P(C.c_void_p), _P(C.c_int64), C.c_int32, C.c_int32]),
    "elbm_batch_destroy": (C.c_int32, [C.c_void_p]),
    "elbm_batch_run_static": (C.c_int32, [_P(C.c_void_p), _P(C.c_int64), C.c_int32, C.c_void_p]),
    "elbm_faces_query_bytes": (C.c_int32, [C.c_void_p, _P(ElbmFacesParams), _P(C.c_size_t)]),
    "elbm_faces_create": (C.c_int32, [C.c_void_p, _P(ElbmFacesParams), C.c_void_p, C.c_size_t, _P(C.c_void_p)]),
    "elbm_faces_step": (C.c_int32, [C.c_void_p, C.c_int64]),
    "elbm_faces_destroy": (C.c_int32, [C.c_void_p]),
}
STATIC_MAX_LATTICES = 256
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def header_functions(path: str = HEADER):
    """Names of all functions declared in include/elbm.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(elbm_[a-z0-9_]+)\s*\(", txt)))


def exported_symbols():
    return {name for name in header_functions() if hasattr(_lib, name)}


class ElbmError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.elbm_last_error().decode()
        name = _lib.elbm_status_string(status).decode()
        super().__init__(f"{where}: {name}: {msg}")


def _check(status, where):
    if status != OK:
        raise ElbmError(status, where)


def make_params(n, lam=None, T=1.0 / 3.0, omega=1.0, u_adv=None, force=None, walls=None,
                storage="f32", extended=True, diag_every=0, diag_capacity=0, mode_k=None, mode_dir=None,
                omega_bulk=None, omega_ghost=None):
    """elbm_params from Python values. ``n`` has 2 (D2Q9) or 3 (D3Q27) extents.
    Giving omega_bulk or omega_ghost selects the multi-relaxation-time
    collision (the other rate defaults to omega)."""
    D = len(n)
    if D not in (2, 3):
        raise ValueError("n must have 2 or 3 extents")
    p = ElbmParams()
    p.abi_version = ABI_VERSION
    p.lattice = 9 if D == 2 else 27
    nn = list(n) + [1] * (3 - D)
    lam = list(lam) if lam is not None else [1.0] * D
    for a in range(3):
        p.n[a] = int(nn[a])
        p.lambda_[a] = float(lam[a]) if a < D else 1.0
        p.u_adv[a] = float(u_adv[a]) if (u_adv is not None and a < D) else 0.0
        p.force[a] = float(force[a]) if (force is not None and a < D) else 0.0
        p.bc[a] = (BC_BOUNCEBACK if walls[a] else BC_PERIODIC) if (walls is not None and a < D) else BC_PERIODIC
        p.mode_k[a] = float(mode_k[a]) if (mode_k is not None and a < len(mode_k)) else 0.0
        p.mode_dir[a] = float(mode_dir[a]) if (mode_dir is not None and a < len(mode_dir)) else 0.0
    p.T = float(T)
    p.omega = float(omega)
    p.storage = STORAGE_NAMES[storage] if isinstance(storage, str) else int(storage)
    p.extended = 1 if extended else 0
    p.diag_every = int(diag_every)
    p.diag_capacity = int(diag_capacity)
    mrt = omega_bulk is not None or omega_ghost is not None
    p.collision = COLLISION_MRT if mrt else COLLISION_BGK
    p.omega_bulk = float(omega_bulk) if omega_bulk is not None else float(omega)
    p.omega_ghost = float(omega_ghost) if omega_ghost is not None else float(omega)
    return p


def validate(params: ElbmParams) -> int:
    return _lib.elbm_validate(C.byref(params))


def query_bytes(params: ElbmParams) -> int:
    out = C.c_size_t(0)
    _check(_lib.elbm_query_bytes(C.byref(params), C.byref(out)), "elbm_query_bytes")
    return int(out.value)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Lattice:
    """One lattice resident in device memory owned by a torch uint8 tensor."""

    def __init__(self, params: ElbmParams, device=None, stream=None, buffer=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.params = params
        self.D = 3 if params.lattice == 27 else 2
        self.Q = params.lattice
        self.n = tuple(int(params.n[a]) for a in range(self.D))
        self.N = int(np.prod(self.n))
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.nbytes = query_bytes(params)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if buffer is None:
                # allocated for the lattice's stream (torch's allocator ties
                # a block to the stream it is allocated on)
                with torch.cuda.stream(self.stream):
                    buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.buffer = buffer
            h = C.c_void_p()
            _check(_lib.elbm_create(C.byref(params), C.c_void_p(buffer.data_ptr()), buffer.numel(),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)), "elbm_create")
        self.handle = h

    # grid shape of host arrays: (n_y, n_x) or (n_z, n_y, n_x)
    @property
    def grid(self):
        return tuple(reversed(self.n))

    def init(self, rho, u):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        if rho.size != self.N or u.size != self.D * self.N:
            raise ValueError("rho / u sizes do not match the lattice")
        _check(_lib.elbm_init(self.handle, _dptr(rho), _dptr(u)), "elbm_init")
        return self

    def step(self, nsteps=1):
        _check(_lib.elbm_step(self.handle, int(nsteps)), "elbm_step")
        return self

    @property
    def step_count(self):
        return int(_lib.elbm_step_count(self.handle))

    def kernel_info(self):
        """The step kernel and launch shape chosen for this lattice."""
        k = ElbmKernelInfo()
        _check(_lib.elbm_kernel(self.handle, C.byref(k)), "elbm_kernel")
        return {"kernel": "staged" if k.kernel == 1 else "register", "block_threads": k.block_threads,
                "tile": tuple(k.tile), "blocks_per_cu": k.blocks_per_cu, "tiles": k.tiles}

    def fields(self):
        rho = np.empty(self.N)
        u = np.empty(self.D * self.N)
        _check(_lib.elbm_fields(self.handle, _dptr(rho), _dptr(u)), "elbm_fields")
        return rho.reshape(self.grid), u.reshape((self.D,) + self.grid)

    def populations(self):
        f = np.empty(self.Q * self.N)
        _check(_lib.elbm_populations(self.handle, _dptr(f)), "elbm_populations")
        return f.reshape((self.Q,) + self.grid)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if f.size != self.Q * self.N:
            raise ValueError("population array size does not match the lattice")
        _check(_lib.elbm_set_populations(self.handle, _dptr(f)), "elbm_set_populations")
        return self

    def diag(self, check=True):
        d = ElbmDiag()
        s = _lib.elbm_diag(self.handle, C.byref(d))
        if check:
            _check(s, "elbm_diag")
        return d.as_dict()

    def diag_history(self, max_records=1 << 20):
        cap = min(int(max_records), max(1, int(self.params.diag_capacity)))
        arr = (ElbmDiag * cap)()
        cnt = C.c_int32(0)
        _check(_lib.elbm_diag_history(self.handle, arr, cap, C.byref(cnt)), "elbm_diag_history")
        return [arr[k].as_dict() for k in range(cnt.value)]

    def checkpoint_bytes(self):
        out = C.c_size_t(0)
        _check(_lib.elbm_checkpoint_bytes(self.handle, C.byref(out)), "elbm_checkpoint_bytes")
        return int(out.value)

    def save(self) -> np.ndarray:
        buf = np.empty(self.checkpoint_bytes(), dtype=np.uint8)
        _check(_lib.elbm_save(self.handle, _dptr(buf), buf.size), "elbm_save")
        return buf

    def load(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(_lib.elbm_load(self.handle, _dptr(buf), buf.size), "elbm_load")
        return self

    def sync(self):
        _check(_lib.elbm_sync(self.handle), "elbm_sync")

    def close(self):
        if getattr(self, "handle", None):
            _check(_lib.elbm_destroy(self.handle), "elbm_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _face_kind(k):
    return FACE_NAMES[k] if isinstance(k, str) else int(k)


class Faces:
    """Open boundaries (elbm_faces_*) of a D2Q9 lattice that carries a
    ghost ring on each non-periodic axis (its extents are the fluid extents
    plus 2 there), or Grad walls on the y faces of a D3Q27 channel (any
    storage format)
    (kinds ["periodic", "periodic", "wall", "wall"], n_y = fluid rows + 2;
    wall_velocity[2], [3]: the walls' x-velocities).

    kinds: four entries (x-, x+, y-, y+), each a kind for the whole face or a
    sequence with one kind per fluid node along it; wall_velocity: four
    tangential wall velocities; inlet_velocity: four (u_x, u_y);
    outlet_density: four outlet densities."""

    def __init__(self, lattice: "Lattice", kinds, wall_velocity=(0.0, 0.0, 0.0, 0.0),
                 inlet_velocity=((0.0, 0.0),) * 4, outlet_density=(1.0, 1.0, 1.0, 1.0)):
        import torch

        self.lattice = lattice
        fp = ElbmFacesParams()
        fp.abi_version = ABI_VERSION
        self._arrays = []
        for F in range(4):
            k = kinds[F]
            if isinstance(k, (str, int, np.integer)):
                fp.kind[F] = _face_kind(k)
            else:
                arr = np.ascontiguousarray([_face_kind(v) for v in k], dtype=np.int8)
                self._arrays.append(arr)
                fp.kind[F] = int(arr[0])
                fp.node_kind[F] = arr.ctypes.data_as(C.POINTER(C.c_int8))
            fp.wall_velocity[F] = float(wall_velocity[F])
            fp.inlet_velocity[F][0] = float(inlet_velocity[F][0])
            fp.inlet_velocity[F][1] = float(inlet_velocity[F][1])
            fp.outlet_density[F] = float(outlet_density[F])
        self.params = fp
        nb = C.c_size_t(0)
        _check(_lib.elbm_faces_query_bytes(lattice.handle, C.byref(fp), C.byref(nb)), "elbm_faces_query_bytes")
        with torch.cuda.device(lattice.device), torch.cuda.stream(lattice.stream):
            self.buffer = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=lattice.device)
        h = C.c_void_p()
        _check(_lib.elbm_faces_create(lattice.handle, C.byref(fp), C.c_void_p(self.buffer.data_ptr()),
                                      self.buffer.numel(), C.byref(h)), "elbm_faces_create")
        self.handle = h

    def step(self, nsteps=1):
        _check(_lib.elbm_faces_step(self.handle, int(nsteps)), "elbm_faces_step")
        return self

    def close(self):
        if getattr(self, "handle", None):
            _check(_lib.elbm_faces_destroy(self.handle), "elbm_faces_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Fused multi-lattice launches (elbm_batch_*), optionally replayed from HIP graphs."""

    def __init__(self, capacity, stream=None):
        import torch

        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(_lib.elbm_batch_create(int(capacity), C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "elbm_batch_create")
        self.handle = h
        self.capacity = int(capacity)

    def run(self, lattices, steps, use_graph=True):
        count = len(lattices)
        hs = (C.c_void_p * max(count, 1))(*[lat.handle for lat in lattices])
        st = (C.c_int64 * max(count, 1))(*[int(s) for s in steps])
        _check(_lib.elbm_batch_run(self.handle, hs, st, count, 1 if use_graph else 0), "elbm_batch_run")

    def close(self):
        if getattr(self, "handle", None):
            _check(_lib.elbm_batch_destroy(self.handle), "elbm_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run_static(lattices, steps, stream=None):
    """elbm_batch_run_static: the batched run with the library's fixed device
    tables (no allocation); `stream` defaults to torch's current stream."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream()
    count = len(lattices)
    hs = (C.c_void_p * max(count, 1))(*[lat.handle for lat in lattices])
    ks = (C.c_int64 * max(count, 1))(*[int(k) for k in steps])
    _check(_lib.elbm_batch_run_static(hs, ks, count, C.c_void_p(st.cuda_stream)), "elbm_batch_run_static")
