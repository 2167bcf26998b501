"""The ABI from a plain C program on the GPU: tests/c/abi_run.c (built by
__graft_entry__.build() into paper_2101_04550_amd/_build/abi_run) allocates
the device buffer with the HIP runtime's C API, runs 50 steps of a D3Q27
channel-like lattice (lambda = (2, 1, 1), walls in y, force) and prints the
FP64 diagnostics record. The same problem through the Python binding gives
the same record bit for bit: same library, same kernels, same exact inputs."""
import os
import subprocess

import numpy as np
import pytest

from gpu_helpers import lib

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(os.path.dirname(HERE), "paper_2101_04550_amd", "_build", "abi_run")
NX, NY, NZ = 64, 32, 16


def _python_record(storage, mrt):
    E = lib()
    kw = dict(omega_bulk=1.2, omega_ghost=1.0) if mrt else {}
    p = E.make_params((NX, NY, NZ), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.7, walls=(False, True, False),
                      force=(1e-5, 0.0, 0.0), storage=storage, mode_k=(6.283185307179586 / (NX * 2.0), 0.0, 0.0),
                      mode_dir=(0.0, 0.0, 1.0), **kw)
    z, y, x = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    rho = 1.0 + ((y % 4).astype(np.float64) - 1.5) / 1024.0
    u = np.zeros((3, NZ, NY, NX))
    u[0] = 0.02
    u[2] = ((x % 8).astype(np.float64) - 3.5) / 400.0
    lat = E.Lattice(p)
    lat.init(rho, u)
    lat.step(50)
    d = lat.diag()
    k = lat.kernel_info()
    lat.close()
    return d, k


@pytest.mark.parametrize("storage,mrt", [("f32", 0), ("f16", 0), ("f32", 1), ("bf16", 1)])
def test_c_client_equals_python_binding(storage, mrt):
    if not os.path.exists(EXE):
        raise FileNotFoundError(f"{EXE} is missing: run __graft_entry__.build()")
    st = {"f32": 0, "f16": 1, "bf16": 2}[storage]
    out = subprocess.run([EXE, str(st), str(mrt)], check=True, capture_output=True, text=True, timeout=120).stdout
    r = {line.split()[0]: line.split()[1:] for line in out.strip().splitlines()}
    d, k = _python_record(storage, mrt)
    assert int(r["step"][0]) == d["step"] == 50
    assert float(r["mass"][0]) == d["mass"]
    assert [float(v) for v in r["mom"]] == list(d["mom"])
    assert float(r["ke"][0]) == d["ke"]
    assert float(r["enstrophy"][0]) == d["enstrophy"]
    assert [float(v) for v in r["mode"]] == [d["mode"].real, d["mode"].imag]
    assert float(r["min_rho"][0]) == d["min_rho"]
    assert int(r["nan_count"][0]) == d["nan_count"] == 0
    assert int(r["kernel"][1]) == k["block_threads"]
