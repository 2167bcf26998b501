"""The boundary from C: include/elbm.h compiles as strict C99 and as C++17,
and a C client linked against the built library gets the same validation,
footprint and error reporting as the Python binding (host-only calls)."""
import os
import shutil
import subprocess

import pytest

from paper_2101_04550_amd import elbm as E

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c", "abi_client.c")


def _build_and_run(tmp_path, compiler, flags):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} is not installed")
    exe = str(tmp_path / f"abi_client_{compiler.replace('+', 'p')}")
    libdir = os.path.dirname(E.LIB_PATH)
    cmd = [compiler, *flags, "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"), SRC,
           "-o", exe, "-L", libdir, "-l:libelbm.so", f"-Wl,-rpath,{libdir}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return dict(line.split(" ", 1) for line in out.strip().splitlines())


@pytest.mark.parametrize("compiler,flags", [("gcc", ["-std=c99"]), ("g++", ["-std=c++17", "-x", "c++"])])
def test_c_client(tmp_path, compiler, flags):
    r = _build_and_run(tmp_path, compiler, flags)
    assert r["d3q27_f16_validate"] == "0"
    want = E.query_bytes(E.make_params((64, 32, 16), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.8, storage="f16"))
    assert r["d3q27_f16_bytes"] == f"0 {want}"
    want = E.query_bytes(E.make_params((96, 40), lam=(2.0, 1.0), T=0.5, omega=1.8, walls=(False, True),
                                       force=(1e-5, 0.0), omega_bulk=1.2, omega_ghost=1.0))
    assert r["d2q9_mrt_bytes"] == f"0 {want}"
    status, name = r["bad_omega"].split(" ", 1)
    assert int(status) == E.EINVAL and name == "ELBM_EINVAL"
    assert "omega" in r["bad_omega_message"]
    assert int(r["bad_abi"]) == E.EINVAL
    assert int(r["static_max"]) == 256
