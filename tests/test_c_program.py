"""The C ABI from a plain C program (tests/c/abi_step.c): it compiles
against the header as C99 and links to the library here; on the GPU it runs
a box through the C calls alone and must give the same mass and minimum
radius, bitwise, as the Python binding on the same input."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import lbm_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1905_09554_amd")
SRC = os.path.join(ROOT, "tests", "c", "abi_step.c")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(out_dir):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(PKG, "liblbsc.so")):
        pytest.skip("liblbsc.so not built")
    exe = os.path.join(str(out_dir), "abi_step")
    subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
                    "-L", PKG, "-llbsc", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm",
                    "-o", exe], check=True)
    return exe


def test_c_program_compiles_and_links(tmp_path):
    assert os.access(_build(tmp_path), os.X_OK)


@pytest.mark.gpu
def test_c_program_matches_the_binding_bitwise(tmp_path):
    from paper_1905_09554_amd import lbsc
    exe = _build(tmp_path)
    nx, ny, nz, steps = 32, 32, 64, 200
    rv, rl = lbm_inputs.coexistence(-5.0)
    rho0 = lbm_inputs.ligament_density(nx, ny, nz, 8.0, 0.1, 1, rv, rl)
    path = tmp_path / "rho0.bin"
    np.ascontiguousarray(rho0, dtype=np.float64).tofile(str(path))
    print("C program: %dx%dx%d BGK f64, %d steps" % (nx, ny, nz, steps), flush=True)
    res = subprocess.run([exe, str(path), str(nx), str(ny), str(nz), str(steps), repr(rv), repr(rl)],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    got = dict(line.split() for line in res.stdout.strip().split("\n"))
    sim = lbsc.Simulation(rho0, lbsc.make_params(nx, ny, nz, G=-5.0, tau=1.0))
    d0 = sim.diagnostics(rv, rl)
    sim.step(steps)
    d1 = sim.diagnostics(rv, rl)
    sim.close()
    assert int(got["steps"]) == steps
    assert float(got["mass0"]) == d0["mass"] and float(got["mass1"]) == d1["mass"]
    assert float(got["r_min0"]) == d0["r_min"] and float(got["r_min1"]) == d1["r_min"]
