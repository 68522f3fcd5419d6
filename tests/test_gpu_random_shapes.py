"""Seeded random boxes and launch shapes against the float64 oracle.

Twenty cases drawn from default_rng(2024).  Each case draws:

* a box: nx in 1..300, ny in 1..12, nz in 1..10;
* an operator: BGK, MRT, or BGK with the velocity shift;
* a launch shape: work-group size, nodes per thread, tile width (0 = default,
  whole rows, or a multiple of 64), rows per tile, z chunk and tile order.

Shapes the library rejects are skipped case by case; the rest must match the
oracle's populations after 6 steps within 1e-12 (float64).  Together with
the fixed ragged-shape cases this covers the two-dimensional tiling, with
ragged last tiles in x, y and z, at sizes the oracle finishes in seconds.
"""
import numpy as np
import pytest

from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def _cases(n=20, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(1, 301))
        ny = int(rng.integers(1, 13))
        nz = int(rng.integers(1, 11))
        op = ["bgk", "mrt", "shift"][int(rng.integers(0, 3))]
        threads = int(rng.choice([256, 512, 1024]))
        npt = int(rng.choice([1, 2]))
        widths = [0, nx] + [w for w in (64, 128, 192, 256) if w < nx]
        bx = int(rng.choice(widths))
        by = int(rng.integers(0, 6))
        zc = int(rng.integers(0, nz + 1))
        remap = int(rng.integers(0, 2))
        out.append(((nx, ny, nz), op, dict(threads=threads, nodes_per_thread=npt, block_x=bx,
                                           block_y=by, z_chunk=zc, xcd_remap=remap)))
    return out


@pytest.mark.parametrize("case", range(20))
def test_random_box_and_launch_shape(case):
    from paper_1905_09554_amd import lbsc
    (nx, ny, nz), op, tuning = _cases()[case]
    rng = np.random.default_rng(case)
    rho0 = 1.0 + 0.4 * rng.random((nz, ny, nx))
    coll = "mrt" if op == "mrt" else "bgk"
    forcing = "shift" if op == "shift" else "guo"
    print("case %d: box %dx%dx%d %s %s" % (case, nx, ny, nz, op, tuning), flush=True)
    try:
        g = gc.run_gpu(rho0, 6, collision=coll, forcing=forcing, tau=0.9, tuning=tuning)
    except lbsc.LbscError as e:
        pytest.skip("launch shape rejected: %s" % e)
    g["sim"].close()
    o = gc.run_oracle(rho0, 6, collision=coll, forcing=forcing, tau=0.9)
    assert float(np.abs(g["state"] - o["state"]).max()) < F64_TOL


@pytest.mark.parametrize("case", range(0, 20, 2))
def test_random_box_and_launch_shape_f32(case):
    """The same boxes and launch shapes in FP32 shifted storage: density
    within 2e-6 relative of the FP64 oracle after 6 steps (the FP32 storage
    rounding floor over a few steps)."""
    from paper_1905_09554_amd import lbsc
    (nx, ny, nz), op, tuning = _cases()[case]
    rng = np.random.default_rng(case)
    rho0 = 1.0 + 0.4 * rng.random((nz, ny, nx))
    coll = "mrt" if op == "mrt" else "bgk"
    forcing = "shift" if op == "shift" else "guo"
    try:
        g = gc.run_gpu(rho0, 6, collision=coll, forcing=forcing, tau=0.9, tuning=tuning,
                       precision="f32", want_state=False)
    except lbsc.LbscError as e:
        pytest.skip("launch shape rejected: %s" % e)
    g["sim"].close()
    o = gc.run_oracle(rho0, 6, collision=coll, forcing=forcing, tau=0.9)
    rel = float((np.abs(g["rho"] - o["rho"]) / o["rho"]).max())
    print("case %d f32: max rel drho %.2e" % (case, rel), flush=True)
    assert rel < 2e-6


@pytest.mark.parametrize("case", range(6))
def test_random_box_two_kernel_form(case):
    """The two-kernel form of the step on seeded random boxes (including
    one-node-thick ones): float64 populations within 1e-12 of the oracle
    after 6 steps."""
    rng = np.random.default_rng(7000 + case)
    nx, ny, nz = (int(rng.integers(1, 200)), int(rng.integers(1, 10)), int(rng.integers(1, 9)))
    op = ["bgk", "mrt", "shift"][case % 3]
    coll = "mrt" if op == "mrt" else "bgk"
    forcing = "shift" if op == "shift" else "guo"
    rho0 = 1.0 + 0.4 * rng.random((nz, ny, nx))
    print("two-kernel case %d: box %dx%dx%d %s" % (case, nx, ny, nz, op), flush=True)
    g = gc.run_gpu(rho0, 6, collision=coll, forcing=forcing, tau=0.9,
                   tuning=dict(two_kernel=1))
    g["sim"].close()
    o = gc.run_oracle(rho0, 6, collision=coll, forcing=forcing, tau=0.9)
    assert float(np.abs(g["state"] - o["state"]).max()) < F64_TOL
