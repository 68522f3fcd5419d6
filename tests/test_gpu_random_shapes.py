"""Seeded random boxes and launch shapes against the float64 oracle.

Twenty cases drawn from default_rng(2024).  Each case draws:

* a box: nx in 1..300, ny in 1..12, nz in 1..10;
* an operator: BGK, MRT, or BGK with the velocity shift;
* a launch shape: work-group size, nodes per thread, tile width (0 = default,
  whole rows, or a multiple of 64), rows per tile, z chunk and tile order.

Every drawn shape is valid (tile width at most nodes_per_thread x threads,
rows clamped so that the tile fits); each case must match the oracle's
populations after 6 steps within 1e-12 (float64), and any library error
fails the test.  Refusal of invalid shapes is tested on its own.  Together with
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
        cap = threads * npt
        widths = [0] + [w for w in [nx] + [w for w in (64, 128, 192, 256) if w < nx] if w <= cap]
        bx = int(rng.choice(widths))
        by = int(rng.integers(0, 6))
        if bx > 0:
            by = min(by, cap // bx)
        zc = int(rng.integers(0, nz + 1))
        remap = int(rng.integers(0, 2))
        out.append(((nx, ny, nz), op, dict(threads=threads, nodes_per_thread=npt, block_x=bx,
                                           block_y=by, z_chunk=zc, xcd_remap=remap)))
    return out


@pytest.mark.parametrize("case", range(20))
def test_random_box_and_launch_shape(case):
    (nx, ny, nz), op, tuning = _cases()[case]
    rng = np.random.default_rng(case)
    rho0 = 1.0 + 0.4 * rng.random((nz, ny, nx))
    coll = "mrt" if op == "mrt" else "bgk"
    forcing = "shift" if op == "shift" else "guo"
    print("case %d: box %dx%dx%d %s %s" % (case, nx, ny, nz, op, tuning), flush=True)
    g = gc.run_gpu(rho0, 6, collision=coll, forcing=forcing, tau=0.9, tuning=tuning)
    g["sim"].close()
    o = gc.run_oracle(rho0, 6, collision=coll, forcing=forcing, tau=0.9)
    assert float(np.abs(g["state"] - o["state"]).max()) < F64_TOL


@pytest.mark.parametrize("case", range(0, 20, 2))
def test_random_box_and_launch_shape_f32(case):
    """The same boxes and launch shapes in FP32 shifted storage: density
    within 2e-6 relative of the FP64 oracle after 6 steps (the FP32 storage
    rounding floor over a few steps)."""
    (nx, ny, nz), op, tuning = _cases()[case]
    rng = np.random.default_rng(case)
    rho0 = 1.0 + 0.4 * rng.random((nz, ny, nx))
    coll = "mrt" if op == "mrt" else "bgk"
    forcing = "shift" if op == "shift" else "guo"
    print("case %d f32: box %dx%dx%d %s %s" % (case, nx, ny, nz, op, tuning), flush=True)
    g = gc.run_gpu(rho0, 6, collision=coll, forcing=forcing, tau=0.9, tuning=tuning,
                   precision="f32", want_state=False)
    g["sim"].close()
    o = gc.run_oracle(rho0, 6, collision=coll, forcing=forcing, tau=0.9)
    rel = float((np.abs(g["rho"] - o["rho"]) / o["rho"]).max())
    print("case %d f32: max rel drho %.2e" % (case, rel), flush=True)
    assert rel < 2e-6


@pytest.mark.parametrize("tuning", [
    dict(threads=256, block_x=300),                    # wider than the work-group
    dict(threads=256, block_x=128, block_y=3),         # tile exceeds the work-group
    dict(threads=256, nodes_per_thread=2, block_x=32),  # split tile narrower than 64
    dict(threads=384),
    dict(nodes_per_thread=3),
])
def test_invalid_launch_shapes_are_refused(tuning):
    from paper_1905_09554_amd import lbsc
    rho0 = 1.0 + 0.4 * np.random.default_rng(1).random((4, 6, 300))
    prm = lbsc.make_params(300, 6, 4, collision="bgk", precision="f64", G=-5.0, tau=0.9)
    sim = lbsc.Simulation(rho0, prm, device="cuda:0")
    with pytest.raises(lbsc.LbscError) as e:
        sim.set_tuning(**tuning)
    assert e.value.code == lbsc.LBSC_EINVAL
    sim.step(1)  # the context still steps with its previous shape
    sim.close()


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
