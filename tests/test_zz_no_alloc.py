"""lbsc_interface_diagnostics_static (reduction scratch in the library's
static device array) against lbsc_interface_diagnostics (scratch in the
context's buffer), through the C ABI: two calls in a row on different
contexts, the second on a smaller box, so that what the first call left in the
shared array must not leak into the second.  The two entry points run the same
kernels in the same order, so every output must be equal bitwise."""
import ctypes

import numpy as np
import pytest

from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu


def _both(sim, rv, rl):
    from paper_1905_09554_amd import lbsc
    lib = lbsc.library()
    out = {}
    for name in ("lbsc_interface_diagnostics", "lbsc_interface_diagnostics_static"):
        d = lbsc.Diag()
        r = np.full(sim.params.nz, np.nan)
        rc = getattr(lib, name)(sim._ctx, rv, rl, ctypes.byref(d),
                                r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        assert rc == lbsc.LBSC_OK, (name, rc, lib.lbsc_last_error(sim._ctx))
        out[name] = (d.mass, tuple(d.mom), d.r_min, d.z_argmin, r)
    return out["lbsc_interface_diagnostics"], out["lbsc_interface_diagnostics_static"]


def _same(a, b):
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2] and a[3] == b[3]
    assert np.array_equal(a[4], b[4])


def test_static_scratch_diagnostics_match_two_calls_second_smaller():
    from paper_1905_09554_amd import lbsc
    rv, rl = 0.119351, 1.888275
    big = gc.ligament(96, 80, 160, 20.0, 0.1, 1, noise=1e-4, seed=3)
    small = gc.ligament(20, 18, 24, 5.0, 0.1, 1)
    sims = []
    for rho0, prec in ((big, "f32"), (small, "f64")):
        nz, ny, nx = rho0.shape
        prm = lbsc.make_params(nx, ny, nz, collision="mrt", precision=prec, G=-5.0, tau=0.9)
        sim = lbsc.Simulation(rho0, prm, device="cuda:0")
        sim.step(37)
        sims.append(sim)
    print("static-scratch diagnostics: 96x80x160 f32, then 20x18x24 f64", flush=True)
    # Static entry point first on the large box, then on the small one; the
    # buffer-scratch entry point on each for comparison.
    lib = lbsc.library()
    for sim in sims:
        ref, sta = _both(sim, rv, rl)
        _same(ref, sta)
        assert np.isfinite(sta[4]).all() and sta[2] > 0
    # And the reverse order on the large box again after the small one.
    ref, sta = _both(sims[0], rv, rl)
    _same(ref, sta)
    d = lbsc.Diag()
    rc = lib.lbsc_interface_diagnostics_static(sims[1]._ctx, rv, rl, ctypes.byref(d), None)
    assert rc == lbsc.LBSC_OK
    for sim in sims:
        sim.close()


def test_static_scratch_refuses_a_box_beyond_its_limit():
    from paper_1905_09554_amd import lbsc
    # nz * ceil(nx ny / 4096) * 8 + 4 + nz doubles > 2^21 for a 1 x 1 x 240000 box.
    nz = 240000
    rho0 = np.full((nz, 1, 1), 1.0)
    prm = lbsc.make_params(1, 1, nz, collision="bgk", precision="f32", G=-5.0, tau=1.0)
    sim = lbsc.Simulation(rho0, prm, device="cuda:0")
    lib = lbsc.library()
    d = lbsc.Diag()
    rc = lib.lbsc_interface_diagnostics_static(sim._ctx, 0.1, 1.9, ctypes.byref(d), None)
    assert rc == lbsc.LBSC_EINVAL
    assert b"static scratch" in lib.lbsc_last_error(sim._ctx)
    # The buffer-scratch entry point still serves that box.
    rc = lib.lbsc_interface_diagnostics(sim._ctx, 0.1, 1.9, ctypes.byref(d), None)
    assert rc == lbsc.LBSC_OK and abs(d.mass - nz) < 1e-6 * nz
    sim.close()
