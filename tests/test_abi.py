"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid input before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1905_09554_amd import lbsc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbsc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbsc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbsc.library()
    names = _declared_functions()
    assert "lbsc_init_fields" in names and "lbsc_step" in names
    for name in names:
        assert hasattr(lib, name), name


def test_lattice_table_matches_d3q19():
    c, w = lbsc.lattice()
    assert len({tuple(v) for v in c.tolist()}) == 19
    assert abs(w.sum() - 1.0) < 1e-15
    for v, wv in zip(c.tolist(), w.tolist()):
        n = sum(abs(k) for k in v)
        assert wv == {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[n]


def _params(**kw):
    base = dict(nx=8, ny=8, nz=8)
    base.update(kw)
    return lbsc.make_params(**base)


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(nx=2048, ny=1024, nz=1024), dict(tau=0.5), dict(tau=float("nan")),
    dict(G=float("inf")), dict(psi_rho0=0.0), dict(collision="mrt", s_ghost=2.0),
    dict(collision="mrt", s_bulk=0.0), dict(collision="mrt", forcing="shift"),
])
def test_invalid_params_have_no_state_size(bad):
    assert lbsc.state_bytes(_params(**bad)) == 0


def test_state_size_counts_two_lattices():
    for prec, size in (("f64", 8), ("f32", 4)):
        p = _params(nx=10, ny=6, nz=5, precision=prec)
        n = 10 * 6 * 5
        # two lattices and the psi field of the two-kernel step form
        assert lbsc.state_bytes(p) >= (2 * 19 + 1) * n * size
        # plus room for up to 65536 padding elements between population arrays
        assert lbsc.state_bytes(p) < 2 * 19 * (n + 64 + 65536) * size + n * size + 64 * 1024
    # nx beyond one work-group: tiles split rows (no nx limit of its own)
    assert lbsc.state_bytes(_params(nx=4096, ny=2, nz=2)) > 0


def _init(params, rho0, buf=0x10000000, nbytes=None):
    lib = lbsc.library()
    ctx = ctypes.c_void_p()
    if nbytes is None:
        nbytes = lbsc.state_bytes(params)
    rc = lib.lbsc_init_fields(ctypes.byref(ctx), ctypes.byref(params),
                              rho0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              ctypes.c_void_p(buf), nbytes, None)
    return rc, ctx, lib.lbsc_last_error(None).decode()


def test_init_rejects_bad_density_before_any_device_work():
    p = _params()
    rho = np.ones((8, 8, 8))
    rho[3, 2, 1] = float("nan")
    rc, ctx, msg = _init(p, rho)
    assert rc == lbsc.LBSC_EINVAL and not ctx.value and "rho0" in msg
    rho[3, 2, 1] = -0.1
    rc, _, msg = _init(p, rho)
    assert rc == lbsc.LBSC_EINVAL and "index %d" % (3 * 64 + 2 * 8 + 1) in msg


def test_init_rejects_small_or_misaligned_buffer():
    p = _params()
    rho = np.ones((8, 8, 8))
    rc, _, msg = _init(p, rho, nbytes=lbsc.state_bytes(p) - 1)
    assert rc == lbsc.LBSC_EINVAL and "dev_bytes" in msg
    rc, _, msg = _init(p, rho, buf=0x10000008)
    assert rc == lbsc.LBSC_EINVAL and "aligned" in msg
    rc, _, msg = _init(p, rho, buf=0)
    assert rc == lbsc.LBSC_EINVAL


def test_invalid_params_rejected_by_init():
    p = _params(tau=0.4)
    rc, _, msg = _init(p, np.ones((8, 8, 8)), nbytes=1 << 30)
    assert rc == lbsc.LBSC_EINVAL and "tau" in msg


def test_null_context_calls_are_safe():
    lib = lbsc.library()
    lib.lbsc_destroy(None)
    assert lib.lbsc_step(None, 1) == lbsc.LBSC_EINVAL
    assert lib.lbsc_step_count(None) == -1
    assert lib.lbsc_compute_moments(None, None, None, None) == lbsc.LBSC_EINVAL
    assert lib.lbsc_get_state(None, None, 0, None) == lbsc.LBSC_EINVAL


def test_simulation_requires_built_library_and_raises_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    with pytest.raises(Exception):
        lbsc.Simulation(np.ones((4, 4, 4)), _params(nx=4, ny=4, nz=4), device="cuda:0")


def test_binding_structs_match_the_header_layout(tmp_path):
    """sizeof and every field offset of lbsc_params, lbsc_diag and
    lbsc_tuning as a C compiler lays them out from the header, against the
    ctypes structures of the binding."""
    structs = {"lbsc_params": lbsc.Params, "lbsc_diag": lbsc.Diag, "lbsc_tuning": lbsc.Tuning}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbsc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    seen = {}
    for line in out.split("\n"):
        if line:
            cname, key, value = line.split()
            seen[(cname, key)] = int(value)
    for cname, py in structs.items():
        assert seen[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert seen[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
    # every field the header declares is in the binding
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct lbsc_tuning \{(.*?)\} lbsc_tuning;", text, flags=re.S).group(1)
    declared = re.findall(r"\b(\w+)\s*;", body)
    assert declared == [f for f, _ in lbsc.Tuning._fields_]


@pytest.mark.parametrize("box,coll,prec,expect", [
    # (threads, block_x, block_y, z_chunk, xcd_remap)
    ((256, 256, 1024), "mrt", "f32", (1024, 256, 4, 256, 1)),   # one wave of 256 groups
    ((256, 256, 1024), "mrt", "f64", (256, 64, 4, 64, 1)),      # eight waves, XCD-local ranges
    ((128, 128, 512), "bgk", "f64", (256, 64, 4, 64, 1)),       # one wave: XCD-local ranges
    ((64, 64, 256), "mrt", "f32", (1024, 64, 16, 4, 1)),
    ((32, 32, 64), "bgk", "f64", (256, 32, 8, 1, 1)),           # small box: one-plane chunks
    ((384, 384, 1024), "mrt", "f32", (512, 128, 4, 64, 1)),     # rows wider than 256 nodes
])
def test_default_launch_shapes(box, coll, prec, expect):
    """The library's default launch shape (host only) for the boxes whose
    measurements chose the policy."""
    nx, ny, nz = box
    t = lbsc.default_tuning(_params(nx=nx, ny=ny, nz=nz, collision=coll, precision=prec))
    got = (t["threads"], t["block_x"], t["block_y"], t["z_chunk"], t["xcd_remap"])
    assert got == expect
    assert t["block_x"] * t["block_y"] <= t["threads"] * t["nodes_per_thread"]
    assert t["persistent"] == 0 and t["two_kernel"] == 0


def test_default_tuning_rejects_invalid_parameters():
    with pytest.raises(lbsc.LbscError):
        lbsc.default_tuning(_params(tau=0.5))
