"""Host-side logic of the drivers, without a GPU: fits, closed forms, launch
shape candidates, observable bookkeeping and input builders."""
import math
import os

import numpy as np
import pytest
import torch

import lbm_inputs


def test_tau_for_ohnesorge_inverts_eq_oh_tcap():
    from paper_1905_09554_amd import calibration
    for rl, sigma, R0, oh in ((2.1086, 0.0495, 14, 0.1), (2.1775, 0.08991, 98, 0.1),
                              (1.9, 0.035, 30, 0.25)):
        tau = calibration.tau_for_ohnesorge(oh, rl, sigma, R0)
        nu = (tau - 0.5) / 3.0
        assert abs(rl * nu / math.sqrt(rl * sigma * R0) - oh) < 1e-14
    # Table 2 (MRT, sigma independent of tau): tau of the R0 = 14 column.
    t = lbm_inputs.PAPER_TABLE["mrt"]
    tau = calibration.tau_for_ohnesorge(0.1, t["rho_l"][0], t["sigma"][0], 14)
    assert abs(tau / t["tau"][0] - 1) < 0.005


def test_autotune_candidates_are_valid_shapes():
    from paper_1905_09554_amd import autotune
    for nx, prec, nodes in ((256, "f32", None), (256, "f64", None), (32, "f64", 65536),
                            (600, "f32", None), (672, "f32", None)):
        cands = autotune.candidates(nx, prec, nodes=nodes)
        assert cands
        assert any(c["z_chunk"] < 16 for c in cands) == (nodes is not None)
        for c in cands:
            cap = c["threads"] * c["nodes_per_thread"]
            assert c["block_x"] <= min(nx, cap)
            if c["block_x"] < nx:
                even_split = nx % c["block_x"] == 0 and c["block_x"] % 16 == 0
                assert (c["block_x"] % 64 == 0 or even_split) and 2 * c["block_x"] <= cap
                assert c["block_x"] >= 64
            if prec == "f64":
                assert c["threads"] <= 512 and c["nodes_per_thread"] == 1
    # A 672-node row also splits into 2, 3 and 6 even tiles (336, 224, 112).
    widths = {c["block_x"] for c in autotune.candidates(672, "f32")}
    assert {336, 224, 112} <= widths


def test_batch_autotune_candidates_are_valid_shapes():
    from paper_1905_09554_amd import autotune
    cands = autotune.batch_candidates()
    assert len(cands) == len({tuple(sorted(c.items())) for c in cands})
    for c in cands:
        assert c["threads"] in (256, 512, 1024)
        assert c["z_chunk"] >= 1 and c["xcd_remap"] in (0, 1) and c["persistent"] == 0
    # the measured default (1024 threads, 8-plane chunks, plain order) is among them
    assert dict(threads=1024, z_chunk=8, xcd_remap=0, persistent=0) in cands


def test_growth_fit_recovers_an_exponential():
    from paper_1905_09554_amd import dispersion
    t = np.arange(0, 5000, 50.0)
    a = 0.3 * np.exp(4e-4 * t)
    assert abs(dispersion.fit_growth(t, a, R=30, t_start=1000) - 4e-4) < 1e-12
    # the window stops at a <= 0.15 R: too few samples left -> None
    assert dispersion.fit_growth(t, a, R=30, t_start=4900) is None


def test_mode_amplitude_of_a_cosine():
    from paper_1905_09554_amd import dispersion
    nz = 96
    z = np.arange(nz)
    r = 20.0 + 0.7 * np.cos(2 * math.pi * z / nz) + 0.3 * np.cos(4 * math.pi * z / nz)
    assert abs(dispersion.mode_amplitude(r) - 0.7) < 1e-12


class _FakeSim:
    """Stands in for lbsc.Simulation: a radius profile of m wavelengths
    (info["wavelengths"], default 2) that narrows at the necks z = nz/(2m)
    (2k + 1) and a uniform velocity field."""

    def __init__(self, info):
        self.info = info
        self.k = 0

    def diagnostics(self, rho_v, rho_l):
        nz = self.info["nz"]
        m = self.info.get("wavelengths", 2)
        z = np.arange(nz)
        amp = 1.0 + 0.1 * self.k
        r = self.info["R0"] * (1.0 + 0.1 * amp * np.cos(2 * m * math.pi * z / nz))
        return {"r_of_z": r}

    def moments(self, want_u=True, want_p=False):
        i = self.info
        u = torch.zeros((3, i["nz"], i["ny"], i["nx"]), dtype=torch.float64)
        u[2] = 0.01
        return None, u, None


def test_recorder_bookkeeping():
    from paper_1905_09554_amd import breakup
    info = {"nx": 8, "ny": 8, "nz": 64, "R0": 14, "t_cap": 100.0, "rho_v": 0.08, "rho_l": 2.1}
    rec = breakup.Recorder(info, silhouette_tstar=(1.0, 2.0), velocity_tstar=(1.5,))
    sim = _FakeSim(info)
    for k in range(0, 26):
        sim.k = k
        rec.sample(sim, 10 * k, last=(k == 25))
    r = rec.result()
    assert r["t_star"][0] == 0.0 and abs(r["t_star"][-1] - 2.5) < 1e-12
    # perturbation amplitude 1 + 0.1 k, normalised by its initial value
    assert np.allclose(r["neck_perturbation"], 1.0 + 0.1 * np.arange(26))
    assert np.allclose(r["crest_perturbation"], 1.0 + 0.1 * np.arange(26))
    assert sorted(r["silhouettes"]) == [1.0, 2.0]
    assert r["silhouettes"][1.0][0] == 100 and r["silhouettes"][2.0][0] == 200
    st, v = r["velocity"][1.5]
    assert st == 150 and v.shape == (64, 8)
    assert np.allclose(v, 0.01 / (14 / 100.0))
    assert abs(r["h_min_over_R0"][0] - 0.9) < 1e-12


def test_recorder_neck_of_a_one_wavelength_box():
    """With one wavelength in the box the neck is the middle slice."""
    from paper_1905_09554_amd import breakup
    info = {"nx": 8, "ny": 8, "nz": 64, "R0": 14, "t_cap": 100.0, "rho_v": 0.08, "rho_l": 2.1,
            "wavelengths": 1}
    rec = breakup.Recorder(info, silhouette_tstar=(), velocity_tstar=())
    sim = _FakeSim(info)
    for k in range(0, 11):
        sim.k = k
        rec.sample(sim, 10 * k)
    r = rec.result()
    assert np.allclose(r["neck_perturbation"], 1.0 + 0.1 * np.arange(11))
    assert np.allclose(r["crest_perturbation"], 1.0 + 0.1 * np.arange(11))
    _, info2 = lbm_inputs.paper_ligament(14, "mrt", wavelengths=1)
    assert info2["wavelengths"] == 1 and info2["nz"] == 128


def test_droplet_and_slab_inputs():
    d = lbm_inputs.droplet_density(24, 6.0, 0.1, 2.0)
    assert d.shape == (24, 24, 24)
    assert d[12, 12, 12] > 1.99 and d[0, 0, 0] < 0.11
    assert np.allclose(d, d.transpose(1, 0, 2)) and np.allclose(d, d.transpose(2, 1, 0))
    s = lbm_inputs.slab_density(32, 8, 0.1, 2.0)
    assert s.shape == (32, 1, 1) and s[16, 0, 0] > 1.99 and s[0, 0, 0] < 0.11


@pytest.mark.parametrize("R0,op", [(14, "mrt"), (28, "srt")])
def test_paper_ligament_geometry(R0, op):
    rho, info = lbm_inputs.paper_ligament(R0, op)
    assert rho.shape == (256 * R0 // 14, 96 * R0 // 14, 96 * R0 // 14)
    assert info["nz"] == 256 * R0 // 14
    # k R0 of two wavelengths in L_x is the fastest mode, 4 pi 14 / 256
    assert abs(4 * math.pi * R0 / info["nz"] - 0.687) < 0.001


def test_drop_segmentation_and_satellites():
    from paper_1905_09554_amd import breakup
    r = np.full(20, 2.0)
    r[6:8] = 1.0
    smax = np.where(np.isin(np.arange(20), [4, 5, 9, 10, 14]), 0.05, 2.0)
    bodies = breakup.drops(smax, 1.0, r)
    # runs: 15..3 (wraps), 6..8, 11..13
    assert [(b[0], b[1]) for b in bodies] == [(6, 3), (11, 3), (15, 9)]
    assert abs(bodies[0][2] - math.pi * (1 + 1 + 4)) < 1e-12
    info = {"t_cap": 100.0}
    big = (0, 9, 100.0)
    sat = (0, 2, 5.0)
    # satellites from the sample at t = 50 to the first sample without them
    # (150): 1.0 t_cap; again from 200 to the end of the run (300): 1.0
    history = [(0, [big, big]), (50, [big, sat, big]), (100, [big, sat, big, sat]),
               (150, [big, big]), (200, [big, sat, big]), (300, [big, sat, big])]
    s = breakup.satellites(history, info)
    assert s["max"] == 2 and s["final"] == 1 and abs(s["life_tcap"] - 1.0) < 1e-12
    assert s["bodies_final"] == 3
    # a satellite that outlives the run is counted up to the last sample
    s = breakup.satellites([(0, [big]), (100, [big, sat]), (400, [big, sat])], info)
    assert abs(s["life_tcap"] - 3.0) < 1e-12


def test_counter_reduction_scales_by_the_copy(tmp_path):
    """traffic.py on synthetic rocprofv3 counter files: the copy's reading
    calibrates each counter (FETCH_SIZE reads half a copy's bytes), and the
    step kernel's per-launch bytes follow."""
    import csv as _csv
    from paper_1905_09554_amd import traffic
    from paper_1905_09554_amd.prof_driver import COPY_BYTES
    kib = COPY_BYTES / 1024.0
    nodes = 1000
    for counter, copy_val, step_val in (("FETCH_SIZE", kib / 2, 80.0), ("WRITE_SIZE", kib, 75.0)):
        d = tmp_path / counter
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as fh:
            w = _csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for v in (step_val - 1, step_val + 1):
                w.writerow({"Kernel_Name": "void k_step<float, 1, 0, 1024, 1>(...)",
                            "Counter_Name": counter, "Counter_Value": v})
            w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter,
                        "Counter_Value": copy_val})
    rec = traffic.reduce_counters(traffic._rows(str(tmp_path / "FETCH_SIZE"), "FETCH_SIZE"),
                                  traffic._rows(str(tmp_path / "WRITE_SIZE"), "WRITE_SIZE"),
                                  "f32", nodes)
    assert rec["dispatches"] == [2, 2]
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 80.0 * 2 * 1024
    assert rec["write_bytes_per_launch"] == 75.0 * 1024
    assert rec["algorithmic_bytes_per_launch"] == 2 * 19 * 4 * nodes


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_stale_counter_files_are_ignored(monkeypatch):
    """The benchmark uses the committed counter files only for the kernel
    sources and launch shape they were taken with."""
    import bench
    for prec in ("f32", "f64"):
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: "not-these-sources")
        assert bench.measured_traffic(bench.WORKLOAD, prec) is None
        monkeypatch.undo()
