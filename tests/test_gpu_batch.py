"""Batched boxes: many ligaments of uneven size and parameters stepped together
(one launch per step, or one cooperative launch with grid barriers).  Each
member must match a run of the same box alone, bitwise, and the oracle."""
import numpy as np
import pytest
import torch

import lbm_inputs
from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu


def _members(precision, collision, forcing="guo"):
    from paper_1905_09554_amd import lbsc
    rv, rl = lbm_inputs.coexistence(-5.0)
    specs = [(32, 32, 50, 8.0, 1.0), (44, 44, 37, 11.0, 0.8), (24, 24, 60, 6.0, 0.9),
             (36, 20, 18, 5.0, 0.7)]
    rhos, params = [], []
    for nx, ny, nz, R, tau in specs:
        rhos.append(lbm_inputs.ligament_density(nx, ny, nz, R, 0.05, 1, rv, rl, noise=1e-4,
                                                seed=nx))
        params.append(lbsc.make_params(nx, ny, nz, collision=collision, forcing=forcing,
                                       precision=precision, G=-5.0, tau=tau))
    return rhos, params


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("precision,collision", [("f32", "mrt"), ("f64", "bgk"), ("f32", "bgk")])
def test_batch_members_equal_single_runs_bitwise(precision, collision, persistent):
    from paper_1905_09554_amd import lbsc
    rhos, params = _members(precision, collision)
    b = lbsc.Batch(rhos, params)
    b.set_tuning(persistent=persistent)
    b.step(7)
    b.step(6)
    assert b.step_count == 13
    for i, (r, p) in enumerate(zip(rhos, params)):
        sim = lbsc.Simulation(r, p)
        sim.step(13)
        single, _ = sim.get_state()
        sim.close()
        assert np.array_equal(b.get_state(i), single), i
    b.close()


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_velocity_shift_members_equal_single_runs_bitwise(precision, persistent):
    """The paper's SRT operator (BGK with the velocity shift) in a batch."""
    from paper_1905_09554_amd import lbsc
    rhos, params = _members(precision, "bgk", forcing="shift")
    b = lbsc.Batch(rhos, params)
    b.set_tuning(persistent=persistent)
    b.step(11)
    for i, (r, p) in enumerate(zip(rhos, params)):
        sim = lbsc.Simulation(r, p)
        sim.step(11)
        single, _ = sim.get_state()
        sim.close()
        assert np.array_equal(b.get_state(i), single), i
    b.close()


def test_persistent_single_box_equals_plain_launches():
    from paper_1905_09554_amd import lbsc
    rho0 = gc.ligament(40, 36, 30, 8.0, 0.1, 1, noise=1e-4)
    for prec in ("f32", "f64"):
        prm = lbsc.make_params(40, 36, 30, collision="mrt", precision=prec)
        a = lbsc.Simulation(rho0, prm)
        a.step(11)
        b = lbsc.Simulation(rho0, prm)
        b.set_tuning(persistent=1)
        b.step(11)
        assert np.array_equal(a.get_state()[0], b.get_state()[0])


def test_batch_member_matches_oracle_and_diagnostics():
    from paper_1905_09554_amd import lbsc
    rhos, params = _members("f64", "mrt")
    b = lbsc.Batch(rhos, params)
    b.set_tuning(persistent=1)
    b.step(25)
    rv, rl = lbm_inputs.coexistence(-5.0)
    for i in (1, 3):
        p = params[i]
        o = gc.run_oracle(rhos[i], 25, collision="mrt", tau=p.tau)
        st = b.get_state(i)[gc.population_perm()]
        assert float(np.abs(st - o["state"]).max()) < 1e-12
        d = b.diagnostics(i, rv, rl)
        from oracle import diagnostics
        od = diagnostics.interface_diagnostics(o["f"], o["params"], rv, rl)
        assert abs(d["mass"] - od["mass"]) < 1e-12 * od["mass"]
        assert float(np.abs(d["r_of_z"] - od["r_of_z"].numpy()).max()) < 1e-12
        assert d["z_argmin"] == od["z_argmin"]
        rho, u, _ = b.moments(i)
        assert float(np.abs(rho.cpu().numpy() - o["rho"]).max()) < 1e-12
        assert float(np.abs(u.cpu().numpy() - o["u"]).max()) < 1e-12
    b.close()


def test_dispersion_batch_full_size_sampled():
    """The 64-ligament sweep (R ~ U{8..48}, kR ~ U[0.3, 0.95], 4R x 4R boxes)
    in the launch configuration the benchmark times; sampled nodes of every
    member against the oracle on patches."""
    from paper_1905_09554_amd import dispersion, lbsc
    sweep = dispersion.make_sweep(seed=0)
    b = dispersion.build_batch(sweep)
    steps = 2
    b.step(steps)
    rng = np.random.default_rng(5)
    total = sum(m["rho0"].size for m in sweep["members"])
    print("batch of %d members, %d nodes" % (len(sweep["members"]), total), flush=True)
    for i, m in enumerate(sweep["members"]):
        if i % 4:
            continue
        rho, u, _ = b.moments(i)
        nz, ny, nx = m["rho0"].shape
        nodes = [(int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx)))
                 for _ in range(3)] + [(0, 0, 0), (nz - 1, ny // 2, nx // 2)]
        for node in nodes:
            r_ref, u_ref = gc.oracle_at_node(m["rho0"], node, steps, "bgk", G=m["G"], tau=m["tau"])
            r_gpu = float(rho[node].cpu())
            assert abs(r_gpu - r_ref) <= 1e-5 * r_ref, (i, node, r_gpu, r_ref)
            assert float(np.abs(u[(slice(None),) + node].cpu().numpy() - u_ref).max()) <= 1e-6
        del rho, u
    b.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tuning", [None, dict(threads=1024), dict(threads=256, block_x=64),
                                    dict(threads=1024, block_x=128, persistent=1)])
def test_batch_wide_and_narrow_members_bitwise(tuning):
    """Members whose rows are wider than a work-group (split into x tiles,
    ragged last tile) next to narrow ones, against single runs."""
    from paper_1905_09554_amd import lbsc
    rv, rl = lbm_inputs.coexistence(-5.0)
    specs = [(1100, 3, 4), (300, 6, 8), (40, 40, 12)]
    rhos, params = [], []
    for nx, ny, nz in specs:
        g_ = np.random.default_rng(nx)
        rhos.append(rv + (rl - rv) * g_.random((nz, ny, nx)))
        params.append(lbsc.make_params(nx, ny, nz, collision="mrt", precision="f32", G=-5.0,
                                       tau=0.9))
    b = lbsc.Batch(rhos, params)
    if tuning:
        b.set_tuning(**tuning)
    b.step(9)
    for i, (r, p) in enumerate(zip(rhos, params)):
        sim = lbsc.Simulation(r, p)
        sim.step(9)
        single, _ = sim.get_state()
        sim.close()
        assert np.array_equal(b.get_state(i), single), (i, tuning)
    b.close()


def test_batch_autotune_candidates_bitwise():
    """Every fourth launch shape the batch autotuner times (and the persistent
    form of two of them) leaves every member bitwise equal to its single run."""
    from paper_1905_09554_amd import autotune, lbsc
    rhos, params = _members("f32", "bgk")
    singles = []
    for r, p in zip(rhos, params):
        sim = lbsc.Simulation(r, p)
        sim.step(9)
        singles.append(sim.get_state()[0])
        sim.close()
    cands = autotune.batch_candidates()[::4]
    cands += [dict(cands[0], persistent=1), dict(cands[-1], persistent=1)]
    for shape in cands:
        b = lbsc.Batch(rhos, params)
        b.set_tuning(**shape)
        b.step(9)
        for i in range(len(rhos)):
            assert np.array_equal(b.get_state(i), singles[i]), (i, shape)
        b.close()
