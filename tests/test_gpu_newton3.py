"""The Newton's-third-law variant (newton3=1) on the GPU against the oracle.

Contract:
  half list: bit-exact against the oracle's half list (the full list's
    entries whose partner comes later in cell order, cell index then id), in
    atom-id space and in list order, with either list-build method;
  forces: the same per-atom and normwise bounds as the full-list pass
    (1e-12 FP64, 1e-5 FP32-mixed); the reaction forces are added with
    atomics, so the GPU result is reproducible to rounding only;
  runs: the oracle's trajectory within the full-list path's tolerances;
    total momentum stays at rounding level, as every pair adds F and -F.
"""
import numpy as np
import pytest

import oracle
from paper_2003_14061_amd import md

from gpu_helpers import (WCA, check_cells, check_nl, energy_error, force_errors, min_image,
                         oracle_cells, pair, state)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

CASES = {
    # name: (n, rho, r_cut, jitter, lattice, extra)
    "wca13500": (13500, 0.8, WCA, 0.1, True, {}),
    "wca13500_run": (13500, 0.8, WCA, 0.03, True, {}),
    "lj32000": (32000, 0.8, 2.5, 0.05, True, {}),
    "lj5000_random": (5000, 0.5, 2.5, 0.0, False, {}),
    "wca108_nc3": (108, 0.8, WCA, 0.08, True, {}),
    "lj4000_noreorder": (4000, 0.8442, 2.5, 0.05, True, {"reorder": False}),
}


def setup(name, precision="fp64", seed=17):
    n, rho, rc, jit, lat, extra = CASES[name]
    L, pos, vel = state(n, rho, seed, jitter=jit, lattice=lat)
    sim, s = pair(pos, vel, L, r_cut=rc, precision=precision, newton3=True, **extra)
    return sim, s, pos, vel


@pytest.mark.parametrize("method", [md.MD_NL_LANES, md.MD_NL_CELL_WAVES])
@pytest.mark.parametrize("name", [k for k in CASES if not k.endswith("_run")])
def test_half_list_and_forces_fp64(name, method):
    sim, s, pos, vel = setup(name)
    sim.set_tuning(nl_method=method)
    sim.build_cells()
    nc, cells = check_cells(sim, s, pos)
    sim.build_neighbors()
    o_cnt, o_nl = check_nl(sim, s, pos, cells, half=True)
    ref = oracle.forces_half(s, pos, o_cnt, o_nl)
    sim.forces()
    obs = sim.reduce()
    st = sim.state()
    per_atom, normwise = force_errors(st["f"], ref)
    assert per_atom <= TOL["fp64"] and normwise <= TOL["fp64"], (per_atom, normwise)
    assert energy_error(obs["U"], ref) <= TOL["fp64"]
    assert obs["W"] == pytest.approx(ref["w"].sum(), rel=1e-12, abs=1e-12)
    assert obs["max_nl"] == int(o_cnt.max())
    # the half list's forces are the full list's
    f_cnt, f_nl, _ = oracle.build_nl(s, nc, pos, cells)
    full = oracle.forces_nl(s, pos, f_cnt, f_nl)
    per_atom, normwise = force_errors(st["f"], full)
    assert per_atom <= TOL["fp64"] and normwise <= TOL["fp64"]


@pytest.mark.parametrize("name", ["wca13500", "lj32000", "lj5000_random"])
def test_half_forces_fp32_mixed(name):
    sim, s, pos, vel = setup(name, precision="fp32")
    sim.prepare()
    obs = sim.reduce()
    nc, cells = oracle_cells(sim, s, pos)
    cnt, nl, _ = oracle.build_nl_half(s, nc, pos, cells)
    ref = oracle.forces_half(s, pos, cnt, nl)
    per_atom, normwise = force_errors(sim.state()["f"], ref)
    assert per_atom <= TOL["fp32"] and normwise <= TOL["fp32"], (per_atom, normwise)
    assert energy_error(obs["U"], ref) <= TOL["fp32"]
    assert obs["W"] == pytest.approx(ref["w"].sum(), rel=1e-5)


TUNINGS = ([dict(force_lanes=l, force_block=b) for l in (1, 2, 4, 8) for b in (256, 1024)] +
           [dict(stage_cap=64), dict(stage_cap=64, force_lanes=4, tile_cells=2),
            dict(tile_cells=1, force_block=64), dict(tile_cells=1000, force_block=512),
            dict(tile_cells=2, tile_y=3, tile_z=2), dict(tile_y=2, tile_z=2, stage_cap=64)])


@pytest.mark.parametrize("name", ["lj32000", "wca108_nc3", "lj4000_noreorder"])
def test_every_tuning_matches_the_oracle(name):
    """Including tiles too large for LDS (stage_cap=64), whose reactions go
    straight to the force arrays."""
    sim, s, pos, vel = setup(name)
    sim.build_cells()
    nc, cells = check_cells(sim, s, pos)
    o_cnt, o_nl, _ = oracle.build_nl_half(s, nc, pos, cells)
    ref = oracle.forces_half(s, pos, o_cnt, o_nl)
    base = sim.get_tuning()
    for tu in TUNINGS:
        kw = dict(base, tile_cells=0, tile_y=0, tile_z=0, stage_cap=0)
        kw.update(tu)
        sim.set_tuning(**kw)
        sim.build_neighbors()
        check_nl(sim, s, pos, cells, half=True)
        sim.forces()
        obs = sim.reduce()
        per_atom, normwise = force_errors(sim.state()["f"], ref)
        assert per_atom <= TOL["fp64"] and normwise <= TOL["fp64"], tu
        assert energy_error(obs["U"], ref) <= TOL["fp64"], tu


@pytest.mark.parametrize("name", ["wca13500_run", "lj32000", "lj4000_noreorder", "wca108_nc3"])
def test_short_run_fp64(name):
    steps = 40
    sim, s, pos, vel = setup(name, seed=23)
    sim.prepare()
    sim.step(steps, record_every=1)
    h = sim.history()
    st = sim.state()
    p_ref, v_ref, _, o_ref, nreb = oracle.run(s, pos, vel, steps)
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(h["U"] - o_ref["U"])) <= 1e-10 * e_scale
    assert np.max(np.abs(h["K"] - o_ref["K"])) <= 1e-10 * e_scale
    assert np.abs(min_image(st["pos"] - p_ref, s.L)).max() < 1e-10
    assert np.abs(st["vel"] - v_ref).max() < 1e-9


def test_short_run_fp32_mixed():
    steps = 40
    sim, s, pos, vel = setup("lj32000", precision="fp32", seed=23)
    sim.prepare()
    sim.step(steps, record_every=1)
    h = sim.history()
    p_ref, v_ref, _, o_ref, _ = oracle.run(s, pos, vel, steps)
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(h["U"] - o_ref["U"])) <= 1e-5 * e_scale
    assert np.abs(min_image(sim.state()["pos"] - p_ref, s.L)).max() < 1e-5


def test_momentum_and_energy_conservation():
    L, pos, vel = state(32000, 0.8, 5)
    sim, s = pair(pos, vel, L, r_cut=2.5, dt=0.004, newton3=True)
    sim.prepare()
    sim.step(1000, record_every=10)
    h = sim.history()
    E = (h["U"] + h["K"]) / s.n
    assert np.abs(h["P"]).max() < 1e-9
    assert E.max() - E.min() < 5e-3


def test_batch_with_the_third_law():
    from test_gpu_batch import systems

    sys_ = systems(n_replicas=4, seed=13)
    b = md.Batch(sys_, precision="fp64", newton3=True)
    b.prepare()
    steps = 20
    b.run(steps, record_every=1)
    for r, sy in enumerate(sys_):
        s = oracle.make_sys(len(sy["pos"]), sy["L"], r_cut=sy["r_cut"], skin=sy["skin"],
                            dt=sy["dt"])
        p_ref, v_ref, _, o_ref, _ = oracle.run(s, sy["pos"], sy["vel"], steps)
        st, h = b.state(r), b.history(r)
        e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
        assert np.max(np.abs(h["U"] - o_ref["U"])) <= 1e-10 * e_scale, r
        assert np.abs(min_image(st["pos"] - p_ref, sy["L"])).max() < 1e-10, r


def test_unsupported_combinations_are_rejected():
    from test_gpu_batch import systems

    sys_ = systems(n_replicas=2)
    p = [md.Params(len(sy["pos"]), md.MD_LJ_SHIFTED, sy["L"], 1.0, 1.0, 1.0, sy["r_cut"], 0.3,
                   0.005, md.MD_FP64, md.MD_NEIGHBOR_LIST, r, 0, 1, 256)
         for r, sy in enumerate(sys_)]
    with pytest.raises(md.MDError):  # mixed newton3 in one batch
        md.md_batch_init(p, 2)
    L, pos, vel = state(4000, 0.8, 3)
    sim, s = pair(pos, vel, L, r_cut=2.5, reorder=False, newton3=True)
    sim.prepare()
    with pytest.raises(md.MDError):  # the reverse mode differentiates the full-list pass
        sim.traj_forward(10, 5)
