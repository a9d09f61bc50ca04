"""The all-pairs force evaluation (MD_PIPE_ALLPAIRS, the comparison method of
section 4.2) on the GPU against the oracle's brute force.

Contract: forces within 1e-12 (FP64) and 1e-5 (FP32-mixed) of the oracle's
all-pairs sums, per atom scaled by S_i and normwise; energy and virial
totals to the same bounds; the same forces bit for bit on a repeated call
(the chunk partials are added in a fixed order); positions folded into
[0, L) by the cell step; short runs follow the oracle's cells-only
trajectory.  The split of the partners into chunks is exercised at 1, 2, 8
and 16 chunks per home block, with a ragged last home block and a ragged
last tile, and on a box smaller than one home block.  At 100 000 and
256 000 atoms the oracle's brute force runs on a sample of atoms and its
list-based pass gives the totals."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2003_14061_amd import md

from gpu_helpers import WCA, energy_error, force_errors, min_image, state

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

CASES = {
    # name: (n, rho, r_cut, jitter, lattice); chunks per home block in the comment
    "wca4000": (4000, 0.8, WCA, 0.05, True),         # 16 chunks, ragged tile and block
    "lj2000_random": (2000, 0.5, 2.5, 0.0, False),  # 8 chunks
    "lj2048": (2048, 0.8, 2.5, 0.05, True),          # 8 chunks, whole tiles and blocks
    "wca40_tiny": (40, 0.3, WCA, 0.05, True),        # one chunk, one partial home block
}


def setup(name, precision="fp64", seed=29):
    n, rho, rc, jit, lat = CASES[name]
    L, pos, vel = state(n, rho, seed, jitter=jit, lattice=lat)
    sim = md.Simulation(pos, vel, L, r_cut=rc, dt=0.005, precision=precision,
                        pipeline="allpairs")
    s = oracle.make_sys(n, L, r_cut=rc, dt=0.005, use_nl=False)
    return sim, s, pos, vel, L


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_allpairs_forces_match_the_oracle(name, precision):
    sim, s, pos, _, _ = setup(name, precision)
    sim.prepare()
    obs = sim.reduce()
    ref = oracle.forces_allpairs(s, pos)
    per_atom, normwise = force_errors(sim.state()["f"], ref)
    assert per_atom <= TOL[precision] and normwise <= TOL[precision], (per_atom, normwise)
    assert energy_error(obs["U"], ref) <= TOL[precision]
    assert obs["W"] == pytest.approx(ref["w"].sum(), rel=10 * TOL[precision], abs=1e-9)
    assert obs["flags"] == 0


def test_allpairs_forces_repeat_bit_for_bit():
    sim, _, _, _, _ = setup("wca4000")
    sim.prepare()
    f0 = sim.state()["f"]
    u0 = sim.reduce()["U"]
    for _ in range(3):
        sim.forces()
    assert np.array_equal(sim.state()["f"], f0)
    assert sim.reduce()["U"] == u0


def test_allpairs_cell_step_folds_positions():
    n, rho, rc, jit, lat = CASES["wca4000"]
    L, pos, vel = state(n, rho, 31, jitter=jit, lattice=lat)
    moved = pos.copy()
    moved[::7] += L        # one box length above
    moved[3::11] -= L      # and below
    sim = md.Simulation(moved, vel, L, r_cut=rc, dt=0.005, pipeline="allpairs")
    sim.prepare()
    st = sim.state()
    assert st["pos"].min() >= 0.0 and st["pos"].max() < L
    assert np.abs(min_image(st["pos"] - pos, L)).max() < 1e-12
    s = oracle.make_sys(n, L, r_cut=rc, dt=0.005, use_nl=False)
    ref = oracle.forces_allpairs(s, st["pos"])
    per_atom, normwise = force_errors(st["f"], ref)
    assert per_atom <= 1e-12 and normwise <= 1e-12


@pytest.mark.parametrize("name", ["wca4000", "wca40_tiny", "lj2048"])
def test_allpairs_short_run_follows_the_oracle(name):
    steps = 40
    n, rho, rc, jit, lat = CASES[name]
    L, pos, vel = state(n, rho, 37, jitter=min(jit, 0.03), lattice=lat)
    sim = md.Simulation(pos, vel, L, r_cut=rc, dt=0.004, pipeline="allpairs")
    s = oracle.make_sys(n, L, r_cut=rc, dt=0.004, use_nl=False)
    sim.prepare()
    sim.step(steps, record_every=1)
    h = sim.history()
    st = sim.state()
    p_ref, v_ref, _, o_ref, _ = oracle.run(s, pos, vel, steps)
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(h["U"] - o_ref["U"])) <= 1e-10 * e_scale
    assert np.max(np.abs(h["K"] - o_ref["K"])) <= 1e-10 * e_scale
    assert np.abs(min_image(st["pos"] - p_ref, L)).max() < 1e-10
    assert np.abs(st["vel"] - v_ref).max() < 1e-9
    assert st["pos"].min() >= 0.0 and st["pos"].max() < L


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [100000, 256000])
def test_allpairs_large_systems_on_samples(n, precision):
    """Two chunks per home block at 100 000 atoms, one at 256 000."""
    L, pos, vel = state(n, 0.8, 41, jitter=0.05)
    sim = md.Simulation(pos, vel, L, r_cut=WCA, dt=0.005, precision=precision,
                        pipeline="allpairs")
    sim.prepare()
    obs = sim.reduce()
    f = sim.state()["f"]
    s = oracle.make_sys(n, L, r_cut=WCA, dt=0.005, use_nl=False)
    idx = np.sort(np.random.default_rng(3).choice(n, 1500, replace=False)).astype(np.int32)
    # the sample reaches both chunks and the ragged end
    idx[-1] = n - 1
    idx[0] = 0
    ref = oracle.forces_sample(s, pos, idx)
    per_atom, normwise = force_errors(f[idx], ref)
    assert per_atom <= TOL[precision] and normwise <= TOL[precision], (per_atom, normwise)
    # totals from the oracle's list pass (the same pair sums)
    sl = oracle.make_sys(n, L, r_cut=WCA, skin=0.3, dt=0.005)
    nc = oracle.cells_per_side(L, WCA + 0.3)
    cells = oracle.build_cells(sl, nc, pos)
    cnt, nl, _ = oracle.build_nl(sl, nc, pos, cells)
    full = oracle.forces_nl(sl, pos, cnt, nl)
    assert energy_error(obs["U"], full) <= TOL[precision]
    assert obs["W"] == pytest.approx(full["w"].sum(), rel=10 * TOL[precision], abs=1e-9)


def test_allpairs_coincident_atoms_are_flagged():
    n, rho, rc, jit, lat = CASES["wca4000"]
    L, pos, vel = state(n, rho, 43, jitter=jit, lattice=lat)
    pos[1] = pos[0]
    sim = md.Simulation(pos, vel, L, r_cut=rc, dt=0.005, pipeline="allpairs")
    sim.prepare()
    with pytest.raises(md.MDError) as e:
        sim.reduce()
    assert e.value.status == -4
    assert sim.reduce(check=False)["flags"] & 2


def test_allpairs_has_no_cells_and_no_list():
    sim, _, _, _, _ = setup("wca40_tiny")
    sim.prepare()
    with pytest.raises(md.MDError):
        sim.cells()
    with pytest.raises(md.MDError):
        sim.neighbor_list()
    with pytest.raises(md.MDError):
        md.md_build_neighbors(sim.ctx)
    assert sim.reduce()["flags"] == 0
