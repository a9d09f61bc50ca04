"""The paper's own layer-matrix pipeline (MD_PIPE_LAYERS) on the GPU against
the oracle.

Contract: cell of every atom bit-exact; the layer matrix holds exactly each
cell's atoms (in the order of the atomics, so compared as sets) and the
occupancy counts are exact; every atom's neighbor list has the oracle's
length and content, with the cells visited in the canonical (dz, dy, dx)
order (inside a cell the order is the atomics'); forces within 1e-12 (FP64)
and 1e-5 (FP32-mixed) of the oracle; short runs within the trajectory
tolerances of the tiled path; a cell holding more atoms than layers is
latched and reported."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2003_14061_amd import md

from gpu_helpers import WCA, energy_error, force_errors, min_image, state

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

CASES = {
    # name: (n, rho, r_cut, jitter, lattice)
    "wca13500": (13500, 0.8, WCA, 0.1, True),
    "lj32000": (32000, 0.8, 2.5, 0.05, True),
    "lj5000_random": (5000, 0.5, 2.5, 0.0, False),
    "wca108_nc3": (108, 0.8, WCA, 0.08, True),
}


def setup(name, precision="fp64", seed=17):
    n, rho, rc, jit, lat = CASES[name]
    L, pos, vel = state(n, rho, seed, jitter=jit, lattice=lat)
    sim = md.Simulation(pos, vel, L, r_cut=rc, skin=0.3, dt=0.005, precision=precision,
                        pipeline="layers")
    s = oracle.make_sys(n, L, r_cut=rc, skin=0.3, dt=0.005, nl_cap=sim.grid.nl_capacity)
    return sim, s, pos, vel


def stencil_index(c, c2, nc):
    """Position of cells c2 among the 27 neighbors of cell c, (dz, dy, dx) order."""
    cx, cy, cz = c % nc, (c // nc) % nc, c // (nc * nc)
    dx = ((c2 % nc - cx + 1) % nc) - 1
    dy = (((c2 // nc) % nc - cy + 1) % nc) - 1
    dz = ((c2 // (nc * nc) - cz + 1) % nc) - 1
    return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)


@pytest.mark.parametrize("name", list(CASES))
def test_layers_list_and_forces_fp64(name):
    sim, s, pos, vel = setup(name)
    sim.build_cells()
    nc = sim.grid.nc
    o_of, o_start, o_atoms = oracle.build_cells(s, nc, pos)
    # N1: cells (slots are ids: this pipeline never reorders)
    cell_of = sim._host(sim.ws_array(md.MD_ARR_CELL_OF, torch.int32))[0]
    assert np.array_equal(cell_of, o_of), "cell of each atom differs"
    # N2-N4: the layer matrix holds each cell's atoms
    H, occ = sim.layers()
    assert np.array_equal(occ, np.diff(o_start)), "occupancy differs"
    for cell in range(sim.grid.n_cells):
        got = np.sort(H[cell, : occ[cell]])
        assert np.array_equal(got, np.sort(o_atoms[o_start[cell]: o_start[cell + 1]])), cell
    sim.build_neighbors()
    o_cnt, o_nl, _ = oracle.build_nl(s, nc, pos, (o_of, o_start, o_atoms))
    cnt, nl = sim.neighbor_list()
    n = len(pos)
    assert np.array_equal(cnt[:n], o_cnt), "list lengths differ"
    for i in range(n):
        got = nl[: cnt[i], i]
        assert np.array_equal(np.sort(got), np.sort(o_nl[i, : o_cnt[i]])), i
        # cells in canonical stencil order (inside a cell: the atomics' order)
        st = stencil_index(o_of[i], o_of[got], nc)
        assert np.all(np.diff(st) >= 0), i
    ref = oracle.forces_nl(s, pos, o_cnt, o_nl)
    sim.forces()
    obs = sim.reduce()
    f = sim.state()["f"]
    per_atom, normwise = force_errors(f, ref)
    assert per_atom <= TOL["fp64"] and normwise <= TOL["fp64"], (per_atom, normwise)
    assert energy_error(obs["U"], ref) <= TOL["fp64"]
    assert obs["W"] == pytest.approx(ref["w"].sum(), rel=1e-12, abs=1e-12)
    assert obs["max_nl"] == int(o_cnt.max())
    assert obs["max_occupancy"] == int(np.diff(o_start).max())


@pytest.mark.parametrize("name", ["wca13500", "lj32000"])
def test_layers_forces_fp32_mixed(name):
    sim, s, pos, vel = setup(name, precision="fp32")
    sim.prepare()
    obs = sim.reduce()
    nc = sim.grid.nc
    cells = oracle.build_cells(s, nc, pos)
    cnt, nl, _ = oracle.build_nl(s, nc, pos, cells)
    ref = oracle.forces_nl(s, pos, cnt, nl)
    per_atom, normwise = force_errors(sim.state()["f"], ref)
    assert per_atom <= TOL["fp32"] and normwise <= TOL["fp32"], (per_atom, normwise)
    assert energy_error(obs["U"], ref) <= TOL["fp32"]


@pytest.mark.parametrize("name", ["wca13500", "lj32000", "wca108_nc3"])
def test_layers_short_run_fp64(name):
    steps = 40
    n, rho, rc, jit, lat = CASES[name]
    L, pos, vel = state(n, rho, 23, jitter=min(jit, 0.03), lattice=lat)
    sim = md.Simulation(pos, vel, L, r_cut=rc, skin=0.3, dt=0.005, pipeline="layers")
    s = oracle.make_sys(n, L, r_cut=rc, skin=0.3, dt=0.005, nl_cap=sim.grid.nl_capacity)
    sim.prepare()
    sim.step(steps, record_every=1)
    h = sim.history()
    st = sim.state()
    p_ref, v_ref, _, o_ref, nreb = oracle.run(s, pos, vel, steps)
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(h["U"] - o_ref["U"])) <= 1e-10 * e_scale
    assert np.max(np.abs(h["K"] - o_ref["K"])) <= 1e-10 * e_scale
    assert np.abs(min_image(st["pos"] - p_ref, L)).max() < 1e-10
    assert np.abs(st["vel"] - v_ref).max() < 1e-9
    assert sim.reduce()["n_rebuilds"] == nreb


def test_layer_overflow_is_latched():
    # a dilute box with one dense cluster: 64 atoms 0.9 apart inside one cell
    L, pos, vel = state(2000, 0.1, 3, lattice=False)
    grid = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    cluster = 0.5 + 0.6 * grid
    pos[:64] = cluster
    vel[:] = 0.0
    sim = md.Simulation(pos, vel, L, r_cut=2.5, skin=0.3, dt=0.001, pipeline="layers")
    assert sim.grid.n_layers < 64
    sim.prepare()
    with pytest.raises(md.MDError) as e:
        sim.reduce()
    assert e.value.status == -8
    assert sim.reduce(check=False)["flags"] & 4


@pytest.mark.parametrize("name", ["wca13500", "lj32000"])
def test_layers_reorder_every_k_steps(name):
    """The paper's periodic reorder (section 2.4 item (4)): every 10th step
    the atoms are permuted into the layer matrix's cell order and both
    matrices rebuilt.  The trajectory stays the oracle's (the list holds the
    same pairs; only summation order and the rebuild schedule move), the
    slots end up in cell order, and the ids follow the atoms."""
    steps, every = 40, 10
    n, rho, rc, jit, lat = CASES[name]
    L, pos, vel = state(n, rho, 23, jitter=min(jit, 0.03), lattice=lat)
    sim = md.Simulation(pos, vel, L, r_cut=rc, skin=0.3, dt=0.005, pipeline="layers",
                        reorder=every)
    s = oracle.make_sys(n, L, r_cut=rc, skin=0.3, dt=0.005, nl_cap=sim.grid.nl_capacity)
    sim.prepare()
    assert np.array_equal(sim.ids(), np.arange(n))
    # the layer matrix of the last build before step 10 gives the sequence
    sim.step(every - 1, record_every=1)
    nl_ = sim.grid.n_layers
    lay, cnt_, ids0 = sim._host(sim.ws_array(md.MD_ARR_LAYERS, torch.int32),
                                sim.ws_array(md.MD_ARR_LAYER_COUNT, torch.int32), sim.id)
    lay = lay.reshape(-1, nl_)
    seq = np.concatenate([lay[c, :cnt_[c]] for c in range(len(cnt_))])
    assert sorted(seq.tolist()) == list(range(n))
    sim.step(1, record_every=1)
    assert np.array_equal(sim.ids(), ids0[seq])
    sim.step(steps - every, record_every=1)
    h = sim.history()
    st = sim.state()
    p_ref, v_ref, _, o_ref, _ = oracle.run(s, pos, vel, steps)
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(h["U"] - o_ref["U"])) <= 1e-10 * e_scale
    assert np.max(np.abs(h["K"] - o_ref["K"])) <= 1e-10 * e_scale
    assert np.abs(min_image(st["pos"] - p_ref, L)).max() < 1e-10
    assert np.abs(st["vel"] - v_ref).max() < 1e-9
    ids = sim.ids()
    assert sorted(ids.tolist()) == list(range(n)) and not np.array_equal(ids, np.arange(n))
    # forces of the final state against the oracle's
    nc = sim.grid.nc
    p = np.mod(st["pos"], L)
    cells = oracle.build_cells(s, nc, p)
    cnt, nl, _ = oracle.build_nl(s, nc, p, cells)
    per_atom, normwise = force_errors(st["f"], oracle.forces_nl(s, p, cnt, nl))
    assert per_atom <= 1e-12 and normwise <= 1e-12


def test_layers_timing_parts():
    """md_set_timing brackets every part of a step (the rows of the paper's
    Table 2): one group per step for each part, one reorder per k steps, and
    the force part is what md_get_timing reports."""
    n, rho, rc, jit, lat = CASES["wca13500"]
    L, pos, vel = state(n, rho, 23, jitter=0.03, lattice=lat)
    sim = md.Simulation(pos, vel, L, r_cut=rc, skin=0.3, dt=0.005, pipeline="layers",
                        reorder=10)
    sim.prepare()
    sim.set_timing(True)
    sim.step(30)
    parts = sim.get_timing_parts()
    for k in ("neighbors", "forces", "integrate", "energy", "cells"):
        assert parts[k][1] == 30 and parts[k][0] > 0, k
    assert parts["reorder"][1] == 3 and parts["reorder"][0] > 0
    f_ms, f_n = sim.get_timing()
    assert f_n == 30 and f_ms == pytest.approx(parts["forces"][0])
    assert sim.reduce()["flags"] == 0


def test_layers_reorder_with_overflow_leaves_the_state():
    """A latched layer overflow stops the reorder (the layer matrix then
    lacks atoms): the slots keep their atoms."""
    L, pos, vel = state(2000, 0.1, 3, lattice=False)
    grid = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos[:64] = 0.5 + 0.6 * grid
    vel[:] = 0.0
    sim = md.Simulation(pos, vel, L, r_cut=2.5, skin=0.3, dt=0.001, pipeline="layers",
                        reorder=2)
    sim.prepare()
    sim.step(4)
    assert np.array_equal(sim.ids(), np.arange(2000))
    assert sim.reduce(check=False)["flags"] & 4
