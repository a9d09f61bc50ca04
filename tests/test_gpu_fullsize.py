"""Parity at the full workload sizes, in the launch configuration bench.py
times (default tuning, or the autotuner's pick for the ensemble):

  * the 2.048M-atom LJ system and the 256 000-atom WCA system after a stretch
    of steps: cells bit-exact over all atoms, every list entry of every atom
    in list order, brute-force forces of a sample of atoms, total energy and
    virial against the oracle's full-list sums, kinetic energy and momentum;
  * the 64-replica ensemble, every replica against its own oracle run;
  * the 4000-atom cells-only WCA system over its full 1000 steps: momentum
    and energy conservation (the trajectory itself is chaotic at that length).

Tolerances as in the small-size parity tests: 1e-12 (FP64) and 1e-5
(FP32-mixed) on forces per atom against S_i, normwise and on energies.
"""
import numpy as np
import pytest

import oracle
from paper_2003_14061_amd import inputs
from paper_2003_14061_amd import md

from gpu_helpers import (WCA, check_cells, compare_lists, force_errors, min_image, pair,
                         state)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
STEPS = {"lj_2048k": 30, "wca_256k": 60}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["lj_2048k", "wca_256k"])
def test_full_size_state_matches_the_oracle_on_samples(name, precision):
    w = inputs.preset(name).materialize()
    sim = md.Simulation(w.pos, w.vel, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt,
                        precision=precision)
    sim.prepare()
    sim.step(STEPS[name])
    # cells and list at the current positions (the build folds them into the box)
    sim.build_cells()
    sim.build_neighbors()
    sim.forces()
    obs = sim.reduce()
    st = sim.state()
    pos, vel, n = st["pos"], st["vel"], w.n
    assert pos.min() >= 0.0 and pos.max() < w.L
    s = oracle.make_sys(n, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt,
                        nl_cap=sim.grid.nl_capacity)
    nc, cells = check_cells(sim, s, pos)
    o_cnt, o_nl, longest = oracle.build_nl(s, nc, pos, cells)
    assert longest <= sim.grid.nl_capacity
    cnt, nl = sim.neighbor_list()
    ids = sim.ids()
    # every list of every atom, entry by entry in list order
    compare_lists(ids, cnt, nl, o_cnt, o_nl)
    del nl
    assert obs["max_nl"] == int(o_cnt.max())
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(n, 2000, replace=False)).astype(np.int32)
    # forces of the sample against brute force over all atoms
    ref = oracle.forces_sample(s, pos, idx)
    per_atom, normwise = force_errors(st["f"][idx], ref)
    assert per_atom <= TOL[precision] and normwise <= TOL[precision], (per_atom, normwise)
    # totals against the oracle's full-list pass
    full = oracle.forces_nl(s, pos, o_cnt, o_nl)
    assert abs(obs["U"] - full["u"].sum()) <= TOL[precision] * np.abs(full["u"]).sum()
    assert obs["W"] == pytest.approx(full["w"].sum(), rel=TOL[precision] * 10, abs=1e-9)
    assert obs["K"] == pytest.approx(oracle.kinetic(s, vel), rel=1e-13)
    assert np.allclose(obs["P"], oracle.momentum(s, vel), atol=1e-9)
    assert obs["flags"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_ensemble_matches_the_oracle(precision):
    reps = inputs.ensemble(64, seed=4)
    systems = [dict(pos=r.pos, vel=r.vel, L=r.L, r_cut=r.r_cut, dt=r.dt, skin=r.skin)
               for r in reps]
    b = md.Batch(systems, precision=precision)
    b.set_tuning(force_lanes=2, force_block=256)
    b.prepare()
    steps = 20
    b.run(steps, record_every=1, graph=True)
    b.synchronize()
    tol = {"fp64": 1e-10, "fp32": 1e-5}[precision]
    for r, w in enumerate(reps):
        s = oracle.make_sys(w.n, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt)
        p_ref, v_ref, _, o_ref, _ = oracle.run(s, w.pos, w.vel, steps)
        st, h = b.state(r), b.history(r)
        e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
        assert np.max(np.abs(h["U"] - o_ref["U"])) <= tol * e_scale, r
        assert np.max(np.abs(h["K"] - o_ref["K"])) <= tol * e_scale, r
        assert np.abs(min_image(st["pos"] - p_ref, w.L)).max() < tol, r
        assert b.reduce(r)["flags"] == 0, r


def test_cells_only_wca_4000_conserves_over_1000_steps():
    w = inputs.preset("wca_4000").materialize()
    sim = md.Simulation(w.pos, w.vel, w.L, r_cut=w.r_cut, dt=w.dt, neighbor_list=False)
    sim.prepare()
    sim.step(1000, record_every=10)
    h = sim.history()
    assert len(h) == 100
    E = (h["U"] + h["K"]) / w.n
    assert np.abs(h["P"]).max() < 1e-10
    assert E.max() - E.min() < 3e-3
    # the first steps follow the oracle (the short-run tests check this closely)
    s = oracle.make_sys(w.n, w.L, r_cut=w.r_cut, dt=w.dt, use_nl=False)
    _, _, _, o_ref, _ = oracle.run(s, w.pos, w.vel, 10)
    assert h["U"][0] == pytest.approx(o_ref["U"][9], rel=1e-10, abs=1e-10)


def test_fp32_mixed_error_per_observable_on_the_lj_2048k_state(capsys):
    # The state of a 30-step FP64 run of the 2.048M-atom LJ system; the
    # FP32-mixed force pass on it against the FP64 oracle over every atom:
    # forces (per atom against S_i, and normwise), U, W, K, T and pressure.
    w = inputs.preset("lj_2048k").materialize()
    run = md.Simulation(w.pos, w.vel, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt)
    run.prepare()
    run.step(STEPS["lj_2048k"])
    st = run.state()
    del run
    pos = np.mod(st["pos"], w.L)
    pos[pos >= w.L] = 0.0
    vel = st["vel"]
    sim = md.Simulation(pos, vel, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt, precision="fp32")
    sim.prepare()
    obs = sim.reduce()
    f32 = sim.state()["f"]
    s = oracle.make_sys(w.n, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt,
                        nl_cap=sim.grid.nl_capacity)
    del sim
    nc = oracle.cells_per_side(w.L, w.r_cut + w.skin)
    cells = oracle.build_cells(s, nc, pos)
    cnt, nl, _ = oracle.build_nl(s, nc, pos, cells)
    ref = oracle.forces_nl(s, pos, cnt, nl)
    per_atom, normwise = force_errors(f32, ref)
    U, W = ref["u"].sum(), ref["w"].sum()
    K = oracle.kinetic(s, vel)
    V = w.L ** 3
    T = 2.0 * K / (3.0 * (w.n - 1))
    P = (2.0 * K + W) / (3.0 * V)
    err = {"F_per_atom": per_atom, "F_normwise": normwise,
           "U": abs(obs["U"] - U) / abs(U), "W": abs(obs["W"] - W) / abs(W),
           "K": abs(obs["K"] - K) / K, "T": abs(obs["T"] - T) / T,
           # relative to the scale of its two terms (P itself can be near 0)
           "pressure": abs(obs["pressure"] - P) / ((2.0 * K + abs(W)) / (3.0 * V))}
    with capsys.disabled():
        print("\nFP32-mixed vs FP64 oracle, lj_2048k state after 30 steps: " +
              ", ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    for k, v in err.items():
        assert v <= TOL["fp32"], (k, v)
    assert err["K"] <= 1e-13 and err["T"] <= 1e-13  # integration and K stay FP64


def test_cell_wave_lists_past_24_bit_rows_match_the_oracle():
    """2 200 000 WCA atoms: eight times the padded count passes 2^24, so the
    cell-wave build (forced here; the automatic choice at 2.3 atoms per cell is
    a lane per atom) stores its hits through 64-bit addresses in the list
    build's full kernel.  Every list of every atom, entry by entry in list
    order, against the oracle's."""
    n = 2_200_000
    L, pos, vel = state(n, 0.8, 11, jitter=0.05)
    sim, s = pair(pos, vel, L, r_cut=WCA)
    sim.set_tuning(nl_method=md.MD_NL_CELL_WAVES)
    assert 8 * sim.grid.n_pad >= 1 << 24
    sim.build_cells()
    nc, (o_of, o_start, o_atoms) = check_cells(sim, s, pos)
    sim.build_neighbors()
    o_cnt, o_nl, longest = oracle.build_nl(s, nc, pos, (o_of, o_start, o_atoms))
    assert longest <= sim.grid.nl_capacity
    cnt, nl = sim.neighbor_list()
    compare_lists(sim.ids(), cnt, nl, o_cnt, o_nl)
    sim.forces()
    assert sim.reduce()["flags"] == 0

