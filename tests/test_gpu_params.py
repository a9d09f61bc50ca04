"""GPU parity away from unit parameters: eps, sigma and the mass set away
from 1, and the potential cut without the energy shift.

The pair force of step F1 (section 2.3) and its energy and virial depend on
eps and sigma; the kicks and the kinetic energy and momentum depend on the
mass; the shift only on the potential.  With eps = sigma = m = 1 a mistake in
any of these factors cancels, so every contract of the unit-parameter
parity tests is repeated here at eps = 1.3, sigma = 0.9, m = 2:

  cells and neighbor list   bit-exact in atom-id space, entry order included;
  forces                    per atom |dF_i| <= tol S_i and normwise <= tol,
                            tol = 1e-12 (FP64) or 1e-5 (FP32-mixed);
  U, W, K, P, T, pressure   against the oracle's sums on the same state;
  40 leapfrog steps         per-step U, K, W and the final state against the
                            oracle's run, with the same rebuild steps.

The cutoff is given in sigma units (2.5 sigma or 2^(1/6) sigma), the density
as rho sigma^3, the skin as 0.3 sigma, and the velocities are drawn at
k T = eps for mass m.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2003_14061_amd import inputs
from paper_2003_14061_amd import md

from gpu_helpers import (WCA, check_cells, check_nl, energy_error, force_errors, min_image,
                         oracle_cells, pair)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
EPS, SIGMA, MASS = 1.3, 0.9, 2.0

CASES = {
    # name: (n, rho sigma^3, r_cut / sigma, shifted, neighbor list, jitter / sigma)
    "lj_shifted": (32000, 0.8, 2.5, True, True, 0.05),
    "lj_trunc": (32000, 0.8, 2.5, False, True, 0.05),
    "wca": (13500, 0.8, WCA, True, True, 0.08),
    "lj_trunc_random": (6000, 0.5, 2.5, False, True, None),
    "wca_cells": (4000, 0.8, WCA, True, False, 0.06),
    "lj_trunc_cells": (4000, 0.8442, 2.5, False, False, 0.05),
}


def system(name, seed=31, run=False):
    n, rho_s3, rc, shifted, nl, jit = CASES[name]
    if run and jit is not None:
        # Gaussian jitter of 0.08 sigma over 13 500 atoms leaves pairs at
        # 0.55 sigma, whose forces make a 40-step run blow up (in the oracle
        # as well); runs start from at most 0.05 sigma
        jit = min(jit, 0.05)
    rng = np.random.default_rng(seed)
    L = inputs.box_length(n, rho_s3 / SIGMA ** 3)
    if jit is None:
        pos = rng.uniform(0.0, L, (n, 3))
        pos[pos >= L] = 0.0
    else:
        pos = inputs.jitter(inputs.fcc_positions(n, L, rng), L, jit * SIGMA, rng)
    vel = inputs.thermal_velocities(n, EPS, rng, mass=MASS)
    kw = dict(r_cut=rc * SIGMA, skin=0.3 * SIGMA, dt=0.005, nl=nl, shifted=shifted, eps=EPS,
              sigma=SIGMA, mass=MASS)
    return L, pos, vel, kw


def reference(sim, s, pos):
    nc, cells = oracle_cells(sim, s, pos)
    if s.use_nl:
        cnt, nl, _ = oracle.build_nl(s, nc, pos, cells)
        return oracle.forces_nl(s, pos, cnt, nl)
    return oracle.forces_cells(s, nc, pos, cells)


def check_observables(obs, ref, s, vel, tol):
    U = ref["u"].sum()
    W = ref["w"].sum()
    K = oracle.kinetic(s, vel)
    P = oracle.momentum(s, vel)
    V = s.L ** 3
    assert energy_error(obs["U"], ref) <= tol
    assert abs(obs["W"] - W) <= tol * max(np.abs(ref["w"]).sum(), 1e-300)
    assert obs["K"] == pytest.approx(K, rel=1e-13)
    assert np.allclose(obs["P"], P, rtol=0, atol=1e-10 * MASS * np.abs(vel).sum())
    assert obs["T"] == pytest.approx(2.0 * K / (3.0 * (s.n - 1)), rel=1e-13)
    p_ref = (2.0 * K + W) / (3.0 * V)
    assert abs(obs["pressure"] - p_ref) <= tol * (2.0 * K + np.abs(ref["w"]).sum()) / (3.0 * V)


@pytest.mark.parametrize("name", list(CASES))
def test_cells_list_forces_and_observables_fp64(name):
    L, pos, vel, kw = system(name)
    sim, s = pair(pos, vel, L, **kw)
    sim.build_cells()
    nc, cells = check_cells(sim, s, pos)
    if s.use_nl:
        sim.build_neighbors()
        o_cnt, o_nl = check_nl(sim, s, pos, cells)
        ref = oracle.forces_nl(s, pos, o_cnt, o_nl)
    else:
        ref = oracle.forces_cells(s, nc, pos, cells)
    sim.forces()
    obs = sim.reduce()
    per_atom, normwise = force_errors(sim.state()["f"], ref)
    assert per_atom <= TOL["fp64"] and normwise <= TOL["fp64"], (per_atom, normwise)
    check_observables(obs, ref, s, vel, TOL["fp64"])
    if not kw["shifted"] and s.use_nl:
        # the unshifted energy exceeds the shifted one by u(r_cut) per pair
        # inside the cutoff
        s_sh = oracle.make_sys(s.n, L, r_cut=s.r_cut, skin=s.skin, dt=s.dt, eps=EPS,
                               sigma=SIGMA, mass=MASS, nl_cap=s.nl_cap)
        sh = oracle.forces_nl(s_sh, pos, o_cnt, o_nl)
        pairs = sum(int(np.count_nonzero(
            (lambda d: (d * d).sum(1))(min_image(pos[o_nl[i, :o_cnt[i]]] - pos[i], L))
            < s.r_cut ** 2)) for i in range(s.n)) // 2
        # both totals carry rounding of order tol * sum |u_i|; with random
        # positions close pairs make that scale large, so the difference is
        # compared at that scale rather than relative to itself
        scale = np.abs(sh["u"]).sum() + abs(pairs * oracle.shift(s_sh))
        assert abs(obs["U"] - sh["u"].sum() - pairs * oracle.shift(s_sh)) <= max(
            1e-9 * abs(pairs * oracle.shift(s_sh)), 2 * TOL["fp64"] * scale)


@pytest.mark.parametrize("name", list(CASES))
def test_forces_and_observables_fp32_mixed(name):
    L, pos, vel, kw = system(name)
    sim, s = pair(pos, vel, L, precision="fp32", **kw)
    sim.prepare()
    obs = sim.reduce()
    ref = reference(sim, s, pos)
    per_atom, normwise = force_errors(sim.state()["f"], ref)
    assert per_atom <= TOL["fp32"] and normwise <= TOL["fp32"], (per_atom, normwise)
    check_observables(obs, ref, s, vel, TOL["fp32"])


def run_pair(name, precision, steps=40):
    L, pos, vel, kw = system(name, seed=37, run=True)
    sim, s = pair(pos, vel, L, precision=precision, **kw)
    sim.prepare()
    sim.step(steps, record_every=1)
    hist = sim.history()
    obs = sim.reduce()
    st = sim.state()
    p_ref, v_ref, _, o_ref, nreb = oracle.run(s, pos, vel, steps)
    assert len(hist) == steps and obs["step"] == steps
    return s, hist, obs, st, p_ref, v_ref, o_ref, nreb


@pytest.mark.parametrize("name", ["lj_shifted", "lj_trunc", "wca", "wca_cells",
                                  "lj_trunc_cells"])
def test_short_run_fp64(name):
    s, hist, obs, st, p_ref, v_ref, o_ref, nreb = run_pair(name, "fp64")
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(hist["U"] - o_ref["U"])) <= 1e-10 * e_scale
    assert np.max(np.abs(hist["K"] - o_ref["K"])) <= 1e-10 * e_scale
    assert np.max(np.abs(hist["W"] - o_ref["W"])) <= 1e-9 * max(np.abs(o_ref["W"]).max(), 1)
    assert np.allclose(hist["P"], o_ref["P"], rtol=0, atol=1e-9)
    assert np.abs(min_image(st["pos"] - p_ref, s.L)).max() < 1e-10
    assert np.abs(st["vel"] - v_ref).max() < 1e-9
    if s.use_nl:
        thr = (0.5 * s.skin) ** 2
        near = np.abs(o_ref["dmax2"] - thr) < 1e-9 * thr
        assert not np.any((hist["rebuilt"] != o_ref["rebuilt"]) & ~near)
        assert obs["n_rebuilds"] == nreb


@pytest.mark.parametrize("name", ["lj_shifted", "lj_trunc", "wca_cells"])
def test_short_run_fp32_mixed(name):
    s, hist, obs, st, p_ref, v_ref, o_ref, nreb = run_pair(name, "fp32")
    e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
    assert np.max(np.abs(hist["U"] - o_ref["U"])) <= 1e-5 * e_scale
    assert np.max(np.abs(hist["K"] - o_ref["K"])) <= 1e-5 * e_scale
    assert np.abs(min_image(st["pos"] - p_ref, s.L)).max() < 1e-5


def test_mass_scales_the_trajectory_time():
    # the same forces at mass m and time step dt give the positions of mass 1
    # at time step dt / sqrt(m) with velocities scaled by sqrt(m): the leapfrog
    # map is the same in exact arithmetic, so the two GPU runs agree to
    # rounding
    L, pos, vel, kw = system("lj_shifted", seed=41)
    out = []
    for m, dt, v in ((MASS, 0.005, vel), (1.0, 0.005 / math.sqrt(MASS), vel * math.sqrt(MASS))):
        kw2 = dict(kw, mass=m, dt=dt)
        sim, s = pair(pos, v, L, **kw2)
        sim.prepare()
        sim.step(20)
        out.append(sim.state()["pos"])
    assert np.abs(min_image(out[0] - out[1], L)).max() < 1e-9


@pytest.mark.parametrize("name", ["lj_shifted", "lj_trunc"])
def test_third_law_and_layer_pipelines(name):
    L, pos, vel, kw = system(name)
    for extra in (dict(newton3=True), dict(pipeline="layers", reorder=False)):
        sim, s = pair(pos, vel, L, **kw, **extra)
        sim.prepare()
        obs = sim.reduce()
        ref = reference(sim, s, pos)
        per_atom, normwise = force_errors(sim.state()["f"], ref)
        assert per_atom <= TOL["fp64"] and normwise <= TOL["fp64"], (extra, per_atom)
        check_observables(obs, ref, s, vel, TOL["fp64"])


def test_batch_of_replicas_with_their_own_parameters():
    # each replica carries its own eps, sigma, mass and potential form
    rng = np.random.default_rng(43)
    specs = [(1.3, 0.9, 2.0, True, 2.5), (0.7, 1.1, 0.5, False, 2.5), (1.0, 1.0, 1.0, True, WCA),
             (2.0, 0.8, 3.0, True, WCA)]
    systems, refs = [], []
    for k, (eps, sig, m, shifted, rc) in enumerate(specs):
        n = [4000, 6912, 3000, 5000][k]
        L = inputs.box_length(n, 0.8 / sig ** 3)
        pos = inputs.jitter(inputs.fcc_positions(n, L, rng), L, 0.05 * sig, rng)
        vel = inputs.thermal_velocities(n, eps, rng, mass=m)
        systems.append(dict(pos=pos, vel=vel, L=L, r_cut=rc * sig, dt=0.005, skin=0.3 * sig,
                            eps=eps, sigma=sig, mass=m, shifted=shifted))
        refs.append(oracle.make_sys(n, L, r_cut=rc * sig, skin=0.3 * sig, dt=0.005, eps=eps,
                                    sigma=sig, mass=m, potential=oracle.LJ_SHIFTED if shifted
                                    else oracle.LJ_TRUNC))
    steps = 30
    for precision, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        b = md.Batch(systems, precision=precision)
        b.prepare()
        b.run(steps, record_every=1, graph=True)
        b.synchronize()
        for r, (sy, s) in enumerate(zip(systems, refs)):
            p_ref, _, _, o_ref, _ = oracle.run(s, sy["pos"], sy["vel"], steps)
            h, st = b.history(r), b.state(r)
            e_scale = np.abs(o_ref["U"]).max() + np.abs(o_ref["K"]).max()
            assert np.max(np.abs(h["U"] - o_ref["U"])) <= tol * e_scale, (precision, r)
            assert np.max(np.abs(h["K"] - o_ref["K"])) <= tol * e_scale, (precision, r)
            assert np.abs(min_image(st["pos"] - p_ref, sy["L"])).max() < tol, (precision, r)
            assert b.reduce(r)["flags"] == 0
