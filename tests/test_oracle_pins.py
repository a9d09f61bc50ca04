"""Pins for the CPU oracle: closed forms, lattice sums, brute force, invariants.

Each test checks the oracle against something the oracle does not compute
itself: hand-derived values of the 12-6 potential, FCC lattice shell sums,
an independent numpy all-pairs enumeration, finite differences, the
harmonic-dimer frequency of the leapfrog map, and conservation laws.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2003_14061_amd import inputs

WCA = 2.0 ** (1.0 / 6.0)


def lj_sys(n=2, L=20.0, r_cut=2.5, shifted=False, **kw):
    return oracle.make_sys(n, L, r_cut=r_cut, potential=oracle.LJ_SHIFTED if shifted else oracle.LJ_TRUNC,
                           **kw)


# ---------------------------------------------------------------- potential

def test_pair_at_sigma_is_zero_energy_and_24eps_force():
    s = lj_sys()
    u, fr = oracle.pair(s, 1.0)
    assert u == 0.0
    # |F| = fr * r with r = sigma = 1: 48 (1 - 1/2) = 24
    assert fr == pytest.approx(24.0, rel=1e-15)


def test_pair_error_scale_hand_values():
    s = lj_sys()
    # 48 (sr^12 + sr^6 / 2) / r: at r = sigma, 48 * 1.5; at the minimum, 24 / 2^(1/6)
    assert oracle.pair_scale(s, 1.0) == pytest.approx(72.0, rel=1e-15)
    assert oracle.pair_scale(s, WCA * WCA) == pytest.approx(24.0 / WCA, rel=1e-14)
    assert oracle.pair_scale(s, 6.25) == 0.0
    _, fr = oracle.pair(s, 1.0)
    assert oracle.pair_scale(s, 1.0) >= abs(fr)


def test_pair_at_minimum():
    s = lj_sys()
    u, fr = oracle.pair(s, WCA * WCA)
    assert u == pytest.approx(-1.0, rel=1e-14)
    assert abs(fr) < 1e-13


def test_pair_at_lj_cutoff_hand_values():
    # (1/2.5)^6 = 0.004096, (1/2.5)^12 = 1.6777216e-5
    s = lj_sys()
    r = 2.5 * (1 - 1e-15)
    u, fr = oracle.pair(s, r * r)
    assert u == pytest.approx(4 * (1.6777216e-5 - 0.004096), rel=1e-12)        # -0.016316891136
    assert fr * r == pytest.approx(19.2 * (1.6777216e-5 - 0.002048), rel=1e-12)  # -0.0389994774528
    # shifted form: energy continuous at the cutoff, force unchanged
    s2 = lj_sys(shifted=True)
    u2, fr2 = oracle.pair(s2, r * r)
    assert abs(u2) < 1e-12
    assert fr2 == fr
    assert oracle.shift(s2) == pytest.approx(-0.016316891136, rel=1e-12)


@pytest.mark.parametrize("shifted", [False, True])
def test_pair_zero_at_and_beyond_cutoff(shifted):
    s = lj_sys(shifted=shifted)
    for r2 in [6.25, 6.25 * (1 + 1e-15), 7.0, 100.0, 1e300]:
        u, fr = oracle.pair(s, r2)
        assert u == 0.0 and fr == 0.0


def test_wca_shift_makes_energy_vanish_at_cutoff_and_is_eps_at_contact():
    s = oracle.make_sys(2, 20.0, r_cut=WCA, potential=oracle.LJ_SHIFTED)
    u, fr = oracle.pair(s, (WCA * (1 - 1e-12)) ** 2)
    assert abs(u) < 1e-10
    u1, _ = oracle.pair(s, 1.0)
    assert u1 == pytest.approx(1.0, rel=1e-13)  # 0 - (-eps)


def test_pair_scaling_in_eps_and_sigma():
    eps, sig = 1.7, 0.9
    s = oracle.make_sys(2, 20.0, r_cut=2.5 * sig, eps=eps, sigma=sig, potential=oracle.LJ_TRUNC)
    s1 = lj_sys()
    for r in [0.95, 1.1, 1.3, 1.8, 2.2]:
        u, fr = oracle.pair(s, (r * sig) ** 2)
        u1, fr1 = oracle.pair(s1, r * r)
        assert u == pytest.approx(eps * u1, rel=1e-13)
        # F = -du/dr scales as eps/sigma; fr = F/r scales as eps/sigma^2
        assert fr == pytest.approx(eps * fr1 / sig ** 2, rel=1e-13)


def test_force_is_minus_energy_derivative():
    s = lj_sys()
    for r in np.linspace(0.9, 2.45, 23):
        h = 1e-6
        up, _ = oracle.pair(s, (r + h) ** 2)
        um, _ = oracle.pair(s, (r - h) ** 2)
        _, fr = oracle.pair(s, r * r)
        assert fr * r == pytest.approx(-(up - um) / (2 * h), rel=1e-7, abs=1e-9)


# ---------------------------------------------------------------- box

def test_minimum_image_is_odd_and_bounded():
    rng = np.random.default_rng(0)
    L = 13.7
    for d in rng.uniform(-L, L, 2000):
        m = oracle.minimg(d, L)
        assert -L / 2 <= m <= L / 2
        assert oracle.minimg(-d, L) == -m
        assert abs(math.remainder(d - m, L)) < 1e-12


def test_wrap_edges():
    L = 10.0
    assert oracle.wrap(L, L) == 0.0
    assert oracle.wrap(-1e-18, L) == 0.0  # L - tiny rounds to L, mapped to 0
    assert oracle.wrap(-0.5, L) == 9.5
    assert oracle.wrap(10.25, L) == 0.25
    assert oracle.wrap(3.0, L) == 3.0
    x = np.nextafter(L, 0)
    assert oracle.wrap(x, L) == x
    for v in np.random.default_rng(1).uniform(-L, 2 * L, 1000):
        w = oracle.wrap(v, L)
        assert 0.0 <= w < L


# ---------------------------------------------------------------- cells (N1-N4)

def test_cells_contain_their_atoms_and_are_id_ordered():
    rng = np.random.default_rng(2)
    L, n = 11.3, 3000
    pos = rng.uniform(0, L, (n, 3))
    pos[:5] = [[0, 0, 0], [np.nextafter(L, 0)] * 3, [L / 2] * 3, [1e-300, 0, 0], [0, np.nextafter(L, 0), 0]]
    s = oracle.make_sys(n, L, r_cut=2.5, skin=0.3)
    nc = oracle.cells_per_side(L, 2.8)
    assert nc == 4
    cell_of, cell_start, cell_atoms = oracle.build_cells(s, nc, pos)
    w = L / nc
    cx = cell_of % nc
    cy = (cell_of // nc) % nc
    cz = cell_of // (nc * nc)
    for c, p in ((cx, pos[:, 0]), (cy, pos[:, 1]), (cz, pos[:, 2])):
        assert np.all(c * w <= p * (1 + 1e-14) + 1e-14)
        assert np.all(p < (c + 1) * w + 1e-12)
    assert cell_start[0] == 0 and cell_start[-1] == n
    assert np.all(np.diff(cell_start) >= 0)
    assert sorted(cell_atoms.tolist()) == list(range(n))
    for c in range(nc ** 3):
        mem = cell_atoms[cell_start[c]:cell_start[c + 1]]
        assert np.all(np.diff(mem) > 0)
        assert np.all(cell_of[mem] == c)


# ---------------------------------------------------------------- neighbor list (N5)

def brute_pairs(pos, L, r):
    """Independent numpy all-pairs set of (i, j), i != j, minimum image, d < r."""
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    d2 = (d * d).sum(-1)
    np.fill_diagonal(d2, np.inf)
    return d2 < r * r, d2


def _stencil_rank(nc, ci, cj):
    """Position (0..26) of cell cj in the 27-cell visiting order around ci."""
    def split(c):
        return c % nc, (c // nc) % nc, c // (nc * nc)
    ax, ay, az = split(ci)
    bx, by, bz = split(cj)
    def off(a, b):
        o = (b - a) % nc
        return {0: 0, 1: 1, nc - 1: -1}[o]
    return (off(az, bz) + 1) * 9 + (off(ay, by) + 1) * 3 + (off(ax, bx) + 1)


@pytest.mark.parametrize("case", ["wca108", "wca_jit", "lj864", "lj_random"])
def test_nl_equals_bruteforce_and_is_canonical(case):
    rng = np.random.default_rng(7)
    if case == "wca108":
        n, rho, rc = 108, 0.8, WCA
        L = inputs.box_length(n, rho)
        pos = inputs.fcc_positions(n, L)
    elif case == "wca_jit":
        n, rho, rc = 500, 0.8, WCA
        L = inputs.box_length(n, rho)
        pos = inputs.jitter(inputs.fcc_positions(n, L), L, 0.1, rng)
    elif case == "lj864":
        n, rho, rc = 864, 0.8442, 2.5
        L = inputs.box_length(n, rho)
        pos = inputs.jitter(inputs.fcc_positions(n, L), L, 0.05, rng)
    else:
        n, rho, rc = 700, 0.5, 2.5
        L = inputs.box_length(n, rho)
        pos = rng.uniform(0, L, (n, 3))
    skin = 0.3
    s = oracle.make_sys(n, L, r_cut=rc, skin=skin)
    nc = oracle.cells_per_side(L, rc + skin)
    assert nc >= 3
    cells = oracle.build_cells(s, nc, pos)
    cnt, nl, longest = oracle.build_nl(s, nc, pos, cells)
    assert longest <= s.nl_cap
    inside, _ = brute_pairs(pos, L, rc + skin)
    cell_of = cells[0]
    for i in range(n):
        lst = nl[i, :cnt[i]]
        assert set(lst.tolist()) == set(np.nonzero(inside[i])[0].tolist())
        assert len(set(lst.tolist())) == len(lst)
        key = [(_stencil_rank(nc, cell_of[i], cell_of[j]), j) for j in lst]
        assert key == sorted(key)
    # symmetry
    m = np.zeros((n, n), bool)
    for i in range(n):
        m[i, nl[i, :cnt[i]]] = True
    assert np.array_equal(m, m.T)


# ---------------------------------------------------------------- forces (F1)

def numpy_forces(pos, L, rc, shift):
    """Independent vectorized all-pairs 12-6 forces and energy (eps=sigma=1)."""
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r2 = (d * d).sum(-1)
    np.fill_diagonal(r2, np.inf)
    m = r2 < rc * rc
    inv6 = np.where(m, 1.0 / r2 ** 3, 0.0)
    fr = np.where(m, 48 * inv6 * (inv6 - 0.5) / r2, 0.0)
    f = (fr[:, :, None] * d).sum(1)
    u = np.where(m, 4 * inv6 * (inv6 - 1) - shift, 0.0).sum() / 2
    w = (fr * np.where(m, r2, 0.0)).sum() / 2
    return f, u, w


@pytest.mark.parametrize("shifted", [False, True])
def test_forces_three_ways_agree(shifted):
    rng = np.random.default_rng(11)
    n, rho, rc, skin = 864, 0.8442, 2.5, 0.3
    L = inputs.box_length(n, rho)
    pos = inputs.jitter(inputs.fcc_positions(n, L), L, 0.08, rng)
    s = oracle.make_sys(n, L, r_cut=rc, skin=skin,
                        potential=oracle.LJ_SHIFTED if shifted else oracle.LJ_TRUNC)
    nc = oracle.cells_per_side(L, rc + skin)
    cells = oracle.build_cells(s, nc, pos)
    cnt, nl, _ = oracle.build_nl(s, nc, pos, cells)
    a = oracle.forces_nl(s, pos, cnt, nl)
    b = oracle.forces_allpairs(s, pos)
    s0 = oracle.make_sys(n, L, r_cut=rc, skin=0.0, use_nl=False,
                         potential=oracle.LJ_SHIFTED if shifted else oracle.LJ_TRUNC)
    nc0 = oracle.cells_per_side(L, rc)
    c = oracle.forces_cells(s0, nc0, pos, oracle.build_cells(s0, nc0, pos))
    f_np, u_np, w_np = numpy_forces(pos, L, rc, oracle.shift(s))
    scale = a["s"][:, None] + 1e-300
    for other in (b, c):
        assert np.all(np.abs(a["f"] - other["f"]) <= 1e-13 * scale)
        assert a["u"].sum() == pytest.approx(other["u"].sum(), rel=1e-13)
    assert np.all(np.abs(a["f"] - f_np) <= 1e-12 * scale)
    assert a["u"].sum() == pytest.approx(u_np, rel=1e-12)
    assert a["w"].sum() == pytest.approx(w_np, rel=1e-12)
    # Newton's third law holds pairwise, so the total force vanishes
    ftot = a["f"].sum(0)
    assert np.all(np.abs(ftot) <= 1e-12 * np.sqrt(n) * np.sqrt((a["f"] ** 2).mean()))
    # the sampled brute force agrees with the full one
    idx = np.array([0, 5, 77, n - 1], np.int32)
    smp = oracle.forces_sample(s, pos, idx)
    assert np.array_equal(smp["f"], b["f"][idx])


def _fcc_shells_energy(rho, rc):
    """Per-atom energy of a perfect FCC lattice by summing its coordination
    shells: r_k = a sqrt(k/2) with the shell multiplicities of FCC."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    mult = {1: 12, 2: 6, 3: 24, 4: 12, 5: 24, 6: 8, 7: 48, 8: 6}
    u, npair = 0.0, 0
    for k, m in mult.items():
        r = a * math.sqrt(k / 2.0)
        if r < rc:
            u += 0.5 * m * 4.0 * (r ** -12 - r ** -6)
            npair += m
    return u, npair


@pytest.mark.parametrize("rho,expect_u", [(0.8442, -6.773368053), (0.8, -6.364746502)])
def test_fcc_lattice_energy_matches_shell_sum(rho, expect_u):
    u_shell, npair = _fcc_shells_energy(rho, 2.5)
    assert npair == 54
    assert u_shell == pytest.approx(expect_u, abs=2e-9)
    n = 4 * 6 ** 3
    L = inputs.box_length(n, rho)
    pos = inputs.fcc_positions(n, L)
    for shifted in (False, True):
        s = oracle.make_sys(n, L, r_cut=2.5, skin=0.3,
                            potential=oracle.LJ_SHIFTED if shifted else oracle.LJ_TRUNC)
        nc = oracle.cells_per_side(L, 2.8)
        cells = oracle.build_cells(s, nc, pos)
        cnt, nl, _ = oracle.build_nl(s, nc, pos, cells)
        r = oracle.forces_nl(s, pos, cnt, nl)
        expect = u_shell - (0.5 * npair * oracle.shift(s) if shifted else 0.0)
        assert r["u"].sum() / n == pytest.approx(expect, rel=1e-12)
        # every atom sits at a centre of symmetry: forces cancel
        assert np.all(np.linalg.norm(r["f"], axis=1) <= 1e-12 * r["s"])


def test_wca_fcc_lattice_has_no_contacts():
    # at rho = 0.8 the FCC nearest-neighbour distance exceeds 2^(1/6)
    n = 4000
    L = inputs.box_length(n, 0.8)
    pos = inputs.fcc_positions(n, L)
    s = oracle.make_sys(n, L, r_cut=WCA, skin=0.0, use_nl=False)
    nc = oracle.cells_per_side(L, WCA)
    r = oracle.forces_cells(s, nc, pos, oracle.build_cells(s, nc, pos))
    assert np.all(r["f"] == 0.0) and np.all(r["u"] == 0.0)


def test_virial_is_minus_volume_derivative_of_energy():
    rng = np.random.default_rng(3)
    n, rho = 500, 0.7
    L = inputs.box_length(n, rho)
    pos = inputs.jitter(inputs.fcc_positions(n, L, rng), L, 0.1, rng)

    def energy(lam):
        s = oracle.make_sys(n, L * lam, r_cut=2.5, potential=oracle.LJ_TRUNC)
        return oracle.forces_allpairs(s, pos * lam)["u"].sum()

    s = oracle.make_sys(n, L, r_cut=2.5, potential=oracle.LJ_TRUNC)
    w = oracle.forces_allpairs(s, pos)["w"].sum()
    h = 1e-6
    dudl = (energy(1 + h) - energy(1 - h)) / (2 * h)
    assert w == pytest.approx(-dudl, rel=1e-6)


# ---------------------------------------------------------------- integrator

def test_dimer_frequency_matches_leapfrog_map():
    # two atoms near the LJ minimum: u''(2^(1/6)) = 72 / 2^(1/3); reduced mass 1/2
    rmin = WCA
    omega = math.sqrt(72.0 / 2 ** (1 / 3) / 0.5)
    dt = 0.02
    omega_lf = (2.0 / dt) * math.asin(omega * dt / 2.0)
    L = 12.0
    amp = 1e-4
    pos = np.array([[5.0, 6.0, 6.0], [5.0 + rmin + amp, 6.0, 6.0]])
    vel = np.zeros((2, 3))
    s = oracle.make_sys(2, L, r_cut=2.5, skin=0.3, dt=dt, potential=oracle.LJ_SHIFTED)
    steps = 4000
    xs = []
    p, v = pos, vel
    for _ in range(steps):
        p, v, f, obs, _ = oracle.run(s, p, v, 1)
        xs.append(p[1, 0] - p[0, 0] - rmin)
    xs = np.array(xs)
    # upward zero crossings, linearly interpolated
    t = np.arange(1, steps + 1) * dt
    k = np.nonzero((xs[:-1] < 0) & (xs[1:] >= 0))[0]
    tc = t[k] - xs[k] * (t[k + 1] - t[k]) / (xs[k + 1] - xs[k])
    period = (tc[-1] - tc[0]) / (len(tc) - 1)
    w_meas = 2 * math.pi / period
    assert w_meas == pytest.approx(omega_lf, rel=2e-5)
    assert abs(w_meas / omega - 1) > 1e-3  # the leapfrog shift is resolved


def _liquid(n=500, rho=0.8, T=1.0, seed=5, rc=WCA, dt=0.005, shifted=True, melt=100):
    rng = np.random.default_rng(seed)
    L = inputs.box_length(n, rho)
    pos = inputs.jitter(inputs.fcc_positions(n, L, rng), L, 0.05, rng)
    vel = inputs.thermal_velocities(n, T, rng)
    s = oracle.make_sys(n, L, r_cut=rc, skin=0.3, dt=dt,
                        potential=oracle.LJ_SHIFTED if shifted else oracle.LJ_TRUNC)
    if melt:
        pos, vel, _, _, _ = oracle.run(s, pos, vel, melt)
    return s, pos, vel


def test_time_reversibility():
    s, pos, vel = _liquid()
    p1, v1, _, obs, nreb = oracle.run(s, pos, vel, 100)
    assert nreb >= 1
    p2, v2, _, _, _ = oracle.run(s, p1, -v1, 100)
    d = p2 - pos
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + vel).max() < 1e-9


def test_momentum_and_energy_conservation():
    s, pos, vel = _liquid()
    p, v, f, obs, nreb = oracle.run(s, pos, vel, 400)
    P = obs["P"]
    assert np.abs(P).max() < 1e-11 * s.n
    E = (obs["U"] + obs["K"]) / s.n
    assert E.max() - E.min() < 2e-3
    # the list is rebuilt, and only when the displacement rule says so
    thr = (0.5 * s.skin) ** 2
    assert np.all((obs["dmax2"] > thr) == (obs["rebuilt"] == 1))
    assert 5 <= nreb <= 200


def test_energy_fluctuation_scales_as_dt_squared():
    s, pos, vel = _liquid(melt=200)
    sd = []
    for dt in (0.004, 0.002):
        s2 = oracle.make_sys(s.n, s.L, r_cut=s.r_cut, skin=0.3, dt=dt, potential=oracle.LJ_SHIFTED)
        steps = int(round(1.0 / dt))
        _, _, _, obs, _ = oracle.run(s2, pos, vel, steps)
        E = obs["U"] + obs["K"]
        sd.append(E.std())
    assert sd[0] / sd[1] == pytest.approx(4.0, rel=0.3)


def test_list_stays_valid_along_a_run():
    # every pair inside r_cut at every step is in the list: compare the
    # list-driven run with a cells-only run (forces straight from cells of
    # width r_cut, rebuilt every step) over a short stretch
    s, pos, vel = _liquid(n=500, melt=50)
    s0 = oracle.make_sys(s.n, s.L, r_cut=s.r_cut, skin=0.0, dt=s.dt, use_nl=False,
                         potential=oracle.LJ_SHIFTED)
    pa, va, fa, oa, nreb = oracle.run(s, pos, vel, 40)
    pb, vb, fb, ob, _ = oracle.run(s0, pos, vel, 40)
    assert nreb >= 1
    d = pa - pb
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert np.allclose(oa["U"], ob["U"], rtol=1e-10, atol=1e-10)


def test_kick_and_drift_pieces():
    s = oracle.make_sys(3, 5.0, r_cut=2.5, dt=0.01, mass=2.0)
    v = np.array([[1.0, 0.0, -1.0], [0.5, 0.5, 0.5], [0, 0, 0]])
    f = np.array([[4.0, 0.0, 0.0], [0.0, -2.0, 0.0], [1, 1, 1]])
    v2 = oracle.kick(s, v, f)
    assert np.allclose(v2, v + 0.25 * 0.01 * f, rtol=0, atol=1e-17)
    p = np.array([[4.999, 0.0, 1.0], [0.0, 0.0, 0.0], [2.5, 2.5, 2.5]])
    p2 = oracle.drift(s, p, np.array([[1.0, -1.0, 0.0], [0, 0, 0], [0, 0, 0]]))
    assert p2[0, 0] == pytest.approx(0.009, abs=1e-15)
    assert p2[0, 1] == pytest.approx(4.99, abs=1e-15)


def test_half_list_holds_every_pair_once_in_canonical_order():
    # against the pinned full list: the half list of i is the full list of i
    # filtered to partners later in (cell, id) order, and every listed pair of
    # the full list appears in exactly one half list
    rng = np.random.default_rng(71)
    L = inputs.box_length(864, 0.8442)
    pos = inputs.jitter(inputs.fcc_sites(6, L), L, 0.05, rng)
    s = oracle.make_sys(len(pos), L, r_cut=2.5, skin=0.3)
    nc = oracle.cells_per_side(L, 2.8)
    cells = oracle.build_cells(s, nc, pos)
    cell_of = cells[0]
    fc, fl, _ = oracle.build_nl(s, nc, pos, cells)
    hc, hl, _ = oracle.build_nl_half(s, nc, pos, cells)
    later = lambda i, j: (cell_of[j], j) > (cell_of[i], i)
    pairs = set()
    for i in range(s.n):
        want = [j for j in fl[i, : fc[i]] if later(i, j)]
        assert list(hl[i, : hc[i]]) == want
        pairs.update((i, j) for j in want)
    full = {(min(i, j), max(i, j)) for i in range(s.n) for j in fl[i, : fc[i]]}
    assert {(min(p), max(p)) for p in pairs} == full and len(pairs) == len(full)
    # the third-law force pass gives the full-list forces and energy
    f = oracle.forces_nl(s, pos, fc, fl)
    h = oracle.forces_half(s, pos, hc, hl)
    assert np.abs(h["f"] - f["f"]).max() <= 1e-12 * f["s"].max()
    assert abs(h["u"].sum() - f["u"].sum()) <= 1e-12 * np.abs(f["u"]).sum()
    assert abs(h["w"].sum() - f["w"].sum()) <= 1e-12 * np.abs(f["w"]).sum()


def test_kinetic_energy_and_momentum_carry_the_mass():
    # hand values: K = (m/2) sum |v|^2, P = m sum v, at m = 2 and m = 0.5
    v = np.array([[1.0, 2.0, 3.0], [-1.0, 0.0, 2.0], [0.5, -0.25, 0.0]])
    sq = (1 + 4 + 9) + (1 + 0 + 4) + (0.25 + 0.0625 + 0)  # 19.3125
    for m in (2.0, 0.5):
        s = oracle.make_sys(3, 5.0, r_cut=1.0, mass=m)
        assert oracle.kinetic(s, v) == 0.5 * m * sq
        assert np.array_equal(oracle.momentum(s, v), m * np.array([0.5, 1.75, 5.0]))
    # the temperature the oracle's run reports for a box of resting atoms but
    # one moving at speed c: K = m c^2 / 2 exactly
    s = oracle.make_sys(2, 10.0, r_cut=1.0, dt=0.01, mass=3.0, use_nl=False)
    pos = np.array([[1.0, 1.0, 1.0], [6.0, 6.0, 6.0]])
    vel = np.array([[0.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    _, v_end, _, o, _ = oracle.run(s, pos, vel, 3)
    assert np.array_equal(v_end, vel)
    assert np.all(o["K"] == 0.5 * 3.0 * 4.0)
    assert np.all(o["P"][:, 1] == 6.0)
