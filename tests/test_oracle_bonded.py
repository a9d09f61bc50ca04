"""Pins of the oracle's bonded chain forces (section 4.3, item (2); readings
in oracle/md_oracle_bonded.h): closed forms of each term, forces as minus
the gradient of the energy by central differences, zero net force and
torque per chain, the bond virial as minus the derivative of the energy
under a uniform stretch, and a run with every bonded coefficient zero equal
bit for bit to the plain run."""
import math

import numpy as np
import pytest

import oracle


def sys_for(n, L=20.0):
    return oracle.make_sys(n, L, r_cut=2 ** (1 / 6), use_nl=False)


def walk_chains(n_chains, M, L, seed, bond=0.97, lo=25.0, hi=115.0):
    """Random walks with fixed bond length and bond angles (between successive
    bond vectors) drawn in [lo, hi] degrees, so no angle or dihedral is
    degenerate.  Positions folded into [0, L)."""
    rng = np.random.default_rng(seed)
    pos = []
    for _ in range(n_chains):
        r = rng.uniform(0, L, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        chain = [r.copy()]
        for _ in range(M - 1):
            if len(chain) > 1:
                # new direction at a drawn angle from the last one
                a = math.radians(rng.uniform(lo, hi))
                q = rng.normal(size=3)
                q -= q.dot(d) * d
                q /= np.linalg.norm(q)
                d = math.cos(a) * d + math.sin(a) * q
            r = r + bond * d
            chain.append(r.copy())
        pos.extend(chain)
    pos = np.mod(np.array(pos), L)
    pos[pos >= L] = 0.0
    return pos


def unwrap(pos, M, L):
    """Chain-contiguous copies of the positions (each atom moved by whole box
    lengths next to its predecessor)."""
    out = pos.copy()
    for i in range(len(pos)):
        if i % M:
            d = out[i] - out[i - 1]
            out[i] = out[i - 1] + d - L * np.round(d / L)
    return out


def test_fene_closed_form_across_the_boundary():
    L = 10.0
    s = sys_for(2, L)
    b = oracle.make_bonded(2, fene_k=30.0, fene_r0=1.5)
    pos = np.array([[0.2, 5.0, 5.0], [L - 0.9, 5.0, 5.0]])  # 1.1 apart through x = 0
    r = 1.1
    q = 1 - r * r / 2.25
    o = oracle.forces_bonded(s, b, pos)
    assert oracle.energy_bonded(s, b, pos) == pytest.approx(-0.5 * 30 * 2.25 * math.log(q), rel=1e-14)
    # atom 0 pulled toward atom 1, which sits at -x through the boundary
    assert o["f"][0] == pytest.approx([-30 / q * r, 0, 0], rel=1e-14)
    assert o["f"][1] == pytest.approx([30 / q * r, 0, 0], rel=1e-14)
    assert o["w"].sum() == pytest.approx(-30 * r * r / q, rel=1e-14)
    # at R0 the bond has no force: reported, not returned
    with pytest.raises(RuntimeError):
        oracle.forces_bonded(s, b, np.array([[1.0, 1.0, 1.0], [2.5, 1.0, 1.0]]))


@pytest.mark.parametrize("theta_deg", [0.0, 37.0, 90.0, 150.0])
def test_bend_energy_of_a_given_angle(theta_deg):
    s = sys_for(3)
    b = oracle.make_bonded(3, fene_k=0.0, bend_k=2.5)
    t = math.radians(theta_deg)
    # b1 along x; b2 at angle theta from b1
    pos = np.array([[5.0, 5.0, 5.0], [6.0, 5.0, 5.0], [6.0 + 1.2 * math.cos(t), 5.0 + 1.2 * math.sin(t), 5.0]])
    assert oracle.energy_bonded(s, b, pos) == pytest.approx(2.5 * (1 - math.cos(t)), abs=1e-14)
    f = oracle.forces_bonded(s, b, pos)["f"]
    assert np.abs(f.sum(0)).max() < 1e-13
    if theta_deg == 0.0:
        assert np.abs(f).max() < 1e-13  # a straight chain feels no bending force


@pytest.mark.parametrize("phi_deg", [0.0, 60.0, 120.0, 180.0, 250.0])
def test_dihedral_energy_of_a_given_angle(phi_deg):
    s = sys_for(4)
    c = (0.3, -1.1, 0.7, 2.0)
    b = oracle.make_bonded(4, fene_k=0.0, tors_c=c)
    p = math.radians(phi_deg)
    # middle bond along z; the end bonds perpendicular to it, phi apart (0 = cis)
    o = np.array([5.0, 5.0, 5.0])
    pos = o + np.array([[1, 0, 0], [0, 0, 0], [0, 0, 1], [math.cos(p), math.sin(p), 1]], float)
    cp = math.cos(p)
    want = sum(cm * cp ** m for m, cm in enumerate(c))
    assert oracle.energy_bonded(s, b, pos) == pytest.approx(want, abs=1e-13)
    if phi_deg in (0.0, 180.0):  # cis: sum c_m, trans: sum c_m (-1)^m
        assert want == pytest.approx(sum(cm * (1 if phi_deg == 0 else (-1) ** m)
                                         for m, cm in enumerate(c)))


def test_forces_are_minus_the_gradient():
    M, nch, L = 9, 4, 12.0
    pos = walk_chains(nch, M, L, seed=3)
    s = sys_for(len(pos), L)
    b = oracle.make_bonded(M, fene_k=30.0, fene_r0=1.5, bend_k=1.7, tors_c=(0.4, 1.3, -0.8, 0.6))
    f = oracle.forces_bonded(s, b, pos)["f"]
    h = 1e-6
    rng = np.random.default_rng(0)
    for i in rng.choice(len(pos), 12, replace=False):
        for k in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, k] += h
            p2[i, k] -= h
            g = (oracle.energy_bonded(s, b, p1) - oracle.energy_bonded(s, b, p2)) / (2 * h)
            assert -g == pytest.approx(f[i, k], rel=2e-7, abs=2e-7 * np.abs(f).max())


def test_each_term_is_on_and_off_separately():
    """A dropped term or a sign flip in one term fails here: energies add."""
    M, L = 6, 12.0
    pos = walk_chains(3, M, L, seed=5)
    s = sys_for(len(pos), L)
    parts = [oracle.make_bonded(M, fene_k=30.0), oracle.make_bonded(M, fene_k=0.0, bend_k=1.5),
             oracle.make_bonded(M, fene_k=0.0, tors_c=(0.2, -0.9, 0.4, 1.1))]
    whole = oracle.make_bonded(M, fene_k=30.0, bend_k=1.5, tors_c=(0.2, -0.9, 0.4, 1.1))
    e = [oracle.energy_bonded(s, p, pos) for p in parts]
    assert all(abs(v) > 1e-3 for v in e)
    assert oracle.energy_bonded(s, whole, pos) == pytest.approx(sum(e), rel=1e-14)
    f = sum(oracle.forces_bonded(s, p, pos)["f"] for p in parts)
    assert np.allclose(oracle.forces_bonded(s, whole, pos)["f"], f, rtol=1e-13, atol=1e-12)


def test_net_force_and_torque_vanish_per_chain():
    M, L = 11, 10.0
    pos = walk_chains(5, M, L, seed=7)
    s = sys_for(len(pos), L)
    b = oracle.make_bonded(M, fene_k=30.0, bend_k=2.0, tors_c=(0.1, 0.5, -0.3, 0.9))
    f = oracle.forces_bonded(s, b, pos)["f"]
    R = unwrap(pos, M, L)
    scale = np.abs(f).max()
    for c in range(5):
        sl = slice(c * M, (c + 1) * M)
        assert np.abs(f[sl].sum(0)).max() < 1e-12 * scale
        torque = np.cross(R[sl] - R[sl][0], f[sl]).sum(0)
        assert np.abs(torque).max() < 1e-11 * scale


def test_virial_is_minus_the_stretch_derivative():
    M, L = 8, 14.0
    pos = walk_chains(4, M, L, seed=11)
    s = sys_for(len(pos), L)
    b = oracle.make_bonded(M, fene_k=30.0, bend_k=1.2, tors_c=(0.0, 0.7, 0.2, -0.5))
    W = oracle.forces_bonded(s, b, pos)["w"].sum()
    R = unwrap(pos, M, L)
    first = np.repeat(R[::M], M, axis=0)

    def U(lam):
        return oracle.energy_bonded(s, b, np.mod(first + lam * (R - first), L))

    h = 1e-6
    dU = (U(1 + h) - U(1 - h)) / (2 * h)
    assert W == pytest.approx(-dU, rel=1e-7)


def test_zero_coefficients_run_is_the_plain_run():
    from paper_2003_14061_amd import inputs

    n = 500
    rng = np.random.default_rng(2)
    L = inputs.box_length(n, 0.6)
    pos = inputs.fcc_positions(n, L, rng)
    vel = inputs.thermal_velocities(n, 1.0, rng)
    s = oracle.make_sys(n, L, r_cut=2 ** (1 / 6), skin=0.3, dt=0.005)
    b = oracle.make_bonded(5, fene_k=0.0)
    a = oracle.run(s, pos, vel, 20)
    c = oracle.run_bonded(s, b, pos, vel, 20)
    for u, v in zip(a[:3], c[:3]):
        assert np.array_equal(u, v)
    assert np.array_equal(a[3]["U"], c[3]["U"]) and a[4] == c[4]


def test_bonded_run_conserves_energy():
    """A 512-atom melt of 16-atom chains (rho 0.85) with FENE bonds and bending:
    momentum stays zero, the leapfrog keeps the total energy to O(dt^2), and
    halving dt quarters its fluctuation."""
    from paper_2003_14061_amd import inputs

    m = inputs.polymer_preset("melt_4k", n_side=8, chain_length=16).materialize()
    b = oracle.make_bonded(16, fene_k=30.0, fene_r0=1.5, bend_k=1.5)
    spread = []
    for dt, steps in ((0.002, 150), (0.001, 300)):
        s = oracle.make_sys(m.n, m.L, r_cut=m.r_cut, skin=m.skin, dt=dt)
        _, _, _, obs, _ = oracle.run_bonded(s, b, m.pos, m.vel, steps)
        E = obs["U"] + obs["K"]
        assert np.abs(obs["P"]).max() < 1e-9
        spread.append(E.max() - E.min())
    assert spread[1] < 0.35 * spread[0]
