"""Pins of the oracle's reverse mode (oracle/md_oracle_adjoint.c).

Each pin checks the oracle against something other than its own formulas:
central finite differences of the independently pinned force routine, of
the pair routine, of the g(r) sum and of whole trajectories; symmetry of the
force Jacobian; brute force over all pairs; the ideal-gas limit of g(r);
translation invariance.  The whole-trajectory finite differences run on WCA
soft spheres, whose force is continuous at the cutoff, so the pathwise
adjoint and the finite difference measure the same derivative.
"""
import numpy as np
import pytest

import oracle
from paper_2003_14061_amd import inputs

WCA_RC = 2.0 ** (1.0 / 6.0)


def jittered(n_cells, rho, amp, seed):
    L = inputs.box_length(4 * n_cells ** 3, rho)
    pos = inputs.fcc_sites(n_cells, L)
    rng = np.random.default_rng(seed)
    pos = np.mod(pos + amp * rng.standard_normal(pos.shape), L)
    return L, pos


def lists(s, pos):
    nc = oracle.cells_per_side(s.L, s.r_cut + s.skin)
    assert nc >= 3  # the 27-cell stencil needs distinct cells
    cells = oracle.build_cells(s, nc, pos)
    cnt, nl, longest = oracle.build_nl(s, nc, pos, cells)
    assert longest <= s.nl_cap
    return cnt, nl


def min_gap_to_cutoff(s, pos, cnt, nl):
    gap = np.inf
    for i in range(s.n):
        js = nl[i, : cnt[i]]
        d = pos[i] - pos[js]
        d -= s.L * np.rint(d / s.L)
        r = np.sqrt((d * d).sum(1))
        gap = min(gap, np.abs(r - s.r_cut).min())
    return gap


@pytest.mark.parametrize("r", [0.95, 1.0, 1.1, 1.3, 2.0, 2.45])
def test_pair_derivatives_match_differences_of_the_pair_routine(r):
    s = oracle.make_sys(10, 10.0, r_cut=2.5, eps=1.3, sigma=0.9)
    fr, gr, fs = oracle.pair_deriv(s, r * r)
    _, fr_pair = oracle.pair(s, r * r)
    assert fr == pytest.approx(fr_pair, rel=1e-13, abs=1e-15)
    h = 1e-6 * r
    d = (oracle.pair(s, (r + h) ** 2)[1] - oracle.pair(s, (r - h) ** 2)[1]) / (2 * h)
    assert gr * r == pytest.approx(d, rel=1e-7, abs=1e-9)
    hs = 1e-6
    sp = oracle.make_sys(10, 10.0, r_cut=2.5, eps=1.3, sigma=0.9 + hs)
    sm = oracle.make_sys(10, 10.0, r_cut=2.5, eps=1.3, sigma=0.9 - hs)
    d = (oracle.pair(sp, r * r)[1] - oracle.pair(sm, r * r)[1]) / (2 * hs)
    assert fs == pytest.approx(d, rel=1e-7, abs=1e-9)


def test_pair_derivatives_vanish_beyond_the_cutoff():
    s = oracle.make_sys(10, 10.0, r_cut=2.5)
    assert oracle.pair_deriv(s, 2.5 ** 2) == (0.0, 0.0, 0.0)
    assert oracle.pair_deriv(s, 7.0) == (0.0, 0.0, 0.0)


@pytest.mark.parametrize("pot,rc,amp", [("wca", WCA_RC, 0.05), ("lj", 2.5, 0.08)])
def test_force_jacobian_matches_differences_of_the_forces(pot, rc, amp):
    L, pos = jittered(5, 0.8, amp, 11)
    s = oracle.make_sys(len(pos), L, r_cut=rc, skin=0.3, eps=1.1, sigma=1.0)
    cnt, nl = lists(s, pos)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal(pos.shape)
    h = 1e-6
    # no pair may cross the cutoff under the +-h lam perturbation
    assert min_gap_to_cutoff(s, pos, cnt, nl) > 10 * 2 * h * np.abs(lam).max()
    jl, de, ds = oracle.hvp(s, pos, cnt, nl, lam)
    fp = oracle.forces_nl(s, pos + h * lam, cnt, nl)["f"]
    fm = oracle.forces_nl(s, pos - h * lam, cnt, nl)["f"]
    fd = (fp - fm) / (2 * h)
    assert np.linalg.norm(jl - fd) <= 1e-6 * np.linalg.norm(fd)
    # parameter contractions: sum_i lam_i . dF_i/dtheta
    he = 1e-6
    f = {}
    for k, kw in (("e+", dict(eps=1.1 + he)), ("e-", dict(eps=1.1 - he)),
                  ("s+", dict(sigma=1.0 + he)), ("s-", dict(sigma=1.0 - he))):
        sk = oracle.make_sys(len(pos), L, r_cut=rc, skin=0.3, **dict(dict(eps=1.1, sigma=1.0), **kw),
                             nl_cap=s.nl_cap)
        f[k] = (lam * oracle.forces_nl(sk, pos, cnt, nl)["f"]).sum()
    assert de == pytest.approx((f["e+"] - f["e-"]) / (2 * he), rel=1e-7)
    assert ds == pytest.approx((f["s+"] - f["s-"]) / (2 * he), rel=1e-6)


def test_force_jacobian_is_symmetric_and_blind_to_uniform_shifts():
    L, pos = jittered(6, 0.8442, 0.06, 12)
    s = oracle.make_sys(len(pos), L, r_cut=2.5, skin=0.3)
    cnt, nl = lists(s, pos)
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(pos.shape), rng.standard_normal(pos.shape)
    ja = oracle.hvp(s, pos, cnt, nl, a)[0]
    jb = oracle.hvp(s, pos, cnt, nl, b)[0]
    lhs, rhs = (a * jb).sum(), (b * ja).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(a * jb).sum()
    shift = np.tile(rng.standard_normal(3), (s.n, 1))
    assert np.abs(oracle.hvp(s, pos, cnt, nl, shift)[0]).max() == 0.0


def test_gr_over_the_list_equals_brute_force():
    L, pos = jittered(5, 0.8, 0.1, 13)
    s = oracle.make_sys(len(pos), L, r_cut=2.5, skin=0.3)
    g = oracle.gr_spec(50, 2.5)
    cnt, nl = lists(s, pos)
    a = oracle.gr(s, g, pos, cnt, nl)
    b = oracle.gr_allpairs(s, g, pos)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)
    with pytest.raises(RuntimeError):
        oracle.gr(s, oracle.gr_spec(50, 2.8), pos, cnt, nl)


def test_gr_of_an_ideal_gas_is_one():
    # uniform random points: E g_b = (N-1)/N (m0 + m2 w^2 / r_b^2), with m0 and
    # m2 the zeroth and second moments (in units of w) of the kernel, a
    # standard normal density lowered by its value at 3 and cut there; the
    # w^2 / r_b^2 term comes from the r^2 weight of the shell
    n, rho = 6000, 0.8
    L = (n / rho) ** (1 / 3)
    pos = np.random.default_rng(5).uniform(0, L, (n, 3))
    s = oracle.make_sys(n, L, r_cut=2.5, skin=0.3)
    g = oracle.gr_spec(50, 2.5)
    cnt, nl = lists(s, pos)
    gb = oracle.gr(s, g, pos, cnt, nl)
    rb = (np.arange(50) + 0.5) * 0.05
    from scipy.stats import norm
    inner, p3 = 2 * norm.cdf(3.0) - 1, norm.pdf(3.0)
    m0 = inner - 6 * p3                  # int_{-3}^{3} (phi(z) - phi(3)) dz
    m2 = inner - 6 * p3 - 18 * p3        # int_{-3}^{3} z^2 (phi(z) - phi(3)) dz
    expect = (n - 1) / n * (m0 + m2 * (0.05 / rb) ** 2)
    sel = rb >= 1.0
    npairs = n * rho * 4 * np.pi * (2.5 ** 3 - 1.0) / 3  # pairs counted in the selection
    tol = 4.0 / np.sqrt(npairs)
    assert abs(gb[sel].mean() / expect[sel].mean() - 1.0) < tol


def test_gr_gradient_matches_differences_of_gr():
    L, pos = jittered(5, 0.8, 0.1, 14)
    s = oracle.make_sys(len(pos), L, r_cut=2.5, skin=0.3)
    g = oracle.gr_spec(50, 2.5)
    cnt, nl = lists(s, pos)
    rng = np.random.default_rng(6)
    wgt = rng.standard_normal(50)
    grad = oracle.gr_grad(s, g, pos, cnt, nl, wgt)
    for k in range(3):
        d = rng.standard_normal(pos.shape)
        # the kernel has kinks at +-3 widths: a step small enough that no pair
        # distance crosses one
        h = 1e-8
        fp = (wgt * oracle.gr(s, g, pos + h * d, cnt, nl)).sum()
        fm = (wgt * oracle.gr(s, g, pos - h * d, cnt, nl)).sum()
        assert (grad * d).sum() == pytest.approx((fp - fm) / (2 * h), rel=1e-5)


# ---- whole trajectories ----

def wca_case(n_cells=4, steps=20, seed=21):
    L, pos = jittered(n_cells, 0.8, 0.04, seed)
    vel = inputs.thermal_velocities(len(pos), 1.0, np.random.default_rng(seed + 1))
    g = oracle.gr_spec(24, 1.2, 0.05)
    return L, pos, vel, g, steps


def wca_sys(n, L, eps=1.0, sigma=1.0):
    return oracle.make_sys(n, L, r_cut=WCA_RC * sigma, skin=0.3, dt=0.005, eps=eps, sigma=sigma)


def loss(s, g, steps, pos, vel, gU, gG):
    ub, gb = oracle.traj_obs(s, g, steps, pos, vel)
    return gU * ub + (gG * gb).sum()


def test_trajectory_gradient_matches_finite_differences():
    L, pos, vel, g, steps = wca_case()
    n = len(pos)
    rng = np.random.default_rng(7)
    gU, gG = 1.0, rng.standard_normal(g.n_bins)
    s = wca_sys(n, L)
    a = oracle.traj_adjoint(s, g, steps, pos, vel, gU, gG)
    ub, gb = oracle.traj_obs(s, g, steps, pos, vel)
    assert a["ubar"] == ub and np.array_equal(a["g"], gb)
    h = 1e-6
    # eps and sigma (the cutoff moves with sigma)
    for k, (p, m) in enumerate(((wca_sys(n, L, eps=1 + h), wca_sys(n, L, eps=1 - h)),
                                (wca_sys(n, L, sigma=1 + h), wca_sys(n, L, sigma=1 - h)))):
        fd = (loss(p, g, steps, pos, vel, gU, gG) - loss(m, g, steps, pos, vel, gU, gG)) / (2 * h)
        assert a["grad_theta"][k] == pytest.approx(fd, rel=1e-5)
    # initial positions and velocities along random directions
    for key, base in (("grad_x0", "pos"), ("grad_v0", "vel")):
        d = rng.standard_normal(pos.shape)
        args_p = dict(pos=pos, vel=vel)
        args_m = dict(pos=pos, vel=vel)
        args_p[base] = args_p[base] + h * d
        args_m[base] = args_m[base] - h * d
        fd = (loss(s, g, steps, args_p["pos"], args_p["vel"], gU, gG) -
              loss(s, g, steps, args_m["pos"], args_m["vel"], gU, gG)) / (2 * h)
        assert (a[key] * d).sum() == pytest.approx(fd, rel=1e-5)


def test_trajectory_gradient_is_translation_invariant():
    L, pos, vel, g, steps = wca_case(steps=10, seed=31)
    s = wca_sys(len(pos), L)
    a = oracle.traj_adjoint(s, g, steps, pos, vel, 1.0, np.ones(g.n_bins))
    gx = a["grad_x0"]
    assert np.abs(gx.sum(0)).max() <= 1e-10 * np.abs(gx).sum()


def test_one_step_gradient_has_its_closed_form():
    # one step, energy term only: L = U(x_1)/N with
    # x_1 = x_0 + dt (v_0 + c F(x_0)),  c = dt / (2 m), F linear in eps, so
    #   dL/dv_0 = -dt F(x_1) / N
    #   dL/deps = U(x_1) / (eps N) - dt c F(x_1) . F(x_0) / (eps N)
    L, pos, vel, g, _ = wca_case(steps=1, seed=41)
    n = len(pos)
    eps = 1.3
    s = wca_sys(n, L, eps=eps)
    a = oracle.traj_adjoint(s, g, 1, pos, vel, 1.0, np.zeros(g.n_bins))
    cnt, nl = lists(s, pos)
    f0 = oracle.forces_nl(s, pos, cnt, nl)["f"]
    pos1, _, f1, obs, _ = oracle.run(s, pos, vel, 1)
    c = 0.5 * s.dt / s.mass
    assert np.allclose(a["grad_v0"], -s.dt * f1 / n, rtol=1e-12, atol=1e-15)
    want = obs["U"][0] / (eps * n) - s.dt * c * (f1 * f0).sum() / (eps * n)
    assert a["grad_theta"][0] == pytest.approx(want, rel=1e-11)


def test_short_lj_trajectory_gradient_matches_finite_differences():
    # full LJ: the force jumps at r_cut, so the pathwise gradient equals the
    # difference quotient only while no pair crosses the cutoff; a few steps
    # and a tiny step size keep it so.  The cutoff moves with sigma (2.5 sigma).
    L, pos = jittered(5, 0.8, 0.05, 51)
    n = len(pos)
    vel = inputs.thermal_velocities(n, 1.0, np.random.default_rng(52))
    g = oracle.gr_spec(50, 2.5)
    steps, h = 5, 1e-8

    def sys(eps=1.0, sigma=1.0):
        return oracle.make_sys(n, L, r_cut=2.5 * sigma, skin=0.3, dt=0.004, eps=eps, sigma=sigma)

    rng = np.random.default_rng(53)
    gG = 0.1 * rng.standard_normal(g.n_bins)
    a = oracle.traj_adjoint(sys(), g, steps, pos, vel, 1.0, gG)
    for k, (p, m) in enumerate(((sys(eps=1 + h), sys(eps=1 - h)),
                                (sys(sigma=1 + h), sys(sigma=1 - h)))):
        fd = (loss(p, g, steps, pos, vel, 1.0, gG) - loss(m, g, steps, pos, vel, 1.0, gG)) / (2 * h)
        assert a["grad_theta"][k] == pytest.approx(fd, rel=1e-5)
    # along the gradient itself the derivative is |grad| (far above the
    # rounding noise of the difference quotient); along a random direction
    # the error is measured against |grad| |d|
    gx = a["grad_x0"]
    for d in (gx / np.linalg.norm(gx), rng.standard_normal(pos.shape)):
        fd = (loss(sys(), g, steps, pos + h * d, vel, 1.0, gG) -
              loss(sys(), g, steps, pos - h * d, vel, 1.0, gG)) / (2 * h)
        assert abs((gx * d).sum() - fd) <= 1e-4 * np.linalg.norm(gx) * np.linalg.norm(d)
