"""Reverse mode on the GPU (md_traj_forward / md_traj_backward, through the C
ABI, and the torch.autograd.Function over them) against the oracle's reverse
pass, plus properties that hold at any size: independence of the checkpoint
interval, finite differences of the GPU's own forward, FP32-mixed against
FP64, and the full 32000-atom, 200-step configuration."""
import numpy as np
import pytest

import oracle
from gpu_helpers import WCA, state
from paper_2003_14061_amd import md

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# name: n, rho, r_cut, dt, steps, checkpoint interval, bins, gr_rmax, gr_width, seed
CASES = {
    "lj4000": (4000, 0.8, 2.5, 0.004, 40, 10, 50, 2.5, 0.05, 61),
    "wca4000": (4000, 0.8, WCA, 0.005, 40, 7, 24, 1.2, 0.05, 62),
    "lj500_nc3": (500, 0.8, 2.5, 0.004, 20, 6, 50, 2.5, 0.05, 63),
    "lj4000_nogr": (4000, 0.8, 2.5, 0.004, 30, 10, 0, 2.5, 0.05, 64),
}


def setup(name, precision="fp64", checkpoint=None):
    n, rho, rc, dt, steps, k, bins, rmax, w, seed = CASES[name]
    L, pos, vel = state(n, rho, seed, jitter=0.05)
    sim = md.Simulation(pos, vel, L, r_cut=rc, dt=dt, skin=0.3, precision=precision,
                        reorder=False)
    tp = dict(n_steps=steps, checkpoint_every=checkpoint or k, n_bins=bins, gr_rmax=rmax,
              gr_width=w)
    rng = np.random.default_rng(seed + 100)
    gobs = np.concatenate([[1.0], 0.1 * rng.standard_normal(bins)])
    s = oracle.make_sys(n, L, r_cut=rc, skin=0.3, dt=dt)
    g = oracle.gr_spec(bins, rmax, w)
    return sim, tp, gobs, (s, g, steps, pos, vel)


def run_gpu(sim, tp, gobs):
    obs = sim.traj_forward(tp["n_steps"], tp["checkpoint_every"], tp["n_bins"], tp["gr_rmax"],
                           tp["gr_width"])
    gx, gv, gth = sim.traj_backward(torch.tensor(gobs, dtype=torch.float64))
    torch.cuda.synchronize()
    return obs.cpu().numpy(), gx.cpu().numpy(), gv.cpu().numpy(), gth.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_gradients_match_the_oracle(name):
    sim, tp, gobs, (s, g, steps, pos, vel) = setup(name)
    obs, gx, gv, gth = run_gpu(sim, tp, gobs)
    ref = oracle.traj_adjoint(s, g, steps, pos, vel, gobs[0], gobs[1:])
    assert abs(obs[0] - ref["ubar"]) <= 1e-10 * abs(ref["ubar"])
    if tp["n_bins"]:
        assert np.abs(obs[1:] - ref["g"]).max() <= 1e-9 * max(1.0, np.abs(ref["g"]).max())
    assert rel(gx, ref["grad_x0"]) <= 1e-8
    assert rel(gv, ref["grad_v0"]) <= 1e-8
    assert np.allclose(gth, ref["grad_theta"], rtol=1e-8, atol=0)
    st = sim.reduce()  # the state is back at step S, nothing latched
    assert st["flags"] == 0


def test_checkpoint_interval_changes_nothing_but_rounding():
    outs = []
    for k in (1, 7, 40):
        sim, tp, gobs, _ = setup("lj4000", checkpoint=k)
        outs.append(run_gpu(sim, tp, gobs))
    base = outs[0]
    for o in outs[1:]:
        assert abs(o[0][0] - base[0][0]) <= 1e-13 * abs(base[0][0])
        for a, b in zip(o[1:], base[1:]):
            assert rel(a, b) <= 1e-10


def test_fp32_mixed_gradients_stay_close_to_fp64():
    sim, tp, gobs, _ = setup("lj4000")
    o64 = run_gpu(sim, tp, gobs)
    sim, tp, gobs, _ = setup("lj4000", precision="fp32")
    o32 = run_gpu(sim, tp, gobs)
    assert abs(o32[0][0] - o64[0][0]) <= 1e-5 * abs(o64[0][0])
    assert rel(o32[1], o64[1]) <= 1e-2
    assert rel(o32[2], o64[2]) <= 1e-2
    assert np.allclose(o32[3], o64[3], rtol=1e-3, atol=0)


def test_gradient_matches_differences_of_the_gpu_forward():
    # WCA: the force is continuous at the cutoff, so the difference quotient
    # of the GPU's own observables measures the same derivative
    name = "wca4000"
    sim, tp, gobs, (s, g, steps, pos, vel) = setup(name)
    obs, gx, gv, gth = run_gpu(sim, tp, gobs)
    n, rho, rc, dt = CASES[name][:4]

    def loss(eps=1.0, sigma=1.0, dpos=0.0):
        sm = md.Simulation(pos + dpos, vel, s.L, r_cut=rc * sigma, dt=dt, skin=0.3, eps=eps,
                           sigma=sigma, reorder=False)
        o = sm.traj_forward(tp["n_steps"], tp["checkpoint_every"], tp["n_bins"],
                            tp["gr_rmax"], tp["gr_width"]).cpu().numpy()
        return float(gobs @ o)

    h = 1e-6
    assert gth[0] == pytest.approx((loss(eps=1 + h) - loss(eps=1 - h)) / (2 * h), rel=1e-5)
    assert gth[1] == pytest.approx((loss(sigma=1 + h) - loss(sigma=1 - h)) / (2 * h), rel=1e-5)
    d = gx / np.linalg.norm(gx)
    fd = (loss(dpos=h * d) - loss(dpos=-h * d)) / (2 * h)
    assert fd == pytest.approx(np.linalg.norm(gx), rel=1e-5)


def test_autograd_function_gives_the_same_gradients():
    from paper_2003_14061_amd.adjoint import TrajectorySpec, trajectory_observables

    name = "lj4000"
    n, rho, rc, dt, steps, k, bins, rmax, w, seed = CASES[name]
    _, tp, _, (s, g, _, pos, vel) = setup(name)
    spec = TrajectorySpec(L=s.L, n_steps=steps, dt=dt, r_cut_over_sigma=2.5, skin=0.3,
                          checkpoint_every=k, n_bins=bins, gr_rmax=rmax, gr_width=w)
    dev = torch.device("cuda")
    x0 = torch.tensor(pos, device=dev, requires_grad=True)
    v0 = torch.tensor(vel, device=dev, requires_grad=True)
    eps = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    sigma = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    ubar, gr = trajectory_observables(x0, v0, eps, sigma, spec)
    target = 0.9 * gr.detach() + 0.05
    loss = ubar + ((gr - target) ** 2).sum()
    gx, gv, ge, gs = torch.autograd.grad(loss, [x0, v0, eps, sigma])
    gG = (2.0 * (gr - target)).detach().cpu().numpy()
    ref = oracle.traj_adjoint(s, g, steps, pos, vel, 1.0, gG)
    assert gx.device == x0.device and ge.device == eps.device
    assert rel(gx.cpu().numpy(), ref["grad_x0"]) <= 1e-8
    assert rel(gv.cpu().numpy(), ref["grad_v0"]) <= 1e-8
    assert float(ge) == pytest.approx(ref["grad_theta"][0], rel=1e-8)
    assert float(gs) == pytest.approx(ref["grad_theta"][1], rel=1e-8)


@pytest.mark.parametrize("eps,sigma", [(1.0, 1.0), (1.05, 0.98)])
def test_full_size_differentiable_run_matches_the_oracle(eps, sigma):
    # 32000 atoms (20^3 FCC, rho 0.8, T 1), LJ r_c 2.5 sigma, dt 0.004, 200
    # steps, checkpoints every 20, 50 g(r) bins on [0, 2.5); (1.05, 0.98) is the
    # parameter point of the target run whose g(r) the loss compares against
    L, pos, vel = state(32000, 0.8, 5)
    sim = md.Simulation(pos, vel, L, r_cut=2.5 * sigma, dt=0.004, skin=0.3, eps=eps,
                        sigma=sigma, reorder=False)
    rng = np.random.default_rng(500)
    gobs = np.concatenate([[1.0], 0.1 * rng.standard_normal(50)])
    tp = dict(n_steps=200, checkpoint_every=20, n_bins=50, gr_rmax=2.5, gr_width=0.05)
    obs, gx, gv, gth = run_gpu(sim, tp, gobs)
    s = oracle.make_sys(32000, L, r_cut=2.5 * sigma, skin=0.3, dt=0.004, eps=eps, sigma=sigma)
    ref = oracle.traj_adjoint(s, oracle.gr_spec(50, 2.5, 0.05), 200, pos, vel, gobs[0], gobs[1:])
    assert abs(obs[0] - ref["ubar"]) <= 1e-10 * abs(ref["ubar"])
    assert np.abs(obs[1:] - ref["g"]).max() <= 1e-9 * np.abs(ref["g"]).max()
    assert rel(gx, ref["grad_x0"]) <= 1e-7
    assert rel(gv, ref["grad_v0"]) <= 1e-7
    assert np.allclose(gth, ref["grad_theta"], rtol=1e-7, atol=0)
    # any size: the loss does not change under a uniform translation
    assert np.abs(gx.sum(0)).max() <= 1e-9 * np.abs(gx).sum()


@pytest.mark.parametrize("eps,sigma,mass", [(1.05, 0.98, 1.0), (1.3, 0.9, 2.0)])
def test_gradients_match_the_oracle_away_from_unit_parameters(eps, sigma, mass):
    # the pair derivatives scale with eps and sigma, the kicks of the reverse
    # pass with 1/m; at eps = sigma = m = 1 a wrong factor would cancel
    n, steps, k, bins, dt = 4000, 40, 10, 50, 0.004
    rng = np.random.default_rng(71)
    from paper_2003_14061_amd import inputs

    L = inputs.box_length(n, 0.8 / sigma ** 3)
    pos = inputs.jitter(inputs.fcc_positions(n, L, rng), L, 0.05 * sigma, rng)
    vel = inputs.thermal_velocities(n, eps, rng, mass=mass)
    rmax, width = 2.5 * sigma, 0.05
    sim = md.Simulation(pos, vel, L, r_cut=2.5 * sigma, dt=dt, skin=0.3, eps=eps, sigma=sigma,
                        mass=mass, reorder=False)
    gobs = np.concatenate([[1.0], 0.1 * rng.standard_normal(bins)])
    tp = dict(n_steps=steps, checkpoint_every=k, n_bins=bins, gr_rmax=rmax, gr_width=width)
    obs, gx, gv, gth = run_gpu(sim, tp, gobs)
    s = oracle.make_sys(n, L, r_cut=2.5 * sigma, skin=0.3, dt=dt, eps=eps, sigma=sigma,
                        mass=mass)
    ref = oracle.traj_adjoint(s, oracle.gr_spec(bins, rmax, width), steps, pos, vel, gobs[0],
                              gobs[1:])
    assert abs(obs[0] - ref["ubar"]) <= 1e-10 * abs(ref["ubar"])
    assert np.abs(obs[1:] - ref["g"]).max() <= 1e-9 * max(1.0, np.abs(ref["g"]).max())
    assert rel(gx, ref["grad_x0"]) <= 1e-8
    assert rel(gv, ref["grad_v0"]) <= 1e-8
    assert np.allclose(gth, ref["grad_theta"], rtol=1e-8, atol=0)


def test_reverse_mode_arguments_are_checked():
    L, pos, vel = state(4000, 0.8, 66)
    sim = md.Simulation(pos, vel, L, r_cut=2.5, dt=0.004, skin=0.3)  # reorder on
    with pytest.raises(md.MDError):
        sim.traj_forward(10, 5)
    sim = md.Simulation(pos, vel, L, r_cut=2.5, dt=0.004, skin=0.3, reorder=False)
    with pytest.raises(md.MDError):  # g(r) range beyond the list radius
        sim.traj_forward(10, 5, 50, 2.7, 0.05)
    with pytest.raises(RuntimeError):
        sim.traj_backward(torch.zeros(1, dtype=torch.float64))
