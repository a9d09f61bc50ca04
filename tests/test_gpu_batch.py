"""Batched replicas on the GPU (md_batch_*, through the C ABI): every replica
of a batch follows exactly the trajectory the same system follows alone
(same kernels, same tuning: bit for bit), with and without the HIP graph,
and the oracle within the parity tolerances; the autotuner picks one of its
candidates and leaves a working batch."""
import numpy as np
import pytest

import oracle
from gpu_helpers import min_image
from paper_2003_14061_amd import inputs, md

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def systems(n_replicas=6, n_lo=500, n_hi=6000, jitter=0.03, seed=4):
    out = []
    for w in inputs.ensemble(n_replicas, seed=seed, n_lo=n_lo, n_hi=n_hi):
        rng = np.random.default_rng(w.n)
        pos = inputs.jitter(w.pos, w.L, jitter, rng)
        out.append(dict(pos=pos, vel=w.vel, L=w.L, r_cut=w.r_cut, dt=w.dt, skin=w.skin))
    return out


def single(sy, precision, batch=None, r=0):
    """The same system alone; with the batch's integration grid for replica r
    (a batch gives each replica a smaller share), so that the kinetic-energy
    and momentum sums add in the same order, and its tiling (a system alone
    prefers at least a tile per CU), so that the per-tile energy partials do."""
    s = md.Simulation(sy["pos"], sy["vel"], sy["L"], r_cut=sy["r_cut"], dt=sy["dt"],
                      skin=sy["skin"], precision=precision)
    if batch is not None:
        t = md.md_get_tuning(batch.replicas[r])
        s.set_tuning(integrate_grid=t["integrate_grid"], tile_cells=t["tile_cells"],
                     tile_y=t["tile_y"], tile_z=t["tile_z"])
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("graph", [True, False])
def test_every_replica_matches_its_single_system_run_bitwise(precision, graph):
    sys_ = systems()
    b = md.Batch(sys_, precision=precision)
    b.prepare()
    b.run(30, record_every=5, graph=graph)
    b.run(30, record_every=5, graph=graph)  # a second launch of the same graph
    for r, sy in enumerate(sys_):
        s = single(sy, precision, b, r)
        s.prepare()
        s.step(30, record_every=5)
        s.step(30, record_every=5)
        a, c = b.state(r), s.state()
        for k in ("pos", "vel", "f"):
            assert np.array_equal(a[k], c[k]), (r, k)
        assert np.array_equal(b.history(r), s.history()), r
        assert b.reduce(r)["flags"] == 0


def test_replicas_follow_the_oracle():
    sys_ = systems(n_replicas=5, seed=9)
    b = md.Batch(sys_, precision="fp64")
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
        assert np.max(np.abs(h["K"] - o_ref["K"])) <= 1e-10 * e_scale, r
        assert np.abs(min_image(st["pos"] - p_ref, sy["L"])).max() < 1e-10, r
        assert np.abs(st["vel"] - v_ref).max() < 1e-9, r


def test_a_replica_of_three_cells_per_side_follows_the_oracle():
    """A 108-atom replica (3 cells per side: the minimum image by rounding) in
    a batch of larger ones sends the whole batch's list build to its full
    kernel; every replica still follows the oracle and its own single run."""
    from gpu_helpers import WCA, state
    sys_ = systems(n_replicas=3, seed=9)
    L, pos, vel = state(108, 0.8, 3, jitter=0.05)
    sys_.append(dict(pos=pos, vel=vel, L=L, r_cut=WCA, dt=0.005, skin=0.3))
    assert oracle.cells_per_side(L, WCA + 0.3) == 3
    b = md.Batch(sys_, precision="fp64")
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
        one = single(sy, "fp64", b, r)
        one.prepare()
        one.step(steps, record_every=1)
        assert np.array_equal(st["pos"], one.state()["pos"]), r
        assert b.reduce(r)["flags"] == 0


def test_autotuner_keeps_its_best_candidate():
    sys_ = systems(n_replicas=4, seed=11)
    b = md.Batch(sys_, precision="fp32")
    cands = [dict(force_lanes=l, force_block=fb) for l in (2, 4, 8) for fb in (256, 512)]
    best, costs = b.autotune(cands, reps=2)
    assert 0 <= best < len(cands) and all(c > 0 for c in costs)
    assert costs[best] == min(costs)
    t = b.get_tuning()
    assert t["force_lanes"] == cands[best]["force_lanes"]
    assert t["force_block"] == cands[best]["force_block"]
    b.run(10)
    for r, sy in enumerate(sys_):
        s = single(sy, "fp32", b, r)
        s.set_tuning(**cands[best])
        s.prepare()
        s.step(10)
        assert np.array_equal(b.state(r)["pos"], s.state()["pos"]), r


def test_batch_arguments_are_checked():
    sys_ = systems(n_replicas=2)
    p = [md.Params(len(sy["pos"]), md.MD_LJ_SHIFTED, sy["L"], 1.0, 1.0, 1.0, sy["r_cut"], 0.3,
                   0.005, md.MD_FP64 if r == 0 else md.MD_FP32_MIXED, md.MD_NEIGHBOR_LIST, 0, 0,
                   1, 256) for r, sy in enumerate(sys_)]
    with pytest.raises(md.MDError):
        md.md_batch_init(p, 2)
    b = md.Batch(sys_)
    with pytest.raises(md.MDError):  # not prepared yet
        b.run(5)


def test_autotune_cache_keeps_and_reuses_the_choice(tmp_path):
    sys_ = systems(n_replicas=3, seed=12)
    cache = tmp_path / "tuning.json"
    cands = [dict(force_lanes=l, force_block=fb) for l in (2, 4) for fb in (256, 512)] + \
        [dict(force_lanes=2, force_block=256, tile_cells=4, tile_y=2, tile_z=2)]
    b = md.Batch(sys_, precision="fp32")
    best, costs = b.autotune(cands, reps=2, cache_path=str(cache))
    assert costs[best] == min(costs) and min(costs) > 0
    text = cache.read_text()
    assert text.startswith("{") and text.rstrip().endswith("}") and text.count('"ms"') == 1
    # the same batch and candidates again: taken from the file, not timed
    b2 = md.Batch(sys_, precision="fp32")
    best2, costs2 = b2.autotune(cands, reps=2, cache_path=str(cache))
    assert best2 == best and all(c == -1.0 for c in costs2)
    t = b2.get_tuning()
    assert t["force_lanes"] == cands[best]["force_lanes"]
    b2.run(10)
    assert max(b2.reduce(r)["flags"] for r in range(len(sys_))) == 0
    # another candidate list is another entry
    b3 = md.Batch(sys_, precision="fp32")
    b3.autotune(cands[:2], reps=2, cache_path=str(cache))
    assert cache.read_text().count('"ms"') == 2


def test_single_system_autotune_with_cache(tmp_path):
    import oracle
    from gpu_helpers import force_errors, pair, state

    L, pos, vel = state(32000, 0.8442, 13, jitter=0.05)
    sim, s = pair(pos, vel, L, r_cut=2.5)
    sim.prepare()
    cands = [dict(force_lanes=4, force_block=512), dict(force_lanes=2, force_block=512),
             dict(force_lanes=4, force_block=512, tile_cells=8, tile_y=1, tile_z=1),
             dict(force_lanes=4, force_block=256, tile_cells=2, tile_y=2, tile_z=2)]
    cache = tmp_path / "tuning.json"
    best, costs = sim.autotune(cands, reps=2, cache_path=str(cache))
    assert costs[best] == min(costs) and min(costs) > 0
    # forces of the chosen shape are current and match the oracle
    st = sim.state()
    nc = oracle.cells_per_side(s.L, s.r_cut + s.skin)
    p = np.mod(st["pos"], L)
    cells = oracle.build_cells(s, nc, p)
    cnt, nl, _ = oracle.build_nl(s, nc, p, cells)
    per_atom, normwise = force_errors(st["f"], oracle.forces_nl(s, p, cnt, nl))
    assert per_atom <= 1e-12 and normwise <= 1e-12
    sim.step(40)
    assert sim.reduce()["flags"] == 0
    sim2, _ = pair(pos, vel, L, r_cut=2.5)
    sim2.prepare()
    best2, costs2 = sim2.autotune(cands, reps=2, cache_path=str(cache))
    assert best2 == best and all(c == -1.0 for c in costs2)
