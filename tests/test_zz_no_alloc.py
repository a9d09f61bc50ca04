"""md_bind_static: a context bound to the library's own static workspace
array gives bitwise the same cells-to-forces pass, observables and run as
the same context bound to a caller-allocated workspace (same kernels, same
launch shape), on two static bindings in a row, the second smaller than the
first, and refuses a context whose workspace exceeds the array."""
import numpy as np
import pytest

from paper_2003_14061_amd import inputs
from paper_2003_14061_amd import md

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


def system(n, rho, jitter, seed):
    rng = np.random.default_rng(seed)
    L = inputs.box_length(n, rho)
    pos = inputs.jitter(inputs.fcc_positions(n, L, rng), L, jitter, rng)
    vel = inputs.thermal_velocities(n, 1.0, rng)
    return pos, vel, L


def run(pos, vel, L, static, steps, **kw):
    sim = md.Simulation(pos, vel, L, device="cuda:0", static_workspace=static, **kw)
    if static:
        assert sim.workspace is None
    sim.prepare()
    first = (sim.state()["f"], sim.reduce())
    sim.step(steps, record_every=1)
    hist = sim.history()
    obs = sim.reduce()
    st = sim.state()
    return sim, first, hist, obs, st


def same(a, b):
    (fa, oa), ha, obs_a, sta = a[1:]
    (fb, ob), hb, obs_b, stb = b[1:]
    assert np.array_equal(fa, fb), "forces after the first pass differ"
    for k in ("U", "K", "W", "T", "pressure"):
        assert oa[k] == ob[k], k
    assert np.array_equal(ha, hb), "step histories differ"
    for k in ("U", "K", "W", "step", "n_rebuilds", "flags", "max_nl"):
        assert obs_a[k] == obs_b[k], k
    for k in ("pos", "vel", "f"):
        assert np.array_equal(sta[k], stb[k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_binding_matches_allocated_workspace_twice(precision):
    # first binding: 32 000-atom LJ with a neighbor list (reorder on)
    pos, vel, L = system(32000, 0.8, 0.05, 61)
    kw = dict(r_cut=2.5, skin=0.3, dt=0.004, precision=precision)
    ref = run(pos, vel, L, False, 60, **kw)
    got = run(pos, vel, L, True, 60, **kw)
    assert md.md_workspace_bytes(got[0].ctx) <= STATIC_BYTES
    same(ref, got)
    assert got[3]["n_rebuilds"] > 0 and got[3]["flags"] == 0
    del got
    # second binding, smaller: 4000 atoms, so what the first left in the
    # array beyond this workspace stays there and what lies inside is cleared
    pos, vel, L = system(4000, 0.8442, 0.05, 62)
    ref = run(pos, vel, L, False, 40, **kw)
    got = run(pos, vel, L, True, 40, **kw)
    same(ref, got)
    # cells only
    pos, vel, L = system(4000, 0.8, 0.06, 63)
    kw = dict(r_cut=2 ** (1 / 6), dt=0.005, neighbor_list=False, precision=precision)
    same(run(pos, vel, L, False, 40, **kw), run(pos, vel, L, True, 40, **kw))


def test_static_binding_refuses_a_workspace_beyond_the_array():
    n = 256000
    L = inputs.box_length(n, 0.8)
    pos = np.zeros((n, 3))
    with pytest.raises(md.MDError) as e:
        md.Simulation(pos, pos, L, r_cut=2 ** (1 / 6), skin=0.3, dt=0.005, device="cuda:0",
                      static_workspace=True)
    assert e.value.status == -11
