"""Shared helpers of the GPU parity tests: build a GPU system and its oracle
twin from the same seeded input, and compare them in atom-id space."""
import math

import numpy as np

import oracle
from paper_2003_14061_amd import inputs
from paper_2003_14061_amd import md

WCA = 2.0 ** (1.0 / 6.0)


def state(n, rho, seed, jitter=0.0, lattice=True):
    rng = np.random.default_rng(seed)
    L = inputs.box_length(n, rho)
    if lattice:
        pos = inputs.fcc_positions(n, L, rng)
    else:
        pos = rng.uniform(0.0, L, (n, 3))
        pos[pos >= L] = 0.0
    vel = inputs.thermal_velocities(n, 1.0, rng)
    if jitter > 0:
        pos = inputs.jitter(pos, L, jitter, rng)
    return L, pos, vel


def pair(pos, vel, L, *, r_cut, dt=0.005, skin=0.3, nl=True, shifted=True,
         precision="fp64", reorder=None, nl_capacity=0, block=256, newton3=False,
         eps=1.0, sigma=1.0, mass=1.0, pipeline="tiled"):
    """A GPU Simulation and the oracle system description with the same
    parameters (same list capacity)."""
    sim = md.Simulation(pos, vel, L, r_cut=r_cut, dt=dt, skin=skin, shifted=shifted,
                        precision=precision, neighbor_list=nl, reorder=reorder,
                        nl_capacity=nl_capacity, block=block, newton3=newton3, eps=eps,
                        sigma=sigma, mass=mass, pipeline=pipeline)
    cap = sim.grid.nl_capacity if nl else 1
    s = oracle.make_sys(len(pos), L, r_cut=r_cut, skin=skin if nl else 0.0, dt=dt, eps=eps,
                        sigma=sigma, mass=mass,
                        potential=oracle.LJ_SHIFTED if shifted else oracle.LJ_TRUNC,
                        use_nl=nl, nl_cap=max(cap, 1))
    return sim, s


def oracle_cells(sim, s, pos):
    nc = sim.grid.nc
    assert nc == oracle.cells_per_side(s.L, s.r_cut + s.skin)
    return nc, oracle.build_cells(s, nc, pos)


def check_cells(sim, s, pos):
    nc, (o_of, o_start, o_atoms) = oracle_cells(sim, s, pos)
    c = sim.cells()
    ids = c["id"]
    n = len(ids)
    assert sorted(ids.tolist()) == list(range(n))
    of_id = np.empty(n, np.int32)
    of_id[ids] = c["cell_of"]
    assert np.array_equal(of_id, o_of), "cell of each atom differs"
    assert np.array_equal(c["cell_start"], o_start), "cell offsets differ"
    assert np.array_equal(ids[c["cell_atoms"]], o_atoms), "cell contents or order differ"
    return nc, (o_of, o_start, o_atoms)


def check_nl(sim, s, pos, cells, half=False):
    """The GPU list against the oracle's (the half list with half=True),
    entry by entry in atom-id space."""
    nc = sim.grid.nc
    build = oracle.build_nl_half if half else oracle.build_nl
    o_cnt, o_nl, longest = build(s, nc, pos, cells)
    cnt, nl = sim.neighbor_list()
    ids = sim.ids()
    n = len(ids)
    cap = sim.grid.nl_capacity
    assert longest <= cap
    cnt_id = np.empty(n, np.int32)
    cnt_id[ids] = cnt[:n]
    assert np.array_equal(cnt_id, o_cnt), "list lengths differ"
    m = np.arange(cap)[:, None] < cnt[None, :n]
    g = np.where(m, ids[np.clip(nl[:, :n], 0, n - 1)], -1)  # (cap, n) in slot order
    g_id = np.empty((n, cap), np.int32)
    g_id[ids] = g.T
    o = np.where(np.arange(cap)[None, :] < o_cnt[:, None], o_nl[:, :cap], -1)
    assert np.array_equal(g_id, o), "list entries or their order differ"
    return o_cnt, o_nl


def compare_lists(ids, cnt, nl, o_cnt, o_nl, chunk=1 << 18):
    """Every list of the GPU (slot space: cnt[n_pad], nl[cap, n_pad] decoded to
    slots) against the oracle's (id space: o_cnt[n], o_nl[n, >= cap]), entry
    by entry in list order, vectorised over chunks of atoms."""
    n = len(ids)
    cap = nl.shape[0]
    slot_of = np.empty(n, np.int64)
    slot_of[ids] = np.arange(n)
    assert np.array_equal(cnt[:n][slot_of], o_cnt), "list lengths differ"
    assert int(o_cnt.max(initial=0)) <= cap
    col = np.arange(cap)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        sl = slot_of[a:b]
        rows = nl[:, sl]
        m = col[:, None] < cnt[sl][None, :]
        g = np.where(m, ids[np.clip(rows, 0, n - 1)], -1).T
        o = np.where(col[None, :] < o_cnt[a:b, None], o_nl[a:b, :cap], -1)
        assert np.array_equal(g, o), f"list entries or their order differ for ids {a}..{b}"


def force_errors(f_gpu, ref):
    """Errors in the contract's norms: per atom scaled by S_i (sum over the
    atom's pairs of the magnitudes of the repulsive and attractive force
    terms), and normwise."""
    d = np.linalg.norm(f_gpu - ref["f"], axis=1)
    scale = np.maximum(ref["s"], 1e-300)
    per_atom = float(np.max(d / scale)) if len(d) else 0.0
    fn = float(np.linalg.norm(ref["f"]))
    normwise = float(np.linalg.norm(f_gpu - ref["f"]) / fn) if fn > 0 else float(np.linalg.norm(f_gpu - ref["f"]))
    return per_atom, normwise


def energy_error(U_gpu, ref):
    return abs(U_gpu - ref["u"].sum()) / max(np.abs(ref["u"]).sum(), 1e-300)


def min_image(d, L):
    return d - L * np.round(d / L)
