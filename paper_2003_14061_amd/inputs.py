"""Seeded synthetic inputs: lattices, velocities and workload presets.

This module only builds initial states.  It holds none of the method's
arithmetic (no potential, cells, lists, forces or integration), so both the
GPU path and the CPU oracle may consume what it produces.

The paper starts from a simple-cubic grid of atoms with random velocities
(section 3.1).  The workloads here start from a face-centred cubic lattice,
n^3 unit cells of edge a = L/n with the four-site basis (0,0,0),
(1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2) offset by a/4, so that every site lies
strictly inside [0, L).  Velocities are standard normal, shifted to zero
total momentum and scaled to the requested temperature with 3(N-1) degrees
of freedom.  Atom ids are the row order of the returned arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

WCA_CUT = 2.0 ** (1.0 / 6.0)

_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def box_length(n: int, rho: float) -> float:
    """Edge of the cube holding n atoms at number density rho."""
    return (n / rho) ** (1.0 / 3.0)


def fcc_sites(n_cells: int, L: float) -> np.ndarray:
    """All 4*n_cells^3 FCC sites in [0, L)^3, shape (4 n^3, 3), float64."""
    a = L / n_cells
    g = np.arange(n_cells, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1)
    pts = (cells[:, None, :] + _BASIS[None, :, :] + 0.25) * a
    return np.ascontiguousarray(pts.reshape(-1, 3))


def sc_positions(n_side: int, L: float) -> np.ndarray:
    """Simple-cubic grid of n_side^3 atoms at cell centres (the paper's
    initial state, section 3.1), shape (n_side^3, 3)."""
    a = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], 1))


def fcc_positions(n_atoms: int, L: float, rng: np.random.Generator | None = None) -> np.ndarray:
    """n_atoms sites of an FCC lattice filling the box.

    When n_atoms = 4 n^3 the full lattice is returned; otherwise the lattice
    with n = ceil((n_atoms/4)^(1/3)) cells per side is built and n_atoms of
    its sites are drawn uniformly without replacement (kept in lattice
    order)."""
    n = round((n_atoms / 4) ** (1.0 / 3.0))
    if 4 * n ** 3 == n_atoms:
        return fcc_sites(n, L)
    n = math.ceil((n_atoms / 4) ** (1.0 / 3.0))
    sites = fcc_sites(n, L)
    if rng is None:
        raise ValueError("a generator is needed to pick a subset of lattice sites")
    pick = np.sort(rng.choice(len(sites), size=n_atoms, replace=False))
    return np.ascontiguousarray(sites[pick])


def thermal_velocities(n_atoms: int, T: float, rng: np.random.Generator,
                       mass: float = 1.0) -> np.ndarray:
    """Gaussian velocities with zero total momentum at temperature T."""
    v = rng.standard_normal((n_atoms, 3))
    v -= v.mean(axis=0)
    if n_atoms > 1 and T > 0:
        t_now = mass * float((v * v).sum()) / (3.0 * (n_atoms - 1))
        v *= math.sqrt(T / t_now)
    else:
        v[:] = 0.0
    return np.ascontiguousarray(v)


def jitter(pos: np.ndarray, L: float, amplitude: float, rng: np.random.Generator) -> np.ndarray:
    """Displace every coordinate by amplitude * N(0,1) and fold into [0, L)."""
    p = pos + amplitude * rng.standard_normal(pos.shape)
    p = np.mod(p, L)
    p[p >= L] = 0.0
    return np.ascontiguousarray(p)


@dataclasses.dataclass
class Workload:
    """One system: physical parameters plus the seeded initial state."""
    name: str
    n: int
    rho: float
    T: float
    dt: float
    r_cut: float
    skin: float
    use_nl: bool
    shifted: bool
    steps: int
    seed: int
    eps: float = 1.0
    sigma: float = 1.0
    mass: float = 1.0
    L: float = 0.0
    pos: np.ndarray | None = None
    vel: np.ndarray | None = None

    def materialize(self, jitter_amp: float = 0.0) -> "Workload":
        rng = np.random.default_rng(self.seed)
        self.L = box_length(self.n, self.rho)
        self.pos = fcc_positions(self.n, self.L, rng)
        self.vel = thermal_velocities(self.n, self.T, rng, self.mass)
        if jitter_amp > 0:
            self.pos = jitter(self.pos, self.L, jitter_amp, rng)
        return self


def preset(name: str, **over) -> Workload:
    """The five workloads the method is exercised on, by descriptive name.

    wca_4000      WCA, N=4000 (10^3 FCC), rho 0.8, T 1, dt 0.005, cells only
    wca_256k      WCA, N=256000 (40^3 FCC), rho 0.8, T 1, dt 0.005, skin 0.3
    lj_2048k      LJ r_c 2.5, N=2048000 (80^3 FCC), rho 0.8442, T 0.72, dt 0.004, skin 0.3
    lj_32k        LJ r_c 2.5, N=32000 (20^3 FCC), rho 0.8, T 1, dt 0.004, skin 0.3
    """
    table = {
        "wca_4000": dict(n=4000, rho=0.8, T=1.0, dt=0.005, r_cut=WCA_CUT, skin=0.3,
                         use_nl=False, shifted=True, steps=1000, seed=1),
        "wca_256k": dict(n=256000, rho=0.8, T=1.0, dt=0.005, r_cut=WCA_CUT, skin=0.3,
                         use_nl=True, shifted=True, steps=2000, seed=2),
        "lj_2048k": dict(n=2048000, rho=0.8442, T=0.72, dt=0.004, r_cut=2.5, skin=0.3,
                         use_nl=True, shifted=True, steps=1000, seed=3),
        "lj_32k": dict(n=32000, rho=0.8, T=1.0, dt=0.004, r_cut=2.5, skin=0.3,
                       use_nl=True, shifted=True, steps=200, seed=5),
    }
    if name not in table:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(table)}")
    kw = dict(table[name])
    kw.update(over)
    return Workload(name=name, **kw)


def ensemble_specs(n_replicas: int = 64, seed: int = 4, n_lo: int = 500, n_hi: int = 32000,
                   rho_lo: float = 0.6, rho_hi: float = 0.9):
    """Atom counts and densities of the independent-replica ensemble.

    Counts uniform on [n_lo, n_hi], densities uniform on [rho_lo, rho_hi];
    replica r draws from child r of SeedSequence(seed)."""
    children = np.random.SeedSequence(seed).spawn(n_replicas)
    out = []
    for r, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n = int(rng.integers(n_lo, n_hi + 1))
        rho = float(rng.uniform(rho_lo, rho_hi))
        out.append((n, rho, ss))
    return out


def ensemble(n_replicas: int = 64, seed: int = 4, T: float = 1.0, dt: float = 0.005,
             skin: float = 0.3, **kw):
    """Materialized replicas (WCA), each with its own seeded state."""
    reps = []
    for r, (n, rho, ss) in enumerate(ensemble_specs(n_replicas, seed, **kw)):
        rng = np.random.default_rng(ss.spawn(1)[0])
        L = box_length(n, rho)
        w = Workload(name=f"replica{r}", n=n, rho=rho, T=T, dt=dt, r_cut=WCA_CUT, skin=skin,
                     use_nl=True, shifted=True, steps=500, seed=seed)
        w.L = L
        w.pos = fcc_positions(n, L, rng)
        w.vel = thermal_velocities(n, T, rng)
        reps.append(w)
    return reps


def snake_sites(n_side: int, L: float) -> np.ndarray:
    """The n_side^3 simple-cubic sites of sc_positions, ordered along a
    boustrophedon path: x runs back and forth along each row, the rows of a
    plane back and forth in y, and the planes in z with every other plane
    walked in reverse, so that consecutive sites are always nearest
    neighbors (lattice spacing L / n_side apart)."""
    a = L / n_side
    order = []
    for z in range(n_side):
        plane = []
        for y in range(n_side):
            xs = range(n_side) if y % 2 == 0 else range(n_side - 1, -1, -1)
            plane.extend((x, y, z) for x in xs)
        if z % 2 == 1:
            plane.reverse()
        order.extend(plane)
    return np.ascontiguousarray((np.array(order, dtype=np.float64) + 0.5) * a)


@dataclasses.dataclass
class PolymerMelt:
    """Linear chains of consecutive ids (atoms c*M .. c*M + M - 1 form chain
    c) cut from a boustrophedon path through a simple-cubic lattice at number
    density rho, Gaussian-jittered, with thermal velocities."""
    name: str
    n_side: int
    chain_length: int
    rho: float
    T: float
    dt: float
    r_cut: float
    skin: float
    jitter: float
    seed: int
    n: int = 0
    L: float = 0.0
    pos: np.ndarray | None = None
    vel: np.ndarray | None = None

    def materialize(self) -> "PolymerMelt":
        self.n = self.n_side ** 3
        if self.n % self.chain_length:
            raise ValueError("the lattice does not divide into whole chains")
        rng = np.random.default_rng(self.seed)
        self.L = box_length(self.n, self.rho)
        self.pos = jitter(snake_sites(self.n_side, self.L), self.L, self.jitter, rng)
        self.vel = thermal_velocities(self.n, self.T, rng)
        return self


def polymer_preset(name: str, **over) -> PolymerMelt:
    """Polymer melts by descriptive name.

    melt_256k    4096 chains of 64, 64^3 = 262144 atoms, rho 0.85, T 1, dt 0.005,
                 WCA between all atoms, skin 0.3
    melt_32k     1024 chains of 32, 32^3 = 32768 atoms, otherwise the same
    melt_4k      256 chains of 16, 16^3 = 4096 atoms, otherwise the same
    """
    table = {
        "melt_256k": dict(n_side=64, chain_length=64, rho=0.85, T=1.0, dt=0.005,
                          r_cut=WCA_CUT, skin=0.3, jitter=0.05, seed=21),
        "melt_32k": dict(n_side=32, chain_length=32, rho=0.85, T=1.0, dt=0.005,
                         r_cut=WCA_CUT, skin=0.3, jitter=0.05, seed=22),
        "melt_4k": dict(n_side=16, chain_length=16, rho=0.85, T=1.0, dt=0.005,
                        r_cut=WCA_CUT, skin=0.3, jitter=0.05, seed=23),
    }
    if name not in table:
        raise KeyError(f"unknown polymer workload {name!r}; known: {sorted(table)}")
    kw = dict(table[name])
    kw.update(over)
    return PolymerMelt(name=name, **kw)
