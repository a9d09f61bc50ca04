"""CPU FP64 oracle for the short-range MD step -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle.so`` (built from ``md_oracle.c`` by
``oracle/build.py``).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never imports or links it.

Every function takes and returns numpy arrays in atom-id order.  The method
follows Rapaport, arXiv:2003.14061, section 2.3 (steps N1-N5, F1-F2); see
the C header for the conventions.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

LJ_SHIFTED = 0
LJ_TRUNC = 1


class Sys(C.Structure):
    _fields_ = [("n", C.c_int32), ("potential", C.c_int32), ("L", C.c_double),
                ("eps", C.c_double), ("sigma", C.c_double), ("mass", C.c_double),
                ("r_cut", C.c_double), ("skin", C.c_double), ("dt", C.c_double),
                ("use_nl", C.c_int32), ("nl_cap", C.c_int32)]


class Bonded(C.Structure):
    """Chain topology and bonded parameters (md_oracle_bonded.h)."""
    _fields_ = [("chain_length", C.c_int32), ("pad", C.c_int32), ("fene_k", C.c_double),
                ("fene_r0", C.c_double), ("bend_k", C.c_double), ("tors_c", C.c_double * 4)]


def make_bonded(chain_length, fene_k=30.0, fene_r0=1.5, bend_k=0.0, tors_c=(0.0, 0.0, 0.0, 0.0)):
    return Bonded(int(chain_length), 0, float(fene_k), float(fene_r0), float(bend_k),
                  (C.c_double * 4)(*[float(c) for c in tors_c]))


class GrSpec(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("rmax", C.c_double), ("width", C.c_double)]


class Obs(C.Structure):
    _fields_ = [("U", C.c_double), ("K", C.c_double), ("W", C.c_double),
                ("P", C.c_double * 3), ("dmax2", C.c_double),
                ("rebuilt", C.c_int32), ("max_nl", C.c_int32)]


_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_SP = C.POINTER(Sys)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(path)
        L.or_pair.restype = C.c_double
        L.or_pair.argtypes = [_SP, C.c_double, C.POINTER(C.c_double)]
        L.or_pair_scale.restype = C.c_double
        L.or_pair_scale.argtypes = [_SP, C.c_double]
        L.or_shift.restype = C.c_double
        L.or_shift.argtypes = [_SP]
        L.or_wrap.restype = C.c_double
        L.or_wrap.argtypes = [C.c_double, C.c_double]
        L.or_minimg.restype = C.c_double
        L.or_minimg.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_cells_per_side.restype = C.c_int32
        L.or_cells_per_side.argtypes = [C.c_double, C.c_double]
        L.or_build_cells.restype = None
        L.or_build_cells.argtypes = [_SP, C.c_int32, _D, _D, _D, _I, _I, _I]
        L.or_build_nl.restype = C.c_int32
        L.or_build_nl.argtypes = [_SP, C.c_int32, _D, _D, _D, _I, _I, _I, _I, _I]
        L.or_build_nl_half.restype = C.c_int32
        L.or_build_nl_half.argtypes = [_SP, C.c_int32, _D, _D, _D, _I, _I, _I, _I, _I]
        fo = [_D, _D, _D, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_forces_nl.restype = None
        L.or_forces_nl.argtypes = [_SP, _D, _D, _D, _I, _I] + fo
        L.or_forces_half.restype = None
        L.or_forces_half.argtypes = [_SP, _D, _D, _D, _I, _I] + fo
        L.or_forces_cells.restype = None
        L.or_forces_cells.argtypes = [_SP, C.c_int32, _D, _D, _D, _I, _I, _I] + fo
        L.or_forces_allpairs.restype = None
        L.or_forces_allpairs.argtypes = [_SP, _D, _D, _D] + fo
        L.or_forces_sample.restype = None
        L.or_forces_sample.argtypes = [_SP, _D, _D, _D, _I, C.c_int32] + fo
        L.or_kinetic.restype = C.c_double
        L.or_kinetic.argtypes = [_SP, _D, _D, _D]
        L.or_momentum.restype = None
        L.or_momentum.argtypes = [_SP, _D, _D, _D, _D]
        L.or_max_disp2.restype = C.c_double
        L.or_max_disp2.argtypes = [_SP, _D, _D, _D, _D, _D, _D]
        L.or_kick.restype = None
        L.or_kick.argtypes = [_SP, _D, _D, _D, _D, _D, _D]
        L.or_drift.restype = None
        L.or_drift.argtypes = [_SP, _D, _D, _D, _D, _D, _D]
        L.or_run.restype = C.c_int32
        L.or_run.argtypes = [_SP, C.c_int32, _D, _D, _D, _D, _D, _D, _D, _D, _D, C.c_void_p]
        L.or_threads.restype = C.c_int32
        L.or_threads.argtypes = []
        # reverse mode (md_oracle_adjoint.h)
        _GP = C.POINTER(GrSpec)
        _PD = C.POINTER(C.c_double)
        L.or_pair_deriv.restype = None
        L.or_pair_deriv.argtypes = [_SP, C.c_double, _PD, _PD, _PD]
        L.or_hvp.restype = None
        L.or_hvp.argtypes = [_SP, _D, _D, _D, _I, _I, _D, _D, _D, _D, _D, _D, _PD, _PD]
        L.or_gr.restype = C.c_int32
        L.or_gr.argtypes = [_SP, _GP, _D, _D, _D, _I, _I, _D]
        L.or_gr_allpairs.restype = None
        L.or_gr_allpairs.argtypes = [_SP, _GP, _D, _D, _D, _D]
        L.or_gr_grad.restype = None
        L.or_gr_grad.argtypes = [_SP, _GP, _D, _D, _D, _I, _I, _D, _D, _D, _D]
        L.or_traj_obs.restype = C.c_int32
        L.or_traj_obs.argtypes = [_SP, _GP, C.c_int32, _D, _D, _D, _D, _D, _D, _PD, C.c_void_p]
        L.or_traj_adjoint.restype = C.c_int32
        L.or_traj_adjoint.argtypes = ([_SP, _GP, C.c_int32, _D, _D, _D, _D, _D, _D, C.c_double,
                                       C.c_void_p, _PD, C.c_void_p] + [_D] * 6 + [_D])
        # bonded chains (md_oracle_bonded.h)
        _BP = C.POINTER(Bonded)
        L.or_forces_bonded.restype = C.c_int32
        L.or_forces_bonded.argtypes = [_SP, _BP, _D, _D, _D] + fo
        L.or_energy_bonded.restype = C.c_double
        L.or_energy_bonded.argtypes = [_SP, _BP, _D, _D, _D]
        L.or_run_bonded.restype = C.c_int32
        L.or_run_bonded.argtypes = [_SP, _BP, C.c_int32, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                    C.c_void_p]
        _LIB = L
    return _LIB


def make_sys(n, L, *, r_cut, skin=0.0, dt=0.005, eps=1.0, sigma=1.0, mass=1.0,
             potential=LJ_SHIFTED, use_nl=True, nl_cap=None):
    """Pack the system description.  nl_cap defaults to a generous bound."""
    if nl_cap is None:
        rl = r_cut + skin
        mean = 4.0 / 3.0 * np.pi * rl ** 3 * n / L ** 3
        nl_cap = int(min(n, mean * 2.0 + 64))
    return Sys(int(n), int(potential), float(L), float(eps), float(sigma), float(mass),
               float(r_cut), float(skin), float(dt), int(bool(use_nl)), int(nl_cap))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _xyz(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return _c(pos[:, 0], np.float64), _c(pos[:, 1], np.float64), _c(pos[:, 2], np.float64)


def pair(s, r2):
    """Pair energy u(r) and force factor fr (F_i = fr * (r_i - r_j))."""
    fr = C.c_double()
    u = lib().or_pair(C.byref(s), float(r2), C.byref(fr))
    return u, fr.value


def pair_scale(s, r2):
    """48 eps (sr^12 + sr^6/2) / r: the error scale of one pair force."""
    return lib().or_pair_scale(C.byref(s), float(r2))


def shift(s):
    return lib().or_shift(C.byref(s))


def wrap(x, L):
    return lib().or_wrap(float(x), float(L))


def minimg(d, L):
    return lib().or_minimg(float(d), float(L), 1.0 / float(L))


def cells_per_side(L, r_cell):
    return int(lib().or_cells_per_side(float(L), float(r_cell)))


def build_cells(s, nc, pos):
    """N1-N4.  Returns (cell_of[n], cell_start[nc^3+1], cell_atoms[n])."""
    x, y, z = _xyz(pos)
    n = s.n
    cell_of = np.empty(n, np.int32)
    cell_start = np.empty(nc ** 3 + 1, np.int32)
    cell_atoms = np.empty(n, np.int32)
    lib().or_build_cells(C.byref(s), nc, x, y, z, cell_of, cell_start, cell_atoms)
    return cell_of, cell_start, cell_atoms


def build_nl(s, nc, pos, cells):
    """N5.  Returns (nl_count[n], nl[n, cap], longest)."""
    x, y, z = _xyz(pos)
    cell_of, cell_start, cell_atoms = cells
    n = s.n
    cnt = np.empty(n, np.int32)
    nl = np.full((n, s.nl_cap), -1, np.int32)
    longest = lib().or_build_nl(C.byref(s), nc, x, y, z, cell_of, cell_start, cell_atoms, cnt, nl)
    return cnt, nl, int(longest)


def build_nl_half(s, nc, pos, cells):
    """The half list (partner later in (cell, id) order).  Returns
    (nl_count[n], nl[n, cap], longest)."""
    x, y, z = _xyz(pos)
    cell_of, cell_start, cell_atoms = cells
    n = s.n
    cnt = np.empty(n, np.int32)
    nl = np.full((n, s.nl_cap), -1, np.int32)
    longest = lib().or_build_nl_half(C.byref(s), nc, x, y, z, cell_of, cell_start, cell_atoms,
                                     cnt, nl)
    return cnt, nl, int(longest)


def _fout(n):
    return (np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n))


def _pack(o):
    fx, fy, fz, u, w, sm = o
    return {"f": np.stack([fx, fy, fz], 1), "u": u, "w": w, "s": sm}


def _ptrs(o):
    return list(o[:3]) + [a.ctypes.data for a in o[3:]]


def forces_nl(s, pos, nl_count, nl):
    x, y, z = _xyz(pos)
    o = _fout(s.n)
    lib().or_forces_nl(C.byref(s), x, y, z, _c(nl_count, np.int32), _c(nl, np.int32), *_ptrs(o))
    return _pack(o)


def forces_half(s, pos, nl_count, nl):
    x, y, z = _xyz(pos)
    o = _fout(s.n)
    lib().or_forces_half(C.byref(s), x, y, z, _c(nl_count, np.int32), _c(nl, np.int32),
                         *_ptrs(o))
    return _pack(o)


def forces_cells(s, nc, pos, cells):
    x, y, z = _xyz(pos)
    o = _fout(s.n)
    lib().or_forces_cells(C.byref(s), nc, x, y, z, *[_c(a, np.int32) for a in cells], *_ptrs(o))
    return _pack(o)


def forces_allpairs(s, pos):
    x, y, z = _xyz(pos)
    o = _fout(s.n)
    lib().or_forces_allpairs(C.byref(s), x, y, z, *_ptrs(o))
    return _pack(o)


def forces_sample(s, pos, idx):
    """Brute-force forces on the atoms listed in idx (ids)."""
    x, y, z = _xyz(pos)
    idx = _c(idx, np.int32)
    o = _fout(len(idx))
    lib().or_forces_sample(C.byref(s), x, y, z, idx, len(idx), *_ptrs(o))
    return _pack(o)


def kinetic(s, vel):
    vx, vy, vz = _xyz(vel)
    return lib().or_kinetic(C.byref(s), vx, vy, vz)


def momentum(s, vel):
    vx, vy, vz = _xyz(vel)
    p = np.zeros(3)
    lib().or_momentum(C.byref(s), vx, vy, vz, p)
    return p


def max_disp2(s, pos, ref):
    return lib().or_max_disp2(C.byref(s), *_xyz(pos), *_xyz(ref))


def kick(s, vel, f):
    vx, vy, vz = _xyz(vel)
    lib().or_kick(C.byref(s), vx, vy, vz, *_xyz(f))
    return np.stack([vx, vy, vz], 1)


def drift(s, pos, vel):
    x, y, z = _xyz(pos)
    lib().or_drift(C.byref(s), x, y, z, *_xyz(vel))
    return np.stack([x, y, z], 1)


def run(s, pos, vel, n_steps):
    """Advance n_steps of kick-drift-[rebuild]-force-kick.

    Returns (pos, vel, f, obs, n_rebuilds) where obs is a structured array
    with fields U, K, W, P, dmax2, rebuilt, max_nl, one record per step."""
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    fx, fy, fz = np.zeros(s.n), np.zeros(s.n), np.zeros(s.n)
    obs = (Obs * max(n_steps, 1))()
    r = lib().or_run(C.byref(s), int(n_steps), x, y, z, vx, vy, vz, fx, fy, fz,
                     C.cast(obs, C.c_void_p))
    if r < 0:
        raise RuntimeError({-1: "bad arguments", -2: "box too small for 3 cells per side",
                            -3: "neighbor list overflow"}.get(r, f"oracle error {r}"))
    dt = np.dtype([("U", "f8"), ("K", "f8"), ("W", "f8"), ("P", "f8", 3), ("dmax2", "f8"),
                   ("rebuilt", "i4"), ("max_nl", "i4")])
    arr = np.frombuffer(bytes(obs), dtype=dt)[:n_steps].copy()
    return (np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), np.stack([fx, fy, fz], 1),
            arr, int(r))


def threads():
    return int(lib().or_threads())


# ---------------------------------------------------------------------------
# Reverse mode (md_oracle_adjoint.h): pair derivatives, Jacobian-vector
# products of the forces, the soft g(r), and whole-trajectory gradients.

def gr_spec(n_bins=0, rmax=2.5, width=None):
    """Soft g(r) bins on [0, rmax); width defaults to the bin width."""
    if width is None:
        width = rmax / n_bins if n_bins else 0.0
    return GrSpec(int(n_bins), float(rmax), float(width))


def pair_deriv(s, r2):
    """(fr, gr, fs): -u'/r, (1/r) d fr/dr and d fr/d sigma at r^2 = r2."""
    fr, gr, fs = C.c_double(), C.c_double(), C.c_double()
    lib().or_pair_deriv(C.byref(s), float(r2), C.byref(fr), C.byref(gr), C.byref(fs))
    return fr.value, gr.value, fs.value


def hvp(s, pos, nl_count, nl, lam):
    """(J lam [n,3], sum lam.dF/deps, sum lam.dF/dsigma), J = dF/dx."""
    x, y, z = _xyz(pos)
    lx, ly, lz = _xyz(lam)
    jx, jy, jz = np.zeros(s.n), np.zeros(s.n), np.zeros(s.n)
    de, ds = C.c_double(), C.c_double()
    lib().or_hvp(C.byref(s), x, y, z, _c(nl_count, np.int32), _c(nl, np.int32), lx, ly, lz,
                 jx, jy, jz, C.byref(de), C.byref(ds))
    return np.stack([jx, jy, jz], 1), de.value, ds.value


def gr(s, g, pos, nl_count, nl):
    out = np.zeros(g.n_bins)
    r = lib().or_gr(C.byref(s), C.byref(g), *_xyz(pos), _c(nl_count, np.int32),
                    _c(nl, np.int32), out)
    if r:
        raise RuntimeError("g(r) range plus 3 widths exceeds the list radius")
    return out


def gr_allpairs(s, g, pos):
    out = np.zeros(g.n_bins)
    lib().or_gr_allpairs(C.byref(s), C.byref(g), *_xyz(pos), out)
    return out


def gr_grad(s, g, pos, nl_count, nl, wgt):
    gx, gy, gz = np.zeros(s.n), np.zeros(s.n), np.zeros(s.n)
    lib().or_gr_grad(C.byref(s), C.byref(g), *_xyz(pos), _c(nl_count, np.int32),
                     _c(nl, np.int32), _c(wgt, np.float64), gx, gy, gz)
    return np.stack([gx, gy, gz], 1)


_TRAJ_ERR = {-1: "bad arguments", -2: "box too small for 3 cells per side",
             -3: "neighbor list overflow", -4: "g(r) range exceeds the list radius"}


def traj_obs(s, g, n_steps, pos, vel):
    """(ubar, g) of the n_steps trajectory from (pos, vel)."""
    ub = C.c_double()
    out = np.zeros(max(g.n_bins, 1))
    r = lib().or_traj_obs(C.byref(s), C.byref(g), int(n_steps), *_xyz(pos), *_xyz(vel),
                          C.byref(ub), out.ctypes.data)
    if r:
        raise RuntimeError(_TRAJ_ERR.get(r, f"oracle error {r}"))
    return ub.value, out[: g.n_bins]


def traj_adjoint(s, g, n_steps, pos, vel, gU, gG=None):
    """Gradients of L (dL/dubar = gU, dL/dg = gG) with respect to the initial
    positions and velocities and (eps, sigma).  Returns a dict with ubar, g,
    grad_x0 [n,3], grad_v0 [n,3], grad_theta [2]."""
    ub = C.c_double()
    out = np.zeros(max(g.n_bins, 1))
    gG = np.zeros(max(g.n_bins, 1)) if gG is None else _c(gG, np.float64)
    o = [np.zeros(s.n) for _ in range(6)]
    th = np.zeros(2)
    r = lib().or_traj_adjoint(C.byref(s), C.byref(g), int(n_steps), *_xyz(pos), *_xyz(vel),
                              float(gU), gG.ctypes.data, C.byref(ub), out.ctypes.data, *o, th)
    if r:
        raise RuntimeError(_TRAJ_ERR.get(r, f"oracle error {r}"))
    return {"ubar": ub.value, "g": out[: g.n_bins], "grad_x0": np.stack(o[:3], 1),
            "grad_v0": np.stack(o[3:], 1), "grad_theta": th}


# ---------------------------------------------------------------------------
# Bonded chains (md_oracle_bonded.h): FENE bonds, bond angles, dihedrals of
# linear chains of consecutive ids, section 4.3 item (2).

def forces_bonded(s, b, pos):
    """Bonded forces alone: dict f, u (energy booked to each term's first
    atom), w (bond virial), s (rounding-error scale)."""
    x, y, z = _xyz(pos)
    o = _fout(s.n)
    r = lib().or_forces_bonded(C.byref(s), C.byref(b), x, y, z, *_ptrs(o))
    if r < 0:
        raise RuntimeError("bonded forces undefined (bad topology or a bond at R0)")
    return _pack(o)


def energy_bonded(s, b, pos):
    return float(lib().or_energy_bonded(C.byref(s), C.byref(b), *_xyz(pos)))


def run_bonded(s, b, pos, vel, n_steps):
    """As run(), with the bonded forces of b added to the pair forces."""
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    fx, fy, fz = np.zeros(s.n), np.zeros(s.n), np.zeros(s.n)
    obs = (Obs * max(n_steps, 1))()
    r = lib().or_run_bonded(C.byref(s), C.byref(b), int(n_steps), x, y, z, vx, vy, vz,
                            fx, fy, fz, C.cast(obs, C.c_void_p))
    if r < 0:
        raise RuntimeError({-1: "bad arguments", -2: "box too small for 3 cells per side",
                            -3: "neighbor list overflow", -4: "a bond reached R0"}
                           .get(r, f"oracle error {r}"))
    dt = np.dtype([("U", "f8"), ("K", "f8"), ("W", "f8"), ("P", "f8", 3), ("dmax2", "f8"),
                   ("rebuilt", "i4"), ("max_nl", "i4")])
    arr = np.frombuffer(bytes(obs), dtype=dt)[:n_steps].copy()
    return (np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), np.stack([fx, fy, fz], 1),
            arr, int(r))
