"""Python binding of libmd (the C ABI in include/md.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libmd.so.  PyTorch provides the device memory (tensors) and the stream.
There is no CPU fallback: if libmd.so is missing or no GPU is present the
calls raise.

Low-level functions carry the C names (md_init, md_bind, md_build_cells,
md_build_neighbors, md_forces, md_step, md_reduce, ...).  ``Simulation``
owns the tensors of one system and calls them in order.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmd.so")

MD_OK = 0
MD_LJ_SHIFTED, MD_LJ_TRUNC = 0, 1
MD_FP64, MD_FP32_MIXED = 0, 1
MD_CELLS_ONLY, MD_NEIGHBOR_LIST = 0, 1
MD_NL_AUTO, MD_NL_LANES, MD_NL_CELL_WAVES = 0, 1, 2
MD_PIPE_TILED, MD_PIPE_LAYERS, MD_PIPE_ALLPAIRS = 0, 1, 2
(MD_ARR_CELL_OF, MD_ARR_CELL_START, MD_ARR_CELL_ATOMS, MD_ARR_NL, MD_ARR_NL_COUNT, MD_ARR_XREF,
 MD_ARR_LAYERS, MD_ARR_LAYER_COUNT) = range(8)

EXPORTS = ("md_init", "md_workspace_bytes", "md_geometry", "md_layout", "md_bind",
           "md_bind_static", "md_set_graph",
           "md_build_cells", "md_build_neighbors", "md_forces", "md_step", "md_reduce",
           "md_history", "md_set_tuning", "md_get_tuning", "md_set_timing", "md_get_timing",
           "md_get_timing_parts",
           "md_export_neighbors", "md_traj_workspace_bytes", "md_traj_forward",
           "md_traj_backward", "md_batch_init", "md_batch_workspace_bytes", "md_batch_replica",
           "md_batch_bind", "md_batch_prepare", "md_batch_forces", "md_batch_layout",
           "md_batch_run", "md_batch_set_tuning",
           "md_batch_get_tuning", "md_batch_autotune", "md_autotune", "md_batch_destroy",
           "md_destroy",
           "md_status_str", "md_set_bonded")


class MDError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {status_str(status)} ({status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("potential", C.c_int32), ("L", C.c_double),
                ("eps", C.c_double), ("sigma", C.c_double), ("mass", C.c_double),
                ("r_cut", C.c_double), ("skin", C.c_double), ("dt", C.c_double),
                ("precision", C.c_int32), ("mode", C.c_int32), ("newton3", C.c_int32),
                ("nl_capacity", C.c_int32), ("reorder", C.c_int32), ("block", C.c_int32),
                ("pipeline", C.c_int32)]


class Buffers(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz",
                                           "id", "workspace")]


class Bonded(C.Structure):
    """md_bonded: linear chains of consecutive ids, FENE bonds, bond angles,
    dihedrals (section 4.3, item (2))."""
    _fields_ = [("chain_length", C.c_int32), ("pad", C.c_int32), ("fene_k", C.c_double),
                ("fene_r0", C.c_double), ("bend_k", C.c_double), ("tors_c", C.c_double * 4)]


class Grid(C.Structure):
    _fields_ = [("nc", C.c_int32), ("n_cells", C.c_int32), ("nl_capacity", C.c_int32),
                ("n_pad", C.c_int32), ("cell_width", C.c_double), ("n_layers", C.c_int32),
                ("pad", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("force_lanes", C.c_int32), ("force_block", C.c_int32),
                ("nl_block", C.c_int32), ("tile_cells", C.c_int32), ("stage_cap", C.c_int32),
                ("integrate_grid", C.c_int32), ("nl_method", C.c_int32),
                ("tile_y", C.c_int32), ("tile_z", C.c_int32)]


class TrajParams(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("checkpoint_every", C.c_int32), ("n_bins", C.c_int32),
                ("pad", C.c_int32), ("gr_rmax", C.c_double), ("gr_width", C.c_double)]


class Observables(C.Structure):
    _fields_ = [("U", C.c_double), ("K", C.c_double), ("W", C.c_double),
                ("P", C.c_double * 3), ("T", C.c_double), ("pressure", C.c_double),
                ("dmax", C.c_double), ("step", C.c_int64), ("n_rebuilds", C.c_int64),
                ("max_occupancy", C.c_int32), ("max_nl", C.c_int32), ("flags", C.c_int32),
                ("pad", C.c_int32)]


class Record(C.Structure):
    _fields_ = [("step", C.c_int64), ("U", C.c_double), ("K", C.c_double), ("W", C.c_double),
                ("P", C.c_double * 3), ("dmax", C.c_double), ("rebuilt", C.c_int32),
                ("pad", C.c_int32)]


_LIB = None


def lib():
    """Load libmd.so; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "md_init": (C.c_int, [C.POINTER(Params), C.POINTER(P)]),
        "md_workspace_bytes": (C.c_size_t, [P]),
        "md_geometry": (C.c_int, [P, C.POINTER(Grid)]),
        "md_layout": (C.c_int, [P, C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "md_bind": (C.c_int, [P, C.POINTER(Buffers), P]),
        "md_bind_static": (C.c_int, [P, C.POINTER(Buffers), P]),
        "md_build_cells": (C.c_int, [P]),
        "md_build_neighbors": (C.c_int, [P]),
        "md_forces": (C.c_int, [P]),
        "md_step": (C.c_int, [P, C.c_int32, C.c_int32]),
        "md_set_graph": (C.c_int, [P, C.c_int32]),
        "md_reduce": (C.c_int, [P, C.POINTER(Observables)]),
        "md_history": (C.c_int, [P, C.POINTER(Record), C.c_int32, C.POINTER(C.c_int32)]),
        "md_export_neighbors": (C.c_int, [P, P]),
        "md_set_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
        "md_get_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
        "md_set_timing": (C.c_int, [P, C.c_int32]),
        "md_get_timing": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "md_get_timing_parts": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "md_traj_workspace_bytes": (C.c_size_t, [P, C.POINTER(TrajParams)]),
        "md_traj_forward": (C.c_int, [P, C.POINTER(TrajParams), P, P]),
        "md_traj_backward": (C.c_int, [P, C.POINTER(TrajParams), P, P, P, P, P]),
        "md_batch_init": (C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(P)]),
        "md_batch_workspace_bytes": (C.c_size_t, [P]),
        "md_batch_replica": (C.c_int, [P, C.c_int32, C.POINTER(P)]),
        "md_batch_bind": (C.c_int, [P, C.POINTER(Buffers), P, P]),
        "md_batch_prepare": (C.c_int, [P]),
        "md_batch_forces": (C.c_int, [P]),
        "md_batch_layout": (C.c_int, [P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t),
                                      C.POINTER(C.c_size_t)]),
        "md_batch_run": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32]),
        "md_batch_set_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
        "md_batch_get_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
        "md_batch_autotune": (C.c_int, [P, C.POINTER(Tuning), C.c_int32, C.c_int32,
                                        C.c_char_p, C.POINTER(C.c_double),
                                        C.POINTER(C.c_int32)]),
        "md_autotune": (C.c_int, [P, C.POINTER(Tuning), C.c_int32, C.c_int32, C.c_char_p,
                                  C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "md_batch_destroy": (None, [P]),
        "md_destroy": (None, [P]),
        "md_status_str": (C.c_char_p, [C.c_int32]),
        "md_set_bonded": (C.c_int, [P, C.POINTER(Bonded)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def status_str(st):
    return lib().md_status_str(int(st)).decode()


def _check(st, where):
    if st != MD_OK:
        raise MDError(st, where)


# ---- C-named wrappers ------------------------------------------------------

def md_init(params: Params):
    ctx = C.c_void_p()
    _check(lib().md_init(C.byref(params), C.byref(ctx)), "md_init")
    return ctx


def md_set_bonded(ctx, chain_length=None, fene_k=30.0, fene_r0=1.5, bend_k=0.0,
                  tors_c=(0.0, 0.0, 0.0, 0.0)):
    """Bonded chains (chain_length None removes them)."""
    if chain_length is None:
        _check(lib().md_set_bonded(ctx, None), "md_set_bonded")
        return
    b = Bonded(int(chain_length), 0, float(fene_k), float(fene_r0), float(bend_k),
               (C.c_double * 4)(*[float(c) for c in tors_c]))
    _check(lib().md_set_bonded(ctx, C.byref(b)), "md_set_bonded")


def md_workspace_bytes(ctx) -> int:
    return int(lib().md_workspace_bytes(ctx))


def md_geometry(ctx) -> Grid:
    g = Grid()
    _check(lib().md_geometry(ctx, C.byref(g)), "md_geometry")
    return g


def md_layout(ctx, which):
    off, cnt = C.c_size_t(), C.c_size_t()
    _check(lib().md_layout(ctx, int(which), C.byref(off), C.byref(cnt)), "md_layout")
    return off.value, cnt.value


def md_bind(ctx, bufs: Buffers, stream_handle: int):
    _check(lib().md_bind(ctx, C.byref(bufs), C.c_void_p(stream_handle)), "md_bind")


def md_bind_static(ctx, bufs: Buffers, stream_handle: int):
    """md_bind onto the library's own static workspace (bufs.workspace None)."""
    _check(lib().md_bind_static(ctx, C.byref(bufs), C.c_void_p(stream_handle)),
           "md_bind_static")


def md_build_cells(ctx):
    _check(lib().md_build_cells(ctx), "md_build_cells")


def md_build_neighbors(ctx):
    _check(lib().md_build_neighbors(ctx), "md_build_neighbors")


def md_export_neighbors(ctx, dst_ptr: int):
    _check(lib().md_export_neighbors(ctx, C.c_void_p(dst_ptr)), "md_export_neighbors")


def md_forces(ctx):
    _check(lib().md_forces(ctx), "md_forces")


def md_step(ctx, n_steps: int, record_every: int = 0):
    _check(lib().md_step(ctx, int(n_steps), int(record_every)), "md_step")


def md_reduce(ctx, check: bool = True) -> Observables:
    o = Observables()
    st = lib().md_reduce(ctx, C.byref(o))
    if check:
        _check(st, "md_reduce")
    return o


def md_history(ctx, max_records: int = 4096):
    buf = (Record * max_records)()
    n = C.c_int32()
    _check(lib().md_history(ctx, buf, max_records, C.byref(n)), "md_history")
    return list(buf[: n.value])


def traj_params(n_steps, checkpoint_every=20, n_bins=0, gr_rmax=2.5, gr_width=None):
    """Trajectory description for md_traj_*; gr_width defaults to the bin width."""
    if gr_width is None:
        gr_width = gr_rmax / n_bins if n_bins else 0.0
    return TrajParams(int(n_steps), int(checkpoint_every), int(n_bins), 0, float(gr_rmax),
                      float(gr_width))


def md_traj_workspace_bytes(ctx, tp: TrajParams) -> int:
    return int(lib().md_traj_workspace_bytes(ctx, C.byref(tp)))


def md_traj_forward(ctx, tp: TrajParams, ws_ptr: int, obs_ptr: int):
    _check(lib().md_traj_forward(ctx, C.byref(tp), C.c_void_p(ws_ptr), C.c_void_p(obs_ptr)),
           "md_traj_forward")


def md_traj_backward(ctx, tp: TrajParams, ws_ptr: int, gobs_ptr: int, gx_ptr: int, gv_ptr: int,
                     gth_ptr: int):
    _check(lib().md_traj_backward(ctx, C.byref(tp), C.c_void_p(ws_ptr), C.c_void_p(gobs_ptr),
                                  C.c_void_p(gx_ptr), C.c_void_p(gv_ptr), C.c_void_p(gth_ptr)),
           "md_traj_backward")


def md_set_tuning(ctx, force_lanes=2, force_block=512, nl_block=0, tile_cells=0, stage_cap=0,
                  integrate_grid=0, nl_method=MD_NL_AUTO, tile_y=0, tile_z=0):
    t = Tuning(int(force_lanes), int(force_block), int(nl_block), int(tile_cells), int(stage_cap),
               int(integrate_grid), int(nl_method), int(tile_y), int(tile_z))
    _check(lib().md_set_tuning(ctx, C.byref(t)), "md_set_tuning")


def md_get_tuning(ctx) -> dict:
    t = Tuning()
    _check(lib().md_get_tuning(ctx, C.byref(t)), "md_get_tuning")
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


def md_set_timing(ctx, enable: bool):
    _check(lib().md_set_timing(ctx, int(bool(enable))), "md_set_timing")


def md_get_timing(ctx):
    ms, n = C.c_double(), C.c_int64()
    _check(lib().md_get_timing(ctx, C.byref(ms), C.byref(n)), "md_get_timing")
    return ms.value, n.value


MD_PART_NEIGHBORS, MD_PART_FORCES, MD_PART_INTEGRATE, MD_PART_ENERGY, MD_PART_CELLS, \
    MD_PART_REORDER, MD_PART_COUNT = range(7)
PART_NAMES = ("neighbors", "forces", "integrate", "energy", "cells", "reorder")


def md_get_timing_parts(ctx):
    """{part: (ms, launch groups)} of md_set_timing's per-part events."""
    ms = (C.c_double * MD_PART_COUNT)()
    n = (C.c_int64 * MD_PART_COUNT)()
    _check(lib().md_get_timing_parts(ctx, ms, n), "md_get_timing_parts")
    return {PART_NAMES[k]: (ms[k], n[k]) for k in range(MD_PART_COUNT)}


def md_destroy(ctx):
    lib().md_destroy(ctx)


# ---- one system ------------------------------------------------------------

class Simulation:
    """One periodic system on one GPU: tensors, context, and the calls in order.

    pos, vel: (N, 3) arrays in id order.  All per-atom tensors are float64
    except the forces in FP32-mixed mode (float32).  pipeline: "tiled",
    "layers" (the paper's own steps) or "allpairs" (every pair, no cells);
    bonded: None, or md_set_bonded's keywords (chain_length, fene_k, fene_r0,
    bend_k, tors_c) for linear chains of consecutive ids.
    """

    def __init__(self, pos, vel, L, *, r_cut, dt, skin=0.3, eps=1.0, sigma=1.0, mass=1.0,
                 shifted=True, precision="fp64", neighbor_list=True, reorder=None,
                 newton3=False, nl_capacity=0, block=256, pipeline="tiled", bonded=None,
                 device="cuda", stream=None, static_workspace=False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libmd needs a GPU; none is visible")
        lib()
        if not isinstance(pos, torch.Tensor):
            pos = np.asarray(pos, dtype=np.float64)
        if not isinstance(vel, torch.Tensor):
            vel = np.asarray(vel, dtype=np.float64)
        n = pos.shape[0]
        pipe = {"tiled": MD_PIPE_TILED, "layers": MD_PIPE_LAYERS,
                "allpairs": MD_PIPE_ALLPAIRS}[pipeline]
        if pipe == MD_PIPE_ALLPAIRS:
            neighbor_list = False  # no cells and no list: every pair is tested
        if reorder is None:
            reorder = bool(neighbor_list) and pipe == MD_PIPE_TILED
        if pipe == MD_PIPE_LAYERS:
            # the interval in steps of the layer pipeline's reorder (True: the
            # paper's 100), 0 for none
            reorder = 100 if reorder is True else int(reorder or 0)
        else:
            reorder = int(bool(reorder))
        self.params = Params(int(n), MD_LJ_SHIFTED if shifted else MD_LJ_TRUNC, float(L),
                             float(eps), float(sigma), float(mass), float(r_cut), float(skin),
                             float(dt), MD_FP64 if precision == "fp64" else MD_FP32_MIXED,
                             MD_NEIGHBOR_LIST if neighbor_list else MD_CELLS_ONLY,
                             int(bool(newton3)), int(nl_capacity), reorder,
                             int(block), pipe)
        self.n = n
        self.L = float(L)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = md_init(self.params)
        if bonded is not None:  # dict of md_set_bonded's keywords
            md_set_bonded(self.ctx, **bonded)
        self._tuning = None
        self.grid = md_geometry(self.ctx)
        def t(a):
            if isinstance(a, torch.Tensor):
                return a.detach().to(device=self.device, dtype=torch.float64).contiguous().clone()
            return torch.as_tensor(np.ascontiguousarray(a), device=self.device)
        self.x, self.y, self.z = (t(pos[:, k]) for k in range(3))
        self.vx, self.vy, self.vz = (t(vel[:, k]) for k in range(3))
        fdt = torch.float64 if precision == "fp64" else torch.float32
        self.fx, self.fy, self.fz = (torch.zeros(n, dtype=fdt, device=self.device)
                                     for _ in range(3))
        self.id = torch.arange(n, dtype=torch.int32, device=self.device)
        state = [v.data_ptr() for v in (self.x, self.y, self.z, self.vx, self.vy, self.vz,
                                         self.fx, self.fy, self.fz, self.id)]
        self.static_workspace = bool(static_workspace)
        if self.static_workspace:
            # the library's own workspace array: nothing allocated for it here
            self.workspace = None
            self._ws_shift = 0
            torch.cuda.synchronize(self.device)
            md_bind_static(self.ctx, Buffers(*state, None), self.stream.cuda_stream)
            return
        nbytes = md_workspace_bytes(self.ctx)
        # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_shift = (-base) % 256
        bufs = Buffers(*state, base + self._ws_shift)
        torch.cuda.synchronize(self.device)
        md_bind(self.ctx, bufs, self.stream.cuda_stream)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                md_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    # -- the calls, in the paper's order
    def build_cells(self):
        md_build_cells(self.ctx)

    def build_neighbors(self):
        md_build_neighbors(self.ctx)

    def forces(self):
        md_forces(self.ctx)

    def prepare(self):
        """Cells, list (if any) and forces for the current state."""
        self.build_cells()
        if self.params.mode == MD_NEIGHBOR_LIST:
            self.build_neighbors()
        self.forces()

    def step(self, n_steps, record_every=0):
        md_step(self.ctx, n_steps, record_every)

    # -- reverse mode
    def traj_forward(self, n_steps, checkpoint_every=20, n_bins=0, gr_rmax=2.5, gr_width=None):
        """Run n_steps keeping checkpoints; returns the observables (device
        float64 tensor [1 + n_bins]: mean energy per atom over the steps, then
        the soft g(r) of the last positions).  Needs reorder=False."""
        import torch

        tp = traj_params(n_steps, checkpoint_every, n_bins, gr_rmax, gr_width)
        nbytes = md_traj_workspace_bytes(self.ctx, tp)
        if nbytes == 0:
            raise MDError(-1, "md_traj_workspace_bytes")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        wp = ws.data_ptr() + (-ws.data_ptr()) % 256
        obs = torch.empty(1 + tp.n_bins, dtype=torch.float64, device=self.device)
        md_traj_forward(self.ctx, tp, wp, obs.data_ptr())
        self._traj = (tp, ws, wp)
        return obs

    def traj_backward(self, grad_obs):
        """dL/dx0 [n,3], dL/dv0 [n,3], dL/d(eps, sigma) [2] for dL/dobs =
        grad_obs, after traj_forward (storage order; reorder=False keeps it
        the input order)."""
        import torch

        if getattr(self, "_traj", None) is None:
            raise RuntimeError("traj_backward needs a traj_forward first")
        tp, ws, wp = self._traj
        gobs = grad_obs.detach().to(device=self.device, dtype=torch.float64).contiguous()
        if gobs.numel() != 1 + tp.n_bins:
            raise ValueError("grad_obs must hold 1 + n_bins values")
        gx = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        gv = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        gth = torch.empty(2, dtype=torch.float64, device=self.device)
        md_traj_backward(self.ctx, tp, wp, gobs.data_ptr(), gx.data_ptr(), gv.data_ptr(),
                         gth.data_ptr())
        return gx.t().contiguous(), gv.t().contiguous(), gth

    def reduce(self, check=True) -> dict:
        o = md_reduce(self.ctx, check=check)
        return {"U": o.U, "K": o.K, "W": o.W, "P": np.array(o.P[:]), "T": o.T,
                "pressure": o.pressure, "dmax": o.dmax, "step": o.step,
                "n_rebuilds": o.n_rebuilds, "max_occupancy": o.max_occupancy,
                "max_nl": o.max_nl, "flags": o.flags}

    def history(self):
        recs = md_history(self.ctx)
        dt = np.dtype([("step", "i8"), ("U", "f8"), ("K", "f8"), ("W", "f8"), ("P", "f8", 3),
                       ("dmax", "f8"), ("rebuilt", "i4")])
        out = np.zeros(len(recs), dt)
        for k, r in enumerate(recs):
            out[k] = (r.step, r.U, r.K, r.W, tuple(r.P), r.dmax, r.rebuilt)
        return out

    def set_tuning(self, **kw):
        """Change some launch-shape settings; the others keep their last
        requested values (nl_block, tile_cells, tile_y, tile_z, stage_cap and
        integrate_grid start automatic, 0)."""
        if self._tuning is None:
            self._tuning = md_get_tuning(self.ctx)
            self._tuning.update(nl_block=0, tile_cells=0, stage_cap=0, integrate_grid=0,
                                nl_method=MD_NL_AUTO, tile_y=0, tile_z=0)
        req = dict(self._tuning)
        req.update(kw)
        md_set_tuning(self.ctx, **req)
        self._tuning = req

    def get_tuning(self):
        return md_get_tuning(self.ctx)

    def autotune(self, candidates, reps=3, cache_path=None):
        """md_autotune: time each candidate shape (dicts of md_tuning fields)
        on the current state and keep the cheapest (cells, list and forces
        rebuilt for it); returns (index, costs in ms).  With cache_path, a
        cached choice for this system, candidate list and device is taken
        instead (costs -1) and a new one is stored."""
        arr = (Tuning * len(candidates))(*[_tuning_tuple(c) for c in candidates])
        ms = (C.c_double * len(candidates))()
        best = C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().md_autotune(self.ctx, arr, len(candidates), int(reps), path, ms,
                                 C.byref(best)), "md_autotune")
        self._tuning = dict(candidates[best.value]) if best.value >= 0 else None
        return best.value, list(ms)

    def set_timing(self, enable=True):
        md_set_timing(self.ctx, enable)

    def set_graph(self, enable=True):
        _check(lib().md_set_graph(self.ctx, int(bool(enable))), "md_set_graph")

    def get_timing(self):
        return md_get_timing(self.ctx)

    def get_timing_parts(self):
        return md_get_timing_parts(self.ctx)

    # -- views of the device state
    def ws_array(self, which, dtype):
        import torch

        if self.workspace is None:
            raise RuntimeError("the workspace of a static binding is not addressable")
        off, cnt = md_layout(self.ctx, which)
        es = torch.empty((), dtype=dtype).element_size()
        start = self._ws_shift + off
        return self.workspace[start:start + cnt * es].view(dtype)

    def _host(self, *ts):
        self.stream.synchronize()
        return [t.cpu().numpy() for t in ts]

    def ids(self):
        return self._host(self.id)[0]

    def state(self):
        """Positions, velocities, forces (float64) in id order."""
        x, y, z, vx, vy, vz, fx, fy, fz, ids = self._host(self.x, self.y, self.z, self.vx,
                                                          self.vy, self.vz, self.fx, self.fy,
                                                          self.fz, self.id)
        inv = np.empty(self.n, np.int64)
        inv[ids] = np.arange(self.n)
        pos = np.stack([x, y, z], 1)[inv]
        vel = np.stack([vx, vy, vz], 1)[inv]
        f = np.stack([fx, fy, fz], 1).astype(np.float64)[inv]
        return {"pos": pos, "vel": vel, "f": f}

    def cells(self):
        """Cell arrays in slot space plus the slot -> id map."""
        import torch

        co = self.ws_array(MD_ARR_CELL_OF, torch.int32)
        cs = self.ws_array(MD_ARR_CELL_START, torch.int32)
        ca = self.ws_array(MD_ARR_CELL_ATOMS, torch.int32)
        cell_of, cell_start, cell_atoms, ids = self._host(co, cs, ca, self.id)
        return {"cell_of": cell_of, "cell_start": cell_start, "cell_atoms": cell_atoms,
                "id": ids}

    def layers(self):
        """The layer matrix [n_cells, n_layers] and the atoms per cell
        (MD_PIPE_LAYERS), host copies."""
        import torch

        h = self.ws_array(MD_ARR_LAYERS, torch.int32)
        c = self.ws_array(MD_ARR_LAYER_COUNT, torch.int32)
        h_h, c_h = self._host(h, c)
        return h_h.reshape(self.grid.n_cells, self.grid.n_layers), c_h

    def nl_counts(self):
        """List length per slot (host copy)."""
        import torch

        return self._host(self.ws_array(MD_ARR_NL_COUNT, torch.int32))[0]

    def neighbor_list(self):
        """(count[n], nl[cap, n_pad]) in slot space, decoded by md_export_neighbors."""
        import torch

        out = torch.empty(self.grid.nl_capacity * self.grid.n_pad, dtype=torch.int32,
                          device=self.device)
        md_export_neighbors(self.ctx, out.data_ptr())
        cnt = self.ws_array(MD_ARR_NL_COUNT, torch.int32)
        nl_h, cnt_h = self._host(out, cnt)
        return cnt_h, nl_h.reshape(self.grid.nl_capacity, self.grid.n_pad)


# ---- batched replicas ------------------------------------------------------

def md_batch_init(params, n):
    arr = (Params * n)(*params)
    b = C.c_void_p()
    _check(lib().md_batch_init(arr, int(n), C.byref(b)), "md_batch_init")
    return b


def md_batch_replica(b, r):
    c = C.c_void_p()
    _check(lib().md_batch_replica(b, int(r), C.byref(c)), "md_batch_replica")
    return c


def _tuning_tuple(t: dict):
    return Tuning(int(t.get("force_lanes", 2)), int(t.get("force_block", 512)),
                  int(t.get("nl_block", 0)), int(t.get("tile_cells", 0)),
                  int(t.get("stage_cap", 0)), int(t.get("integrate_grid", 0)),
                  int(t.get("nl_method", MD_NL_AUTO)), int(t.get("tile_y", 0)),
                  int(t.get("tile_z", 0)))


class Batch:
    """Independent replicas advanced together (md_batch_*).

    ``systems`` is a list of dicts with keys pos, vel, L, r_cut, dt and
    optionally skin, eps, sigma, mass, shifted.  The state lives in one
    concatenated float64 tensor per component (replica r owns the slice
    [offsets[r], offsets[r+1])); the batch runs on its own stream so that a
    run can be captured into a HIP graph."""

    def __init__(self, systems, *, precision="fp32", neighbor_list=True, reorder=None,
                 newton3=False, block=256, device="cuda"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libmd needs a GPU; none is visible")
        lib()
        if reorder is None:
            reorder = bool(neighbor_list)
        self.device = torch.device(device)
        self.R = len(systems)
        self.sizes = [len(sy["pos"]) for sy in systems]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        params = []
        for sy in systems:
            params.append(Params(len(sy["pos"]), MD_LJ_SHIFTED if sy.get("shifted", True)
                                 else MD_LJ_TRUNC, float(sy["L"]), float(sy.get("eps", 1.0)),
                                 float(sy.get("sigma", 1.0)), float(sy.get("mass", 1.0)),
                                 float(sy["r_cut"]), float(sy.get("skin", 0.3)), float(sy["dt"]),
                                 MD_FP64 if precision == "fp64" else MD_FP32_MIXED,
                                 MD_NEIGHBOR_LIST if neighbor_list else MD_CELLS_ONLY,
                                 int(bool(newton3)), int(sy.get("nl_capacity", 0)),
                                 int(bool(reorder)), int(block)))
        self.params = params
        self.ctx = md_batch_init(params, self.R)
        self.replicas = [md_batch_replica(self.ctx, r) for r in range(self.R)]
        pos = np.concatenate([np.asarray(sy["pos"], np.float64) for sy in systems])
        vel = np.concatenate([np.asarray(sy["vel"], np.float64) for sy in systems])
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=self.device)
        self.x, self.y, self.z = (t(pos[:, k]) for k in range(3))
        self.vx, self.vy, self.vz = (t(vel[:, k]) for k in range(3))
        fdt = torch.float64 if precision == "fp64" else torch.float32
        ntot = int(self.offsets[-1])
        self.fx, self.fy, self.fz = (torch.zeros(ntot, dtype=fdt, device=self.device)
                                     for _ in range(3))
        self.id = torch.cat([torch.arange(n, dtype=torch.int32) for n in self.sizes]).to(
            self.device)
        nbytes = int(lib().md_batch_workspace_bytes(self.ctx))
        self.workspace = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        wp = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        bufs = (Buffers * self.R)()
        for r in range(self.R):
            o = int(self.offsets[r])
            ptr = lambda ten: ten.data_ptr() + o * ten.element_size()
            bufs[r] = Buffers(*[ptr(v) for v in (self.x, self.y, self.z, self.vx, self.vy,
                                                 self.vz, self.fx, self.fy, self.fz, self.id)],
                              0)
        self.stream = torch.cuda.Stream(self.device)
        torch.cuda.synchronize(self.device)
        _check(lib().md_batch_bind(self.ctx, bufs, C.c_void_p(wp),
                                   C.c_void_p(self.stream.cuda_stream)), "md_batch_bind")
        self._tuning = None

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.stream.synchronize()
                lib().md_batch_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def prepare(self):
        _check(lib().md_batch_prepare(self.ctx), "md_batch_prepare")

    def forces(self):
        _check(lib().md_batch_forces(self.ctx), "md_batch_forces")

    def nl_counts(self, r):
        """List length per slot of replica r (host copy)."""
        import torch

        off, cnt = C.c_size_t(), C.c_size_t()
        _check(lib().md_batch_layout(self.ctx, int(r), MD_ARR_NL_COUNT, C.byref(off),
                                     C.byref(cnt)), "md_batch_layout")
        base = (-self.workspace.data_ptr()) % 256 + off.value
        v = self.workspace[base: base + 4 * cnt.value].view(torch.int32)
        self.stream.synchronize()
        return v.cpu().numpy()

    def run(self, n_steps, record_every=0, graph=True):
        _check(lib().md_batch_run(self.ctx, int(n_steps), int(record_every), int(bool(graph))),
               "md_batch_run")

    def synchronize(self):
        self.stream.synchronize()

    def set_tuning(self, **kw):
        if self._tuning is None:
            self._tuning = self.get_tuning()
            self._tuning.update(nl_block=0, tile_cells=0, stage_cap=0, integrate_grid=0,
                                nl_method=MD_NL_AUTO, tile_y=0, tile_z=0)
        req = dict(self._tuning)
        req.update(kw)
        t = _tuning_tuple(req)
        _check(lib().md_batch_set_tuning(self.ctx, C.byref(t)), "md_batch_set_tuning")
        self._tuning = req

    def get_tuning(self):
        t = Tuning()
        _check(lib().md_batch_get_tuning(self.ctx, C.byref(t)), "md_batch_get_tuning")
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def autotune(self, candidates, reps=3, cache_path=None):
        """Time each candidate shape (dicts of md_tuning fields) and keep the
        cheapest; returns (index, costs in ms).  With cache_path, a cached
        choice for this batch, candidate list and device is taken instead
        (costs -1) and a new one is stored."""
        arr = (Tuning * len(candidates))(*[_tuning_tuple(c) for c in candidates])
        ms = (C.c_double * len(candidates))()
        best = C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().md_batch_autotune(self.ctx, arr, len(candidates), int(reps), path, ms,
                                       C.byref(best)), "md_batch_autotune")
        self._tuning = dict(candidates[best.value]) if best.value >= 0 else self.get_tuning()
        return best.value, list(ms)

    # -- per replica
    def reduce(self, r, check=True) -> dict:
        o = md_reduce(self.replicas[r], check=check)
        return {"U": o.U, "K": o.K, "W": o.W, "P": np.array(o.P[:]), "T": o.T,
                "pressure": o.pressure, "dmax": o.dmax, "step": o.step,
                "n_rebuilds": o.n_rebuilds, "flags": o.flags}

    def history(self, r):
        recs = md_history(self.replicas[r])
        dt = np.dtype([("step", "i8"), ("U", "f8"), ("K", "f8"), ("W", "f8"), ("P", "f8", 3),
                       ("dmax", "f8"), ("rebuilt", "i4")])
        out = np.zeros(len(recs), dt)
        for k, rec in enumerate(recs):
            out[k] = (rec.step, rec.U, rec.K, rec.W, tuple(rec.P), rec.dmax, rec.rebuilt)
        return out

    def state(self, r):
        """Positions, velocities, forces of replica r (float64) in id order."""
        self.stream.synchronize()
        a, b = int(self.offsets[r]), int(self.offsets[r + 1])
        x, y, z, vx, vy, vz, fx, fy, fz, ids = [t[a:b].cpu().numpy() for t in (
            self.x, self.y, self.z, self.vx, self.vy, self.vz, self.fx, self.fy, self.fz,
            self.id)]
        inv = np.empty(b - a, np.int64)
        inv[ids] = np.arange(b - a)
        return {"pos": np.stack([x, y, z], 1)[inv], "vel": np.stack([vx, vy, vz], 1)[inv],
                "f": np.stack([fx, fy, fz], 1).astype(np.float64)[inv]}
