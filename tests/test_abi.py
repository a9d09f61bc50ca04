"""The C ABI: libmd.so loads, exports every function include/md.h declares,
and its host-only calls (validation, derived geometry, workspace layout)
behave as documented.  No device work is done here."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2003_14061_amd import inputs
from paper_2003_14061_amd import md

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(md_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = md.lib()
    names = declared_functions()
    assert {"md_init", "md_bind", "md_build_cells", "md_build_neighbors", "md_forces",
            "md_step", "md_reduce", "md_destroy"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(md.EXPORTS) <= names


def params(**kw):
    base = dict(n=256000, rho=0.8, r_cut=2 ** (1 / 6), skin=0.3, dt=0.005)
    base.update(kw)
    L = inputs.box_length(base["n"], base["rho"])
    return md.Params(base["n"], md.MD_LJ_SHIFTED, L, 1.0, 1.0, 1.0, base["r_cut"], base["skin"],
                     base["dt"], base.get("precision", md.MD_FP64),
                     base.get("mode", md.MD_NEIGHBOR_LIST), base.get("newton3", 0),
                     base.get("cap", 0),
                     base.get("reorder", 1), base.get("block", 256), base.get("pipeline", 0))


def test_geometry_of_the_workloads():
    cases = [
        (dict(n=4000, rho=0.8, mode=md.MD_CELLS_ONLY), 15),
        (dict(n=256000, rho=0.8), 48),
        (dict(n=2048000, rho=0.8442, r_cut=2.5), 47),
        (dict(n=32000, rho=0.8, r_cut=2.5), 12),
    ]
    for kw, nc in cases:
        p = params(**kw)
        ctx = md.md_init(p)
        try:
            g = md.md_geometry(ctx)
            assert g.nc == nc
            assert g.n_cells == nc ** 3
            assert g.cell_width == pytest.approx(p.L / nc)
            r_cell = p.r_cut + (p.skin if p.mode == md.MD_NEIGHBOR_LIST else 0.0)
            assert g.cell_width >= r_cell
            assert g.n_pad % 64 == 0 and g.n_pad >= p.n_atoms
            if p.mode == md.MD_NEIGHBOR_LIST:
                mean = 4 / 3 * math.pi * r_cell ** 3 * p.n_atoms / p.L ** 3
                assert g.nl_capacity > mean + 5 * math.sqrt(mean)
            ws = md.md_workspace_bytes(ctx)
            assert ws > 0
            seen = []
            for which in range(6 if p.mode == md.MD_NEIGHBOR_LIST else 5):
                off, cnt = md.md_layout(ctx, which)
                assert off % 256 == 0 and off < ws
                if cnt:
                    seen.append(off)
            assert len(set(seen)) == len(seen)
        finally:
            md.md_destroy(ctx)


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(r_cut=-1.0), dict(dt=0.0), dict(skin=-0.1), dict(block=100),
    dict(block=2048), dict(precision=7), dict(mode=3), dict(reorder=2), dict(cap=-1),
    dict(newton3=2), dict(newton3=-1), dict(newton3=1, mode=md.MD_CELLS_ONLY),
    dict(pipeline=3), dict(pipeline=-1), dict(pipeline=1, reorder=-1), dict(reorder=-1),
    dict(pipeline=1, reorder=0, newton3=1), dict(pipeline=1, reorder=0, mode=md.MD_CELLS_ONLY),
    dict(pipeline=2, reorder=0), dict(pipeline=2, reorder=1, mode=md.MD_CELLS_ONLY),
    dict(pipeline=2, reorder=0, mode=md.MD_CELLS_ONLY, newton3=1),
])
def test_invalid_parameters_are_rejected(bad):
    ctx = C.c_void_p()
    st = md.lib().md_init(C.byref(params(**bad)), C.byref(ctx))
    assert st == -1 and not ctx.value


def test_batch_replica_count_is_bounded():
    """A batch holds 1 to 32768 replicas (their index shares a 16-bit table
    entry with the rebuild gate); the count is checked before anything else."""
    p = params(n=4000)
    for n in (0, 32769):
        arr = (md.Params * max(n, 1))(*([p] * max(n, 1)))
        b = C.c_void_p()
        assert md.lib().md_batch_init(arr, n, C.byref(b)) == -1 and not b.value


def test_third_law_variant_is_accepted_with_a_list():
    for prec in (md.MD_FP64, md.MD_FP32_MIXED):
        ctx = md.md_init(params(n=32000, rho=0.8, r_cut=2.5, newton3=1, precision=prec))
        md.md_destroy(ctx)


def test_layer_pipeline_geometry_and_arrays():
    """The paper's layer-matrix pipeline: layers per cell from the mean
    occupancy, a 32-bit neighbor matrix in place of the 16-bit one, and the
    layer arrays exposed through md_layout only in that pipeline."""
    for n, rho, rc in ((2048000, 0.8442, 2.5), (256000, 0.8, 2 ** (1 / 6))):
        p = params(n=n, rho=rho, r_cut=rc, reorder=0, pipeline=1)
        ctx = md.md_init(p)
        tiled = md.md_init(params(n=n, rho=rho, r_cut=rc, reorder=0))
        try:
            g = md.md_geometry(ctx)
            occ = n / g.n_cells
            assert g.n_layers == math.ceil(occ + 6 * math.sqrt(occ) + 8)
            assert md.md_geometry(tiled).n_layers == 0
            off, cnt = md.md_layout(ctx, md.MD_ARR_LAYERS)
            assert cnt == g.n_cells * g.n_layers and off % 256 == 0
            off, cnt = md.md_layout(ctx, md.MD_ARR_LAYER_COUNT)
            assert cnt == g.n_cells
            off, cnt = md.md_layout(ctx, md.MD_ARR_NL)
            assert cnt == g.nl_capacity * g.n_pad
            for which in (md.MD_ARR_CELL_START, md.MD_ARR_CELL_ATOMS):
                with pytest.raises(md.MDError):
                    md.md_layout(ctx, which)
            for which in (md.MD_ARR_LAYERS, md.MD_ARR_LAYER_COUNT):
                with pytest.raises(md.MDError):
                    md.md_layout(tiled, which)
            # the 32-bit matrix in place of the 16-bit one, which carries one
            # spare row of 4-entry chunks past the capacity
            wl = md.md_workspace_bytes(ctx) - md.md_workspace_bytes(tiled)
            assert wl >= (4 * g.nl_capacity - 2 * (g.nl_capacity + 4)) * g.n_pad + \
                4 * g.n_cells * g.n_layers
        finally:
            md.md_destroy(ctx)
            md.md_destroy(tiled)
    assert md.status_str(-8).startswith("layer matrix overflow")


def test_box_too_small():
    ctx = C.c_void_p()
    p = params(n=100, rho=0.8, r_cut=2.5)  # L = 5.0 < 3 * 2.8
    st = md.lib().md_init(C.byref(p), C.byref(ctx))
    assert st == -2 and md.status_str(st).startswith("box too small")


def test_calls_before_bind_fail_cleanly():
    ctx = md.md_init(params(n=4000, rho=0.8))
    try:
        for f in (md.lib().md_build_cells, md.lib().md_build_neighbors, md.lib().md_forces):
            assert f(ctx) == -6
        assert md.lib().md_step(ctx, 1, 0) == -6
        assert md.lib().md_step(ctx, -1, 0) == -1
        o = md.Observables()
        assert md.lib().md_reduce(ctx, C.byref(o)) == -6
    finally:
        md.md_destroy(ctx)
    assert md.lib().md_build_cells(None) == -1
    md.lib().md_destroy(None)


def test_trajectory_workspace_is_validated_on_the_host():
    ctx = md.md_init(params(n=32000, rho=0.8, r_cut=2.5, reorder=0))
    try:
        ok = md.traj_params(200, 20, 50, 2.5)
        b = md.md_traj_workspace_bytes(ctx, ok)
        n = 32000
        # 11 checkpoints of 6 arrays, 19 snapshots of 3, 9 adjoint arrays
        assert b >= (11 * 6 + 19 * 3 + 9) * 8 * n
        assert b < (11 * 6 + 19 * 3 + 9) * 8 * n + 4 * 1024 * 1024
        # an interval beyond the run is one segment: 2 checkpoints, 199 snapshots
        one = md.md_traj_workspace_bytes(ctx, md.traj_params(200, 1000))
        assert one == md.md_traj_workspace_bytes(ctx, md.traj_params(200, 200)) > b
        for bad in (md.traj_params(0, 20), md.traj_params(4097, 20), md.traj_params(10, 0),
                    md.traj_params(10, 5, 1025, 2.5), md.traj_params(10, 5, 10, 2.5, 0.0),
                    md.traj_params(10, 5, 10, -1.0, 0.1)):
            assert md.md_traj_workspace_bytes(ctx, bad) == 0
    finally:
        md.md_destroy(ctx)


def test_allpairs_pipeline_geometry_and_arrays():
    """The all-pairs comparison pipeline: cells-only box rule, no cell arrays,
    and room for one energy partial per workgroup and the chunk partials."""
    for n in (40, 4000, 100000, 256000):
        p = params(n=n, rho=0.8 if n > 40 else 0.3, mode=md.MD_CELLS_ONLY, reorder=0,
                   pipeline=2)
        ctx = md.md_init(p)
        try:
            g = md.md_geometry(ctx)
            assert g.nc >= 3 and g.cell_width >= p.r_cut
            for which in (md.MD_ARR_CELL_OF, md.MD_ARR_CELL_START, md.MD_ARR_CELL_ATOMS,
                          md.MD_ARR_LAYERS, md.MD_ARR_XREF):
                with pytest.raises(md.MDError):
                    md.md_layout(ctx, which)
            # home blocks of 64 atoms times partner chunks of whole 256-atom tiles;
            # the chunk partials: 3 force components per chunk and padded atom
            blocks = -(-n // 64)
            tiles = -(-n // 256)
            split = max(1, min(-(-2048 // blocks), tiles))
            chunk = -(-(-(-n // split)) // 256) * 256
            split = -(-n // chunk)
            need = 16 * blocks * split + (24 * split * g.n_pad if split > 1 else 0)
            assert md.md_workspace_bytes(ctx) >= need
        finally:
            md.md_destroy(ctx)
    # too small a box for a unique minimum image at this cutoff
    ctx = C.c_void_p()
    bad = params(n=20, rho=0.8, mode=md.MD_CELLS_ONLY, reorder=0, pipeline=2)
    assert md.lib().md_init(C.byref(bad), C.byref(ctx)) == -2


def test_bonded_chains_are_validated_and_grow_the_workspace():
    p = params(n=4096, rho=0.85, reorder=1)
    ctx = md.md_init(p)
    try:
        base = md.md_workspace_bytes(ctx)
        lib = md.lib()
        bad = [dict(chain_length=1), dict(chain_length=3),  # 4096 is not a multiple of 3
               dict(chain_length=16, fene_r0=0.0), dict(chain_length=16, fene_k=-1.0),
               dict(chain_length=16, bend_k=float("nan"))]
        for kw in bad:
            args = dict(fene_k=30.0, fene_r0=1.5, bend_k=0.0)
            args.update(kw)
            b = md.Bonded(args["chain_length"], 0, args["fene_k"], args["fene_r0"],
                          args["bend_k"], (C.c_double * 4)(0, 0, 0, 0))
            assert lib.md_set_bonded(ctx, C.byref(b)) == -1, kw
        md.md_set_bonded(ctx, chain_length=16, bend_k=1.5, tors_c=(0.1, 0.2, 0.3, 0.4))
        grown = md.md_workspace_bytes(ctx)
        # an id-to-slot map and two partials per 256-atom workgroup, 256-byte aligned
        assert grown - base == 4 * 4096 + 16 * 16
        md.md_set_bonded(ctx, None)
        assert md.md_workspace_bytes(ctx) == base
    finally:
        md.md_destroy(ctx)
