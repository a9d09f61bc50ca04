"""Throughput of the MD hot path on one MI355X: atom-steps per second.

Workload (default): Lennard-Jones cut and shifted at r_c = 2.5 sigma,
N = 2,048,000 atoms from an 80^3 FCC lattice at density 0.8442, T = 0.72,
dt = 0.004, neighbor list with skin 0.3 sigma rebuilt when an atom has moved
more than skin/2, atoms reordered by cell at every rebuild.  One "step" is a
whole leapfrog step: kick, drift, rebuild when needed (cells + list),
forces, kick, and the device-side reductions.  The FP64 path gives `value`;
the FP32-mixed path is measured on the same input and reported beside it.

Prints one JSON line.  With --gpus above 1 it exits: the build targets one
GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/sec at N=2.05M LJ (FP64 vs FP32-mixed); adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6   # MI355X dense FP64 vector
# FP32 vector: the published 157.3 TFLOP/s counts packed FP32 (two lanes per
# instruction), which this build switches off, so plain FP32 issues at the
# FP64 rate
FP32_PEAK_TFS = 78.6
FORCE_SOURCES = ("paper_2003_14061_amd/csrc/md_forces.hip", "paper_2003_14061_amd/csrc/md_tiles.h",
                 "paper_2003_14061_amd/csrc/md_pair.h",
                 "paper_2003_14061_amd/csrc/md_device.h", "paper_2003_14061_amd/csrc/md_internal.h")
PROFILES = "profiles"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="lj_2048k")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=24,
                    help="steps of the CPU oracle sample (from the melted FP64 GPU state; "
                         "the list is rebuilt about every 11 steps there)")
    ap.add_argument("--drift-steps", type=int, default=1000,
                    help="untimed steps after the timed ones, energy recorded every 10, "
                         "for the energy-drift slope")
    ap.add_argument("--batch-steps", type=int, default=500,
                    help="steps of the batched ensemble's timed graph launch")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 4000-atom cells-only and 256 000-atom WCA lines")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-mixed measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--tune-cache",
                    default=os.path.join(os.path.expanduser("~"), ".cache",
                                         "paper_2003_14061_amd", "tuning.json"),
                    help="JSON file of autotuned launch shapes ('' for none)")
    ap.add_argument("--batch-tuning", default="",
                    help="JSON object of md_tuning fields: the batch runs with this shape "
                         "instead of autotuning (for profiling)")
    ap.add_argument("--no-newton3", action="store_true",
                    help="skip the third-law (half list, atomic) variant")
    ap.add_argument("--no-layers", action="store_true",
                    help="skip the paper's layer-matrix pipeline (thread-per-atom kernels)")
    ap.add_argument("--no-allpairs", action="store_true",
                    help="skip the all-pairs comparison on the 4000-atom WCA system")
    ap.add_argument("--no-polymer", action="store_true",
                    help="skip the bonded polymer melt (262 144 atoms in chains of 64)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio of the differentiable run")
    ap.add_argument("--no-main", action="store_true",
                    help="skip the FP64 headline leg (profiling runs of the other legs only)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    return ap.parse_args()


def force_bytes_per_atom(mean_nl, precision):
    """Algorithmic HBM bytes of one force pass per atom: the list row
    (2 B per 16-bit entry) and its length (4 B), the atom's own position
    (24 B), and the force written back (24 B in FP64, 12 B in FP32)."""
    return 2.0 * mean_nl + 4.0 + 24.0 + (24.0 if precision == "fp64" else 12.0)


def force_flops_per_atom(mean_nl, mean_in_range):
    """Algorithmic floating-point operations of one force pass per atom:
    8 per list entry (separation and squared distance) and 19 per pair
    inside the cutoff (reciprocal, powers, force, energy and virial sums)."""
    return 8.0 * mean_nl + 19.0 * mean_in_range


def force_sources_hash():
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_atoms, precision, kernel="k_forces_tiles"):
    """HBM bytes per force-pass launch from a committed rocprofv3 counter
    summary (profiles/*_traffic.txt) for this kernel, atom count and
    precision, taken on the current kernel sources; None when there is none."""
    d = os.path.join(ROOT, PROFILES)
    if not os.path.isdir(d):
        return None
    h = force_sources_hash()
    for name in sorted(os.listdir(d)):
        if not name.endswith("_traffic.txt"):
            continue
        kv = {}
        with open(os.path.join(d, name)) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        try:
            if (kv.get("sources_sha256") == h and int(kv.get("n_atoms", -1)) == n_atoms and
                    kv.get("precision") == precision and
                    kv.get("kernel", "").split("<")[0].endswith(kernel)):
                return float(kv["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def energy_drift(sim, w, steps, every=10):
    """Total energy per atom over `steps` further steps, recorded every
    `every`: least-squares slope per unit time, RMS about the line, and the
    change end to start."""
    import numpy as np

    if steps <= 0:
        return None
    sim.step(steps, record_every=every)
    h = sim.history()
    if len(h) < 3:
        return None
    t = h["step"].astype(np.float64) * w.dt
    e = (h["U"] + h["K"]) / w.n
    slope, icpt = np.polyfit(t - t[0], e, 1)
    resid = e - (icpt + slope * (t - t[0]))
    return {"steps": int(steps), "records": int(len(h)), "every": every,
            "slope_per_atom_per_time": float(slope),
            "rms_about_fit_per_atom": float(np.sqrt(np.mean(resid ** 2))),
            "change_per_atom": float(e[-1] - e[0]), "e_per_atom_start": float(e[0])}


def run_gpu(w, precision, steps, warmup, newton3=False, pipeline="tiled", detail=True,
            drift_steps=0, keep_state=False, reorder=None):
    import torch

    from paper_2003_14061_amd import md

    sim = md.Simulation(w.pos, w.vel, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt,
                        shifted=w.shifted, precision=precision, neighbor_list=w.use_nl,
                        newton3=newton3, pipeline=pipeline, reorder=reorder)
    sim.prepare()
    sim.step(warmup)
    o0 = sim.reduce()
    e0 = (o0["U"] + o0["K"]) / w.n
    # the timed run: md_step as it runs by default (direct launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    o1 = sim.reduce()
    e1 = (o1["U"] + o1["K"]) / w.n
    # the same number of steps replayed from md_step's HIP graph (runs of 32
    # steps, captured by a first short run), for comparison
    sim.set_graph(True)
    sim.step(40)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    graphed = w.n * steps / (t3 - t2)
    sim.set_graph(False)
    # and again with every part of each step bracketed by HIP events on the
    # bound stream: the force kernel's average duration and the split of a
    # step's time over its parts (the rows of the paper's Table 2)
    sim.set_timing(True)
    sim.step(steps)
    f_ms, f_launches = sim.get_timing()
    parts = sim.get_timing_parts()
    sim.set_timing(False)
    tot = sum(ms for ms, _ in parts.values())
    split = {k: {"us_per_step": round(1e3 * ms / steps, 2),
                 "pct": round(100.0 * ms / tot, 1) if tot > 0 else None}
             for k, (ms, _) in parts.items()}
    if not detail:
        wall = t1 - t0
        res = {"value": w.n * steps / wall, "ms_per_step": 1e3 * wall / steps,
               "value_graph_replays": graphed,
               "force_ms_avg": f_ms / max(f_launches, 1), "energy_drift_per_atom": e1 - e0,
               "rebuilds": int(o1["n_rebuilds"] - o0["n_rebuilds"]), "parts": split}
        res["energy_drift"] = energy_drift(sim, w, drift_steps)
        del sim
        torch.cuda.synchronize()
        return res
    cnt = sim.nl_counts()
    mean_nl = float(cnt[: w.n].mean())
    mean_in_range = in_range_pairs(sim, w)
    wall = t1 - t0
    res = {
        "value": w.n * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "value_graph_replays": graphed,
        "force_ms_avg": f_ms / max(f_launches, 1),
        "force_launches": f_launches,
        "mean_nl": mean_nl,
        "rebuilds": int(o1["n_rebuilds"] - o0["n_rebuilds"]),
        "energy_drift_per_atom": e1 - e0,
        "T_end": o1["T"],
        "parts": split,
    }
    bpa = force_bytes_per_atom(mean_nl, precision)
    t_force = res["force_ms_avg"] * 1e-3
    achieved = bpa * w.n / t_force / 1e9
    flops = force_flops_per_atom(mean_nl, mean_in_range) * w.n / t_force / 1e12
    alu_peak = FP64_PEAK_TFS if precision == "fp64" else FP32_PEAK_TFS
    res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": measured_traffic(w.n, precision),
                       "kernel": "k_forces_tiles", "bytes_per_atom": round(bpa, 2),
                       "units_per_launch": w.n,
                       "alu": {"achieved": round(flops, 2), "peak": alu_peak, "unit": "TFLOP/s",
                               "frac": round(flops / alu_peak, 4),
                               "flops_per_atom": round(force_flops_per_atom(mean_nl,
                                                                            mean_in_range), 1)}}
    res["mean_in_range"] = mean_in_range
    st = sim.state()
    res["final_pos"] = st["pos"]
    if keep_state:
        res["final_vel"] = st["vel"]
    res["energy_drift"] = energy_drift(sim, w, drift_steps)
    del sim
    torch.cuda.synchronize()
    return res


def error_fp32(w, pos, vel):
    """Per-step error of the FP32-mixed path, observable by observable: its
    forces, U, W, K, T and pressure against the FP64 path's on the same state
    (the state the FP64 run ended in).  The FP64 path itself matches the FP64
    oracle to 1e-12 (the parity tests, also at this size); forces per atom
    relative to the largest FP64 force and normwise, the scalars relative."""
    import numpy as np
    import torch

    from paper_2003_14061_amd import md

    f, o = {}, {}
    for prec in ("fp64", "fp32"):
        sim = md.Simulation(pos, vel, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt,
                            shifted=w.shifted, precision=prec)
        sim.prepare()
        f[prec] = sim.state()["f"]
        o[prec] = sim.reduce()
        del sim
        torch.cuda.synchronize()
    d = np.linalg.norm(f["fp32"] - f["fp64"], axis=1)
    scale = float(np.linalg.norm(f["fp64"], axis=1).max())
    out = {"F_max_per_atom_rel_to_max_force": float(d.max() / scale),
           "F_normwise": float(np.linalg.norm(f["fp32"] - f["fp64"]) /
                               np.linalg.norm(f["fp64"]))}
    for k in ("U", "W", "K", "T", "pressure"):
        out[k + "_rel"] = float(abs(o["fp32"][k] - o["fp64"][k]) / abs(o["fp64"][k]))
    return out


# FP64 lane operations the all-pairs test needs per ordered pair: three
# differences, the minimum image (multiply, round, multiply, subtract) per
# coordinate, the squared length (a multiply and two fused multiply-adds) and
# the cutoff compare; a fused multiply-add counts as one operation.
ALLPAIRS_OPS_PER_PAIR = 3 + 3 * 4 + 3 + 1
# FP64 lane-operation issue rate: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz
FP64_LANE_OPS_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def run_allpairs():
    """The paper's all-pairs comparison (section 4.2, alternative (2); it
    quotes N=4096 soft spheres): WCA, rho 0.8, T 1, dt 0.005 on N = 4000
    (10^3 FCC), 32 000 and 256 000.  The all-pairs pipeline against the tiled
    list pipeline and the layer-matrix pipeline (skin 0.3) on the same
    system, FP64.  The all-pairs force time per launch covers its two kernels
    (the pair pass and, with several partner chunks, the combine)."""
    from paper_2003_14061_amd import inputs

    def leg(r):
        return {"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 6),
                "force_ms_avg": round(r["force_ms_avg"], 6)}

    out = []
    for n, steps, warmup in ((4000, 2000, 100), (32000, 200, 20), (256000, 6, 2)):
        w_ap = inputs.preset("wca_4000", n=n).materialize()
        w_nl = inputs.preset("wca_4000", n=n, use_nl=True).materialize()
        ap = run_gpu(w_ap, "fp64", steps, warmup, pipeline="allpairs", detail=False)
        tl = run_gpu(w_nl, "fp64", steps, warmup, detail=False)
        ly = run_gpu(w_nl, "fp64", steps, warmup, pipeline="layers", detail=False)
        t = ap["force_ms_avg"] * 1e-3
        ops = ALLPAIRS_OPS_PER_PAIR * n * (n - 1) / t / 1e12
        out.append({
            "n": n, "steps": steps,
            "allpairs": dict(leg(ap), pairs_per_s=round(n * (n - 1) / t, 1),
                             roofline={"bound": "alu",
                                       "kernels": "k_forces_allpairs + k_ap_combine",
                                       "achieved": round(ops, 3),
                                       "peak": round(FP64_LANE_OPS_PEAK_TOPS, 2),
                                       "unit": "TOP/s (FP64 lane operations)",
                                       "frac": round(ops / FP64_LANE_OPS_PEAK_TOPS, 4),
                                       "ops_per_pair": ALLPAIRS_OPS_PER_PAIR,
                                       "units_per_launch": n * (n - 1)}),
            "tiled_list": leg(tl),
            "layer_matrix": leg(ly),
            "allpairs_slowdown_vs_tiled": round(tl["value"] / ap["value"], 2),
            "allpairs_slowdown_vs_layers": round(ly["value"] / ap["value"], 2),
        })
        print(f"[bench] all-pairs N={n}: {ap['value']:.3e} atom-steps/s, "
              f"{tl['value'] / ap['value']:.2f}x slower than the tiled list",
              file=sys.stderr, flush=True)
    return {"workload": "WCA (LJ cut and shifted at r_c=2^(1/6) sigma), FCC, rho=0.8, T=1, "
                        "dt=0.005; list pipelines with skin 0.3", "by_n": out}


def run_small(drift_steps):
    """The two smaller workloads.  wca_4000: soft spheres (WCA), N=4000
    (10^3 FCC), rho 0.8, T 1, dt 0.005, cells only, 1000 steps, FP64: the
    whole state fits in L2, so the step time is launch latency.  wca_256k:
    WCA, N=256 000 (40^3 FCC), rho 0.8, T 1, dt 0.005, skin 0.3, 2000 steps,
    FP64 and FP32-mixed; the analogue of the soft-sphere rows of the paper's
    Table 1."""
    from paper_2003_14061_amd import inputs

    w1 = inputs.preset("wca_4000").materialize()
    c1 = run_gpu(w1, "fp64", 1000, 100, detail=False, drift_steps=drift_steps)
    c1 = {"workload": "wca_4000: WCA (LJ cut and shifted at 2^(1/6) sigma), N=4000 FCC, "
                      "rho=0.8, T=1, dt=0.005, cells only, FP64, 1000 steps",
          "value": round(c1["value"], 1), "us_per_step": round(1e3 * c1["ms_per_step"], 3),
          "value_graph_replays": round(c1["value_graph_replays"], 1),
          "force_us_avg": round(1e3 * c1["force_ms_avg"], 3),
          "energy_drift": c1["energy_drift"]}
    print(f"[bench] wca_4000 done: {c1['value']:.3e} atom-steps/s", file=sys.stderr, flush=True)
    w2 = inputs.preset("wca_256k").materialize()
    c2 = {"workload": "wca_256k: WCA, N=256000 FCC, rho=0.8, T=1, dt=0.005, skin 0.3, "
                      "2000 steps"}
    for prec in ("fp64", "fp32"):
        r = run_gpu(w2, prec, 2000, 100, drift_steps=drift_steps)
        c2[prec if prec == "fp64" else "fp32_mixed"] = {
            "value": round(r["value"], 1), "us_per_step": round(1e3 * r["ms_per_step"], 3),
            "value_graph_replays": round(r["value_graph_replays"], 1),
            "force_us_avg": round(1e3 * r["force_ms_avg"], 3), "rebuilds": r["rebuilds"],
            "mean_nl": round(r["mean_nl"], 2), "roofline": r["roofline"],
            "energy_drift": r["energy_drift"]}
    c2["fp32_speedup"] = round(c2["fp32_mixed"]["value"] / c2["fp64"]["value"], 3)
    print(f"[bench] wca_256k done: {c2['fp64']['value']:.3e} atom-steps/s", file=sys.stderr,
          flush=True)
    return c1, c2


POLYMER_BONDED = dict(fene_k=30.0, fene_r0=1.5, bend_k=1.5)


def run_polymer(steps=500, warmup=50):
    """Bonded chains (section 4.3, item (2)): 4096 chains of 64 atoms (64^3 =
    262 144), rho 0.85, T 1, dt 0.005, WCA between all atoms, skin 0.3, FENE
    bonds (k 30, R0 1.5) and bending k_b 1.5, FP64, tiled pipeline.  The same
    system without the bonded terms gives the bonded overhead."""
    import torch

    from paper_2003_14061_amd import inputs, md

    m = inputs.polymer_preset("melt_256k").materialize()
    out = {}
    for key, bonded in (("bonded", dict(chain_length=m.chain_length, **POLYMER_BONDED)),
                        ("pairs_only", None)):
        sim = md.Simulation(m.pos, m.vel, m.L, r_cut=m.r_cut, skin=m.skin, dt=m.dt,
                            bonded=bonded)
        sim.prepare()
        sim.step(warmup)
        o0 = sim.reduce()
        sim.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f_ms, f_n = sim.get_timing()
        sim.set_timing(False)
        o1 = sim.reduce()
        out[key] = {"value": round(m.n * steps / (t1 - t0), 1),
                    "ms_per_step": round(1e3 * (t1 - t0) / steps, 6),
                    "force_ms_avg": round(f_ms / max(f_n, 1), 6),
                    "rebuilds": int(o1["n_rebuilds"] - o0["n_rebuilds"]),
                    "energy_drift_per_atom": (o1["U"] + o1["K"] - o0["U"] - o0["K"]) / m.n}
        del sim
        torch.cuda.synchronize()
    return {"workload": "melt_256k: 4096 chains of 64 (snake-lattice start), rho=0.85, T=1, "
                        "dt=0.005, WCA r_c=2^(1/6) sigma, skin 0.3; FENE k=30, R0=1.5; bending "
                        "k_b=1.5; FP64",
            **out,
            "bonded_overhead_ms_per_step": round(out["bonded"]["ms_per_step"]
                                                 - out["pairs_only"]["ms_per_step"], 6),
            "kernels": "k_bond_map (gated with the cell rebuild) + k_bonded (thread per atom)"}


def run_adjoint(precision, repeats=3):
    """Adjoint/forward time ratio on the differentiable run: LJ r_c 2.5,
    N = 32000 (20^3 FCC, rho 0.8, T 1), dt 0.004, 200 steps, checkpoints every
    20, loss = mean potential energy per atom + sum_b (g_b - g*_b)^2 over 50
    soft g(r) bins on [0, 2.5), g* from a seeded reference run at
    (eps, sigma) = (1.05, 0.98) from the same initial state.  Forward = the
    checkpointed run with its observables (each kernel launched directly);
    backward = segment recompute plus the reverse pass.  Median of `repeats`
    timings of each."""
    import torch

    from paper_2003_14061_amd import inputs, md

    w = inputs.preset("lj_32k").materialize()
    S, k, B = 200, 20, 50

    def sim_at(eps, sigma):
        return md.Simulation(w.pos, w.vel, w.L, r_cut=2.5 * sigma, skin=w.skin, dt=w.dt,
                             eps=eps, sigma=sigma, precision=precision, reorder=False)

    target = sim_at(1.05, 0.98).traj_forward(S, k, B, 2.5)[1:]
    tf, tb = [], []
    for _ in range(repeats + 1):  # the first pass is a warm-up
        sim = sim_at(1.0, 1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obs = sim.traj_forward(S, k, B, 2.5)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gobs = torch.cat([torch.ones(1, dtype=torch.float64, device=obs.device),
                          2.0 * (obs[1:] - target)])
        gx, gv, gth = sim.traj_backward(gobs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tb.append(t2 - t1)
    tf, tb = sorted(tf[1:]), sorted(tb[1:])
    fwd, bwd = tf[len(tf) // 2], tb[len(tb) // 2]
    return {"ratio": bwd / fwd, "forward_ms": 1e3 * fwd, "backward_ms": 1e3 * bwd,
            "forward_atom_steps_per_s": w.n * S / fwd,
            "forward_us_per_step": 1e6 * fwd / S,
            "grad_eps": float(gth[0]), "grad_sigma": float(gth[1])}


def run_batch(steps=500, warmup=20, tune_cache=None, fixed_tuning=None):
    """The batched ensemble: 64 WCA replicas, N uniform on [500, 32000] and
    rho on [0.6, 0.9] (seeded), T 1, dt 0.005, skin 0.3, FP32-mixed, launch
    shape (tile block, lanes per atom, workgroup size) from the autotuner or
    from its cache file tune_cache, all replicas advanced `steps` steps by one HIP
    graph launch.  Throughput = total atoms x steps / wall time; the force
    roofline fraction uses the mean list length over all replicas and the
    batched force pass timed alone with HIP events."""
    import numpy as np
    import torch

    from paper_2003_14061_amd import inputs, md

    reps = inputs.ensemble(64, seed=4)
    systems = [dict(pos=w.pos, vel=w.vel, L=w.L, r_cut=w.r_cut, dt=w.dt, skin=w.skin)
               for w in reps]
    n_tot = sum(w.n for w in reps)
    b = md.Batch(systems, precision="fp32")
    shapes = [{}] + [dict(tile_cells=x, tile_y=y, tile_z=z) for x, y, z in (
        (4, 4, 4), (5, 5, 5), (5, 5, 4), (6, 6, 6), (8, 4, 4), (4, 4, 2), (8, 2, 2))]
    cands = [dict(force_lanes=l, force_block=fb, **t) for t in shapes for l in (1, 2)
             for fb in (128, 192, 256, 320, 512)]
    if fixed_tuning:  # a given shape instead of the autotuner (profiling runs)
        cands, best, costs = [fixed_tuning], 0, [-1.0]
        b.set_tuning(**fixed_tuning)
        b.prepare()
    else:
        if tune_cache:
            os.makedirs(os.path.dirname(os.path.abspath(tune_cache)), exist_ok=True)
        best, costs = b.autotune(cands, reps=3, cache_path=tune_cache or None)
    b.run(warmup, graph=True)  # builds the warm-up graph
    b.synchronize()
    b.run(steps, graph=True)  # capture and instantiate the timed graph once
    b.synchronize()
    t0 = time.perf_counter()
    b.run(steps, graph=True)
    b.synchronize()
    wall = time.perf_counter() - t0
    # the same steps with every kernel launched directly, for comparison
    t0 = time.perf_counter()
    b.run(steps, graph=False)
    b.synchronize()
    wall_direct = time.perf_counter() - t0
    # the force pass alone, all replicas in one launch (HIP events on the batch stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    with torch.cuda.stream(b.stream):
        ev[0].record()
        for _ in range(20):
            b.forces()
        ev[1].record()
    b.synchronize()
    f_ms = ev[0].elapsed_time(ev[1]) / 20
    mean_nl = float(np.mean(np.concatenate([b.nl_counts(r) for r in range(len(reps))])))
    bpa = force_bytes_per_atom(mean_nl, "fp32")
    achieved = bpa * n_tot / (f_ms * 1e-3) / 1e9
    flags = max(b.reduce(r)["flags"] for r in range(len(reps)))
    return {"value": n_tot * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "value_direct_launches": n_tot * steps / wall_direct,
            "n_atoms": n_tot, "replicas": len(reps), "steps": steps,
            "autotune": {"best": cands[best] if best >= 0 else b.get_tuning(),
                         "cache": tune_cache or None, "fixed": bool(fixed_tuning),
                         "cache_hit": not fixed_tuning and all(c < 0 for c in costs),
                         "costs_ms": [round(c, 4) for c in costs]},
            "force_ms_avg": round(f_ms, 5), "mean_nl": round(mean_nl, 2),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic(n_tot, "fp32"),
                         "kernel": "k_forces_tiles<Batch>", "bytes_per_atom": round(bpa, 2),
                         "units_per_launch": n_tot},
            "flags": flags}


def in_range_pairs(sim, w, sample=20000):
    """Mean number of list partners inside r_cut, on a strided sample of
    atoms (host arithmetic on the current state; counts only, for the flop
    model)."""
    import numpy as np

    pos = np.mod(sim.state()["pos"], w.L)
    idx = np.linspace(0, w.n - 1, min(sample, w.n)).astype(np.int64)
    L, rc2 = w.L, w.r_cut * w.r_cut
    tot = 0
    # cell binning of the whole box for the sample's neighborhoods
    nc = max(int(L // w.r_cut), 3)
    cell = np.clip((pos * (nc / L)).astype(np.int64), 0, nc - 1)
    key = (cell[:, 2] * nc + cell[:, 1]) * nc + cell[:, 0]
    order = np.argsort(key, kind="stable")
    start = np.searchsorted(key[order], np.arange(nc ** 3 + 1))
    for i in idx:
        cx, cy, cz = cell[i]
        js = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    c = (((cz + dz) % nc) * nc + (cy + dy) % nc) * nc + (cx + dx) % nc
                    js.append(order[start[c]:start[c + 1]])
        js = np.concatenate(js)
        d = pos[js] - pos[i]
        d -= L * np.rint(d / L)
        r2 = (d * d).sum(1)
        tot += int(((r2 < rc2) & (js != i)).sum())
    return tot / len(idx)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def run_cpu(w, steps, pos=None, vel=None):
    """The oracle on the host cores: `steps` steps of the same system from
    the given state (the melted state of the FP64 GPU run, else the FCC
    start), timed minus its initial cell/list/force build."""
    import oracle

    import numpy as np

    start = "the melted state the FP64 GPU run ended in"
    if pos is None:
        pos, vel, start = w.pos, w.vel, "the FCC start"
    pos = np.mod(pos, w.L)  # between list builds positions may sit outside [0, L)
    pos[pos >= w.L] = 0.0
    s = oracle.make_sys(w.n, w.L, r_cut=w.r_cut, skin=w.skin, dt=w.dt,
                        potential=oracle.LJ_SHIFTED if w.shifted else oracle.LJ_TRUNC,
                        use_nl=w.use_nl)
    t = time.perf_counter()
    oracle.run(s, pos, vel, 0)
    t_build = time.perf_counter() - t
    t = time.perf_counter()
    nreb = oracle.run(s, pos, vel, steps)[4]
    t_run = time.perf_counter() - t
    per = max(t_run - t_build, 1e-9)
    return {"value": w.n * steps / per, "unit": "atom-steps/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "rebuilds": int(nreb),
            "sample": f"{w.name}: full N={w.n}, {steps} steps from {start}, {nreb} list "
                      f"rebuilds inside; time of the run minus the time of its initial "
                      f"cell/list/force build"}


def copy_probe(mib):
    import torch

    a = torch.empty(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2003_14061_amd import inputs

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = inputs.preset(args.workload).materialize()
    fp64 = None
    if not args.no_main:
        fp64 = run_gpu(w, "fp64", args.steps, args.warmup, drift_steps=args.drift_steps,
                       keep_state=True)
        print(f"[bench] fp64 done: {fp64['value']:.3e} atom-steps/s", file=sys.stderr,
              flush=True)
    mixed = None
    if not args.no_mixed:
        mixed = run_gpu(w, "fp32", args.steps, args.warmup, drift_steps=args.drift_steps)
        print(f"[bench] fp32-mixed done: {mixed['value']:.3e} atom-steps/s", file=sys.stderr,
              flush=True)
    lay = None
    if not args.no_layers:
        lay = run_gpu(w, "fp64", args.steps, args.warmup, pipeline="layers", reorder=100)
        print(f"[bench] fp64 layer-matrix pipeline done: {lay['value']:.3e} atom-steps/s",
              file=sys.stderr, flush=True)
    n3 = None
    if not args.no_newton3:
        n3 = run_gpu(w, "fp64", args.steps, args.warmup, newton3=True)
        print(f"[bench] fp64 third-law variant done: {n3['value']:.3e} atom-steps/s",
              file=sys.stderr, flush=True)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    cpu = None
    if not args.no_cpu:
        cpu = run_cpu(w, args.cpu_steps, *((fp64["final_pos"], fp64["final_vel"])
                                           if fp64 is not None else (None, None)))
        print(f"[bench] cpu oracle done: {cpu['value']:.3e} atom-steps/s", file=sys.stderr,
              flush=True)
    if fp64 is None:  # a profiling run of the other legs: no headline figure
        fp64 = {"value": float("nan"), "ms_per_step": float("nan"), "roofline": None,
                "rebuilds": None, "mean_nl": float("nan"), "mean_in_range": float("nan"),
                "energy_drift_per_atom": None, "force_ms_avg": float("nan")}
    out = {
        "metric": METRIC,
        "value": round(fp64["value"], 1),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp64["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: LJ cut and shifted at r_c={w.r_cut:g} sigma, N={w.n} "
                        f"(FCC), rho={w.rho}, T={w.T}, dt={w.dt}, skin={w.skin}, neighbor list "
                        f"rebuilt at max displacement > skin/2, reorder by cell at rebuild",
            "n_atoms": w.n, "precision": "fp64"},
        "roofline": fp64["roofline"],
        "cpu_baseline": cpu,
        "rebuilds": fp64["rebuilds"],
        "mean_nl": round(fp64["mean_nl"], 2),
        "mean_in_range": round(fp64["mean_in_range"], 2),
        "energy_drift_per_atom": fp64["energy_drift_per_atom"],
        "energy_drift": fp64.get("energy_drift"),
        "force_ms_avg": round(fp64["force_ms_avg"], 5),
        "value_graph_replays": (round(fp64["value_graph_replays"], 1)
                                if "value_graph_replays" in fp64 else None),
        "parts": fp64.get("parts"),
    }
    if mixed is not None:
        ferr = (error_fp32(w, fp64["final_pos"], fp64["final_vel"])
                if "final_vel" in fp64 else None)
        out["fp32_mixed"] = {"value": round(mixed["value"], 1),
                             "error_vs_fp64": ferr,
                             "energy_drift": mixed["energy_drift"],
                             "ms_per_step": round(mixed["ms_per_step"], 5),
                             "roofline": mixed["roofline"], "rebuilds": mixed["rebuilds"],
                             "energy_drift_per_atom": mixed["energy_drift_per_atom"],
                             "force_ms_avg": round(mixed["force_ms_avg"], 5),
                             "speedup_vs_fp64": round(mixed["value"] / fp64["value"], 3)}
    if lay is not None:
        out["paper_layers_fp64"] = {
            "value": round(lay["value"], 1), "ms_per_step": round(lay["ms_per_step"], 5),
            "force_ms_avg": round(lay["force_ms_avg"], 5), "rebuilds": lay["rebuilds"],
            "energy_drift_per_atom": lay["energy_drift_per_atom"],
            "tiled_speedup": round(fp64["value"] / lay["value"], 3),
            "steps": args.steps, "reorder_every": 100,
            "parts": lay["parts"], "tiled_parts": fp64.get("parts"),
            "kernels": "k_layer_clear, k_layer_assign, k_layer_nl, k_layer_forces: one thread "
                       "per atom, 32-bit neighbor matrix, partners gathered from HBM; every "
                       "100 steps k_scan, k_layer_pack, k_layer_permute, k_layer_copyback "
                       "and a forced rebuild of both matrices"}
    if n3 is not None:
        out["newton3_fp64"] = {"value": round(n3["value"], 1),
                               "ms_per_step": round(n3["ms_per_step"], 5),
                               "force_ms_avg": round(n3["force_ms_avg"], 5),
                               "mean_half_nl": round(n3["mean_nl"], 2),
                               "rebuilds": n3["rebuilds"],
                               "energy_drift_per_atom": n3["energy_drift_per_atom"],
                               "speedup_vs_full_list": round(n3["value"] / fp64["value"], 3),
                               "kernels": "k_zero_forces + k_forces_half"}
    if not args.no_small:
        out["wca_4000_cells"], out["wca_256k"] = run_small(args.drift_steps)
    if not args.no_batch:
        bt = run_batch(steps=args.batch_steps, tune_cache=args.tune_cache,
                       fixed_tuning=json.loads(args.batch_tuning) if args.batch_tuning else None)
        print(f"[bench] batch done: {bt['value']:.3e} atom-steps/s", file=sys.stderr, flush=True)
        out["batched_ensemble"] = dict(bt, workload="64 WCA replicas, N~U[500,32000], "
                                       "rho~U[0.6,0.9], T=1, dt=0.005, skin 0.3, FP32-mixed, "
                                       f"one HIP graph launch per {args.batch_steps} steps")
    if not args.no_allpairs:
        out["paper_allpairs"] = run_allpairs()
    if not args.no_polymer:
        out["polymer_melt"] = run_polymer()
        print(f"[bench] polymer melt done: {out['polymer_melt']['bonded']['value']:.3e} "
              "atom-steps/s", file=sys.stderr, flush=True)
    if not args.no_adjoint:
        adj = {}
        for prec, key in (("fp64", "fp64"), ("fp32", "fp32_mixed")):
            r = run_adjoint(prec)
            adj[key] = {k: round(v, 6) for k, v in r.items()}
            print(f"[bench] adjoint {key} done: ratio {r['ratio']:.3f}", file=sys.stderr,
                  flush=True)
        out["adjoint_forward_ratio"] = {
            "fp64": adj["fp64"]["ratio"], "fp32_mixed": adj["fp32_mixed"]["ratio"],
            "workload": "lj_32k: LJ r_c=2.5, N=32000 FCC, rho=0.8, T=1, dt=0.004, 200 steps, "
                        "checkpoints every 20, loss = mean PE/N + soft g(r) (50 bins) "
                        "mismatch against a run at eps=1.05, sigma=0.98",
            "detail": adj}
    else:
        out["adjoint_forward_ratio"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
