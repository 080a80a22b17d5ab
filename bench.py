"""Throughput of the FP64 Lennard-Jones MD step on one MI355X.

A step is one velocity-Verlet step of the whole hot path (kick + drift +
wrap, cell binning and neighbor-list rebuild every 20 steps, force sum, kick)
on a seeded synthetic FCC box, with all state resident in HBM.

Primary workload: FCC 32^3 unit cells = 131,072 atoms, rho 0.8442, T 1.44,
cutoff 2.5 + skin 0.3, dt 0.005, rebuild every 20 steps (the paper's
single-core CPU shape).  Secondary (same JSON line): FCC 96^3 = 3,538,944
atoms jittered by +-0.01 (one node's subdomain in the paper's CPU weak
scaling), 500 steps.

Prints one JSON line.  Fields beyond the contract: "roofline" (force kernel
against the HBM roofline, from HIP events recorded around every force launch
on the launch stream), "cpu_baseline" (the CPU oracle on a bounded sample of
the primary workload) and "secondary".
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, AMD published
METRIC = "atom-steps/s (FP64 LJ) at 131k & 3.5M atoms; batched, adjoint vs plain"
KERNEL_SRC = os.path.join(ROOT, "paper_2009_07400_amd", "csrc", "engine.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kernel_traffic.json")

WORKLOADS = {
    "c1": dict(ncell=32, rho=0.8442, T=1.44, jitter=0.0, seed=1001, steps=1000,
               name="LJ FCC 32^3 = 131,072 atoms, rho 0.8442, T 1.44, rc 2.5 + skin 0.3, dt 0.005, rebuild 20"),
    "c2": dict(ncell=96, rho=0.8442, T=1.44, jitter=0.02, seed=1002, steps=500,
               name="LJ FCC 96^3 = 3,538,944 atoms jittered +-0.01, rho 0.8442, T 1.44, rc 2.5 + skin 0.3, "
                    "dt 0.005, rebuild 20"),
}


def _kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def _traffic(workload: str):
    """HBM bytes per force launch from stored rocprofv3 FETCH_SIZE/WRITE_SIZE
    counters, valid only for the kernel source they were taken from."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = rec.get(workload)
    if not ent or rec.get("kernel_sha256_16") != _kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def _schedule(g) -> dict:
    info = g.info()
    return {k: info[k] for k in ("block_edge", "block_parts", "lanes_per_atom", "block_threads", "build_threads",
                                 "build_lanes", "lds_atoms", "half_list", "layout")}


REBUILD_EVERY = 20  # list rebuild interval of every workload here


def _warm_and_tune(g, warmup: int, schedule=None) -> int:
    """Fix the schedule and run the warmup steps, all outside the timed
    region; returns the untimed steps run before the warmup.  Without a
    given schedule, one whole rebuild interval runs first and the autotuner
    picks the schedule at its end (a rebuild step, so the fixed rebuild
    schedule is kept), whatever the warmup: on the initial lattice every list
    has the same length, while a few steps later lengths spread as they do
    in the timed steps, and every wavefront runs to the longest list among
    its atoms, which changes which schedule is fastest."""
    if schedule:  # fixed schedule, e.g. for profiling runs
        sched = dict(schedule)
        half, layout = sched.pop("half_list", 0), sched.pop("layout", 0)
        g.set_half_list(bool(half))  # (resets threads and capacity: first)
        g.set_schedule(**sched)
        g.set_layout(layout)
        g.integrate(warmup)
        return 0
    g.integrate(REBUILD_EVERY)
    # 20 launches per candidate: at 131k atoms several schedules lie within
    # 2% of each other, and five launches ranked them differently from run
    # to run
    g.autotune(repeats=20)
    g.integrate(warmup)
    return REBUILD_EVERY


# Issue rate of unfused FP64 vector instructions (add, mul, compare): 256
# CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz.  The 78.6 TFLOP/s FP64
# vector peak counts a fused multiply-add as two operations of this rate.
FP64_ISSUE_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def _force_roofline(n: int, mean_list: float, avg_s: float, traffic=None, kernel="") -> dict:
    """Force kernel against the HBM roofline at the algorithmic bytes per
    atom of the force sum: count 4 + list 4 n_list + x_i 24 + F_i 24 (each
    neighbor position counted once, gathered from LDS or cache).  The kernel
    fuses the kicks and the drift, so its own traffic replaces the force
    write by the velocity read and write and the drifted position write
    (100 + 4 n_list); that figure is reported beside it."""
    alg = (52.0 + 4.0 * mean_list) * n
    fused = (100.0 + 4.0 * mean_list) * n
    out = {"bound": "hbm", "kernel": kernel, "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
           "alg_bytes_per_atom": 52.0 + 4.0 * mean_list, "alg_bytes_per_launch": alg,
           "avg_launch_us": avg_s * 1e6,
           "fused_kernel": {"bytes_per_atom": 100.0 + 4.0 * mean_list, "achieved": fused / avg_s / 1e9,
                            "frac": fused / avg_s / 1e9 / HBM_PEAK_GBS}}
    if traffic:
        out["traffic_frac"] = traffic / avg_s / 1e9 / HBM_PEAK_GBS
    out.update(_force_flops(n, mean_list, avg_s))
    return out


def _trimmed_subcells(side_over_rl: float, k: int = 24) -> float:
    """Mean number of the 125 half-size subcells around an atom's own
    (offsets -2..2 per axis) that its cutoff sphere reaches, for an atom
    placed uniformly in its subcell (midpoint rule, k^3 points): the list
    build walks only those.  Along an axis, the subcells at offsets -2, -1,
    +1, +2 begin q + h, q, h - q and 2h - q away (q the atom's distance from
    its subcell's low edge, h the subcell side)."""
    h = 0.5 * side_over_rl  # in units of rl
    q = (np.arange(k) + 0.5) / k * h
    d = np.stack([q + h, q, np.zeros_like(q), h - q, 2 * h - q])  # [offset, point]
    sq = d * d
    tot = 0.0
    for qx in sq.T:
        for qy in sq.T:
            # [dz offset, point z] + [dy offset] + [dx offset] for this x, y
            s3 = sq[:, None, None, :] + qy[None, :, None, None] + qx[None, None, :, None]
            tot += (s3 < 1.0).sum()
    return tot / k ** 3


def stencil_candidates(boxes, rl: float = 2.8, block_edge: int = 2) -> float:
    """Mean candidates per atom of the list build over boxes [(n_atoms, L)]:
    atoms per subcell times the subcells walked, the trimmed stencil where a
    block's neighborhood holds no cell twice (cells per axis >= block edge +
    2), else every distinct subcell of the 5^3 stencil."""
    tot = 0.0
    n_all = 0
    for n, L in boxes:
        nc = int(np.floor(L / rl))
        per_sub = n / (8.0 * nc ** 3)
        subs = _trimmed_subcells(L / nc / rl) if nc >= block_edge + 2 else float(min(5, 2 * nc) ** 3)
        tot += n * per_sub * subs
        n_all += n
    return tot / n_all


def _build_rooflines(tm: dict, n: int, mean_list: float, n_cells: int, cand: float) -> dict:
    """Roofline figures of the binning and list-build kernels, per call (one
    call = one rebuild: the binning bucket sums its four to eight launches).

    Binning moves 132 algorithmic bytes per atom (read x and the atom id,
    28; the permutation reads x, v and id and writes them, 52 + 52).  The
    list build reads x (24) and writes the count (4) and the list (4 bytes
    per entry at the method's index width) and tests cand candidates per
    atom (stencil_candidates(): the atoms of the half-size subcells that the
    cutoff sphere reaches; 27 whole cells hold about 2.6x as many), 8
    unfused FP64 instructions each (3 differences, 3 squares, 2 sums, no
    fused multiply-add so that its decisions match any IEEE evaluation): it
    is bound by FP64 instruction issue, so its fraction is taken against the
    issue rate of unfused FP64 instructions, with the HBM fraction beside
    it."""
    out = {}
    if tm.get("binning", (0, 0))[1]:
        ms, calls = tm["binning"]
        t = ms / calls * 1e-3
        b = 132.0 * n
        out["binning"] = {"bound": "hbm", "achieved": b / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": b / t / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_call": b, "avg_call_us": t * 1e6}
    if tm.get("neighbor", (0, 0))[1]:
        ms, calls = tm["neighbor"]
        t = ms / calls * 1e-3
        b = (28.0 + 4.0 * mean_list) * n
        ops = 8.0 * cand * n
        out["neighbor"] = {"bound": "alu", "achieved": ops / t / 1e12, "peak": FP64_ISSUE_PEAK_T,
                           "unit": "T FP64 instr/s", "frac": ops / t / 1e12 / FP64_ISSUE_PEAK_T,
                           "candidates_per_atom": cand, "cell_stencil_candidates_per_atom": 27.0 * n / n_cells,
                           "hbm_achieved_gbs": b / t / 1e9,
                           "hbm_frac": b / t / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_call": b, "avg_call_us": t * 1e6}
    return out


def _force_flops(n: int, mean_list: float, avg_s: float, rc: float = 2.5, rl: float = 2.8) -> dict:
    """Nominal FP64 work of the force kernel beside its HBM roofline: 8
    operations per listed pair (difference, |d|^2, cutoff test) and 15 more
    per interacting pair (reciprocal, force factor, accumulation), the
    interacting share of the list taken as (rc / rl)^3 (uniform density)."""
    n_int = mean_list * (rc / rl) ** 3
    fl = (8.0 * mean_list + 15.0 * n_int) * n
    return {"fp64_flops_per_launch": fl, "fp64_tflops": fl / avg_s / 1e12,
            "fp64_frac": fl / avg_s / 1e12 / FP64_PEAK_TFLOPS}


def run_gpu(workload: str, steps: int, warmup: int, schedule=None):
    import torch

    from paper_2009_07400_amd import System
    from workloads import md_system

    w = WORKLOADS[workload]
    s = md_system(w["ncell"], w["rho"], w["T"], seed=w["seed"], jitter=w["jitter"])
    g = System(s.n, s.L, max_neighbors=128)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    tuning_steps = _warm_and_tune(g, warmup, schedule)
    g.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.integrate(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.sync()
    elapsed = t1 - t0

    # Kernel timing pass: the same number of steps again with HIP events
    # recorded on the launch stream around every kernel.
    g.set_timing(True)
    g.integrate(steps)
    g.sync()
    tm = g.get_timing()
    g.set_timing(False)
    mean_list = float(g.neighbor_counts().double().mean().item())
    n_cells = int(g.info()["n_cells"])
    g.sync()
    ms, launches = tm["force"]
    avg_s = ms / max(launches, 1) * 1e-3
    sched = _schedule(g)
    res = {
        "n": s.n,
        "steps": steps,
        "warmup": warmup,
        "tuning_steps": tuning_steps,
        "elapsed_s": elapsed,
        "value": s.n * steps / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "mean_list_length": mean_list,
        "schedule": sched,
        "kernel_ms": {k: (v[0] / max(v[1], 1), v[1]) for k, v in tm.items() if v[1]},
        "roofline": _force_roofline(s.n, mean_list, avg_s, _traffic(workload),
                                    "k_force<2,false>: LDS-staged block force + kick + kick + drift"),
        "build_rooflines": _build_rooflines(tm, s.n, mean_list, n_cells,
                                            stencil_candidates([(s.n, s.L)], block_edge=sched["block_edge"])),
    }
    g.close()
    return res


def run_batched(steps: int = 200, warmup: int = 20, n_boxes: int = 512):
    """512 replica boxes (FCC n^3, n in 4..12, rho in [0.75, 0.90], T in
    [0.7, 1.5], own seeds) advanced together, against the same boxes run one
    after another as separate single-box systems on the same stream."""
    import torch

    from paper_2009_07400_amd import System
    from workloads import batched_box_specs, md_system

    boxes = [md_system(n, rho, T, seed=seed) for n, rho, T, seed in batched_box_specs(n_boxes)]
    total = sum(b.n for b in boxes)
    g = System.batch([b.n for b in boxes], [b.L for b in boxes], dict(max_neighbors=128))
    g.set_state(torch.from_numpy(np.concatenate([b.pos() for b in boxes])),
                torch.from_numpy(np.concatenate([b.vel() for b in boxes])))
    _warm_and_tune(g, warmup)
    sched = _schedule(g)
    # each whole rebuild interval of the timed run is one captured HIP graph;
    # the two graphs (one per parity of the double-buffered state) are
    # captured in two more untimed intervals
    g.set_graphs(True)
    g.integrate(2 * 20 + 1)
    captured = g.info()["graph_captures"]
    g.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.integrate(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    g.sync()
    info = g.info()
    # kernel timing pass (eager: timing keeps graph mode off)
    g.set_timing(True)
    g.integrate(steps)
    g.sync()
    tm = g.get_timing()
    g.set_timing(False)
    mean_list = float(g.neighbor_counts().double().mean().item())
    g.sync()
    g.close()
    ms, launches = tm["force"]
    roof = _force_roofline(total, mean_list, ms / max(launches, 1) * 1e-3,
                           kernel="k_force<2,false>: one launch over every box's blocks")
    brf = _build_rooflines(tm, total, mean_list, int(info["n_cells"]),
                           stencil_candidates([(b.n, b.L) for b in boxes], block_edge=sched["block_edge"]))
    seq = []
    for b in boxes:
        s = System(b.n, b.L, max_neighbors=128)
        s.set_state(torch.from_numpy(b.pos()), torch.from_numpy(b.vel()))
        s.integrate(warmup)
        seq.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in seq:
        s.integrate(steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for s in seq:
        s.sync()
        s.close()
    per_class = _batch_per_class(boxes, steps, warmup)
    return {"workload": f"{n_boxes} LJ boxes, FCC n^3 with n in 4..12 ({total:,} atoms), rho 0.75-0.90, T 0.7-1.5, "
                        "rc 2.5 + skin 0.3, dt 0.005, rebuild 20",
            "value": total * steps / t_batch, "unit": "atom-steps/s", "steps": steps,
            "ms_per_step": t_batch / steps * 1e3, "sequential_value": total * steps / t_seq,
            "sequential_ms_per_step": t_seq / steps * 1e3, "speedup_vs_sequential": t_seq / t_batch,
            "schedule": sched, "n_blocks": info["n_blocks"], "lds_atoms": info["lds_atoms"],
            "graph_captures_in_warmup": captured, "graph_launches": info["graph_launches"],
            "graph_captures": info["graph_captures"], "mean_list_length": mean_list, "roofline": roof,
            "build_rooflines": brf, "kernel_avg_ms": {k: (v[0] / max(v[1], 1), v[1]) for k, v in tm.items() if v[1]},
            "per_class": per_class}


def _batch_per_class(boxes, steps: int, warmup: int) -> dict:
    """The same boxes split by cells per axis into one batch per class, each
    autotuned on its own and run in graph mode, the classes one after another
    on one stream: the per-box-class schedule against the one schedule of the
    whole batch."""
    import torch

    from paper_2009_07400_amd import System

    classes = {}
    for b in boxes:
        classes.setdefault(int(np.floor(b.L / 2.8)), []).append(b)
    systems, rows = [], []
    for nc, bs in sorted(classes.items()):
        g = System.batch([b.n for b in bs], [b.L for b in bs], dict(max_neighbors=128))
        g.set_state(torch.from_numpy(np.concatenate([b.pos() for b in bs])),
                    torch.from_numpy(np.concatenate([b.vel() for b in bs])))
        _warm_and_tune(g, warmup)
        g.set_graphs(True)
        g.integrate(2 * REBUILD_EVERY + 1)
        rows.append({"cells_per_axis": nc, "boxes": len(bs), "atoms": sum(b.n for b in bs), "schedule": _schedule(g)})
        systems.append(g)
    for g in systems:
        g.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in systems:
        g.integrate(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    for g in systems:
        g.sync()
        g.close()
    total = sum(r["atoms"] for r in rows)
    return {"value": total * steps / t, "ms_per_step": t / steps * 1e3, "classes": rows}


def run_adjoint(steps: int = 200, replicas: int = 64):
    """64 replicas of FCC 10^3 = 4,000 atoms (rho 0.8442, T 1.0): forward with
    checkpoints plus the reverse sweep, against the plain forward run."""
    import torch

    from paper_2009_07400_amd import System
    from workloads import md_system

    reps = [md_system(10, 0.8442, 1.0, seed=3000 + r) for r in range(replicas)]
    total = sum(r.n for r in reps)
    x0 = torch.from_numpy(np.concatenate([r.pos() for r in reps]))
    v0 = torch.from_numpy(np.concatenate([r.vel() for r in reps]))
    g = System.batch([r.n for r in reps], [r.L for r in reps], dict(max_neighbors=128))
    lam = torch.randn(total, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(5))
    # one schedule for both runs (of those the adjoint runs with: full lists,
    # SoA positions), tuned a rebuild interval into the run
    g.set_state(x0, v0)
    g.integrate(20)
    g.autotune(repeats=3, for_adjoint=True)
    sched = _schedule(g)
    for _ in range(2):  # second pass is the timed one
        g.set_state(x0, v0)
        g.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.integrate(steps)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        g.set_state(x0, v0)
        g.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.adjoint_forward(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.adjoint_backward(lam)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g.sync()
    # reverse-kernel timing: one more forward + backward with HIP events
    g.set_state(x0, v0)
    g.adjoint_forward(steps)
    # list of the recorded run's last interval (the backward pass leaves the
    # state but not a valid list)
    mean_list = float(g.neighbor_counts().double().mean().item())
    g.set_timing(True)
    g.adjoint_backward(lam)
    g.sync()
    tm = g.get_timing()
    g.set_timing(False)
    g.close()
    ms, launches = tm["adjoint"]
    avg_s = ms / max(launches, 1) * 1e-3
    # algorithmic bytes per atom of the Hessian-vector product: count 4 + list
    # 4 n_list + x_i and w_i 48 + output 24 (neighbor x_j, w_j from LDS/cache)
    hvp_b = (76.0 + 4.0 * mean_list) * total
    hvp = {"bound": "hbm", "kernel": "k_hvp: Hessian-vector product + parameter partials + drift adjoint",
           "achieved": hvp_b / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": hvp_b / avg_s / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_atom": 76.0 + 4.0 * mean_list,
           "avg_launch_us": avg_s * 1e6, "launches": launches}
    return {"workload": f"{replicas} x LJ FCC 10^3 = {total:,} atoms, rho 0.8442, T 1.0, {steps} steps, "
                        "checkpoints at every rebuild (20)",
            "value": total * steps / (t2 - t0), "unit": "atom-steps/s (forward + reverse per step)",
            "plain_value": total * steps / t_plain, "adjoint_over_plain_time": (t2 - t0) / t_plain,
            "forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3, "plain_ms": t_plain * 1e3,
            "schedule": sched, "hvp_roofline": hvp}


def run_spring_dashpot(steps: int = 200, warmup: int = 20):
    """Spring-Dashpot spheres (Sec. 3.2, Eq. 3): the paper's load-balancing
    geometry - a periodic cube of 96^3 unit cells, one sphere per cell corner
    on one side of a diagonal plane (442,368 spheres, half the domain empty),
    stiffness and damping zero as in the paper (spheres at rest) - and a
    dense packing of 1,048,576 spheres pressing on their twelve neighbours
    (K 1000, gamma 5) in motion.  Diameter 1, list radius 1.3, dt 0.001,
    rebuild every 20 steps."""
    import torch

    from paper_2009_07400_amd import System
    from workloads import sd_half_domain, sd_system

    out = {}
    pos, L = sd_half_domain(96)
    dense = sd_system(64)
    cases = {
        "half_domain": (pos, np.zeros_like(pos), L, 0.0, 0.0,
                        "96^3 unit cells, spheres on one side of the diagonal plane (442,368), K = gamma = 0 "
                        "(the paper's load-balancing setup)"),
        "dense": (dense.pos(), dense.vel(), dense.L, dense.k, dense.gamma,
                  "FCC 64^3 = 1,048,576 spheres at 0.98 sigma spacing (12 contacts each), K 1000, gamma 5, T 0.5"),
    }
    for name, (p, v, Lb, k, gamma, desc) in cases.items():
        g = System(p.shape[0], Lb, model="spring_dashpot", stiffness=k, damping=gamma, sigma=1.0, cutoff=1.0,
                   skin=0.3, dt=1e-3, max_neighbors=32)
        g.set_state(torch.from_numpy(p), torch.from_numpy(v))
        _warm_and_tune(g, warmup)
        g.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.integrate(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.sync()
        g.set_timing(True)
        g.integrate(steps)
        g.sync()
        tm = g.get_timing()
        g.set_timing(False)
        mean_list = float(g.neighbor_counts().double().mean().item())
        g.sync()
        sched = _schedule(g)
        g.close()
        ms, launches = tm["force"]
        avg_s = ms / max(launches, 1) * 1e-3
        n = p.shape[0]
        # algorithmic bytes per sphere of the force sum: count 4 + list
        # 4 n_list + x_i 24 + v_i 24 + F_i 24 (neighbours' x, v from LDS/cache)
        alg = (76.0 + 4.0 * mean_list) * n
        out[name] = {"workload": desc, "value": n * steps / el, "unit": "atom-steps/s", "steps": steps,
                     "ms_per_step": el / steps * 1e3, "mean_list_length": mean_list, "schedule": sched,
                     "roofline": {"bound": "hbm", "kernel": "k_force_sd<2,false>: contact force + kicks + drift",
                                  "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_atom": 76.0 + 4.0 * mean_list,
                                  "avg_launch_us": avg_s * 1e6},
                     "kernel_avg_ms": {k2: (v2[0] / max(v2[1], 1), v2[1]) for k2, v2 in tm.items() if v2[1]}}
    return out


def run_axes(steps: int = 40):
    """The schedule axes the autotuner weighs, measured one by one on the
    131k- and 3.5M-atom workloads at block edges 2 and 3 (default threads):
    the position layout (SoA, AoS, AoSoA; full lists) and half lists inside
    blocks (SoA).  Per variant the mean force (step kernel), list-build and
    binning times over `steps` steps after one rebuild interval, the mean
    list length, and the implied time per step."""
    import torch

    from paper_2009_07400_amd import System
    from workloads import md_system

    out = {}
    for wl in ("c1", "c2"):
        w = WORKLOADS[wl]
        s = md_system(w["ncell"], w["rho"], w["T"], seed=w["seed"], jitter=w["jitter"])
        rows = []
        for edge in (2, 3):
            for half, layout in ((False, "soa"), (False, "aos"), (False, "aosoa"), (True, "soa")):
                g = System(s.n, s.L, max_neighbors=128)
                g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
                g.set_schedule(block_edge=edge)
                g.set_half_list(half)
                g.set_layout(layout)
                g.integrate(REBUILD_EVERY)
                g.set_timing(True)
                g.integrate(steps)
                g.sync()
                tm = g.get_timing()
                g.set_timing(False)
                ml = float(g.neighbor_counts().double().mean().item())
                g.sync()
                g.close()
                us = {k: tm[k][0] / tm[k][1] * 1e3 for k in ("force", "neighbor", "binning") if tm[k][1]}
                rows.append({"block_edge": edge, "half_list": int(half), "layout": layout, "mean_list": ml,
                             "force_us": us["force"], "build_us": us["neighbor"], "binning_us": us["binning"],
                             "us_per_step": us["force"] + (us["neighbor"] + us["binning"]) / REBUILD_EVERY})
        out[wl] = rows
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(workload: str, sample_steps: int, single_steps: int):
    """The oracle on a bounded sample of the workload: OpenMP over atoms on
    the host's threads, then on one thread (the paper's single-core
    protocol), with its time split into force sums, list builds and the rest
    (the Force / Neigh / Other split of the paper's Sec. 6 figures)."""
    import oracle
    from workloads import md_system

    w = WORKLOADS[workload]
    s = md_system(w["ncell"], w["rho"], w["T"], seed=w["seed"], jitter=w["jitter"])
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, sample_steps, thermo=False, maxnb=128)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    r1 = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, single_steps, thermo=False, maxnb=128)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": s.n * sample_steps / dt, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"{w['name']}: first {sample_steps} steps (initial list build + {sample_steps // 20} "
                      f"rebuilds), OpenMP over atoms on {threads} threads, {dt:.1f} s",
            "split_s": r["times"],
            "single_thread": {"value": s.n * single_steps / dt1, "unit": "atom-steps/s", "cores": 1,
                              "sample": f"first {single_steps} steps on one thread, {dt1:.1f} s",
                              "split_s": r1["times"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c1")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 3.5M-atom secondary workload")
    ap.add_argument("--cpu-steps", type=int, default=1000,
                    help="oracle steps on all host threads (default: the whole 1000-step workload)")
    ap.add_argument("--cpu-single-steps", type=int, default=100, help="oracle steps on one thread")
    ap.add_argument("--schedule", default=None,
                    help="fixed schedule for the primary workload: block edge, workgroups per block, lanes per "
                         "atom, force threads[, build threads[, build lanes[, half lists (0/1)[, position layout "
                         "(0 SoA, 1 AoS, 2 AoSoA)]]]], e.g. 3,1,1,640 (default: autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="before the run, copy a 1 GiB buffer 3 times with torch: a kernel of known traffic "
                         "(1 GiB read + 1 GiB written per launch) to calibrate FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    steps = args.steps if args.steps is not None else WORKLOADS[args.workload]["steps"]
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sched = None
    if args.schedule:
        v_ = [int(v) for v in args.schedule.split(",")]
        if len(v_) not in (4, 5, 6, 7, 8):
            ap.error("--schedule takes 4 to 8 comma-separated integers")
        sched = dict(block_edge=v_[0], block_parts=v_[1], lanes_per_atom=v_[2], threads=v_[3],
                     build_threads=v_[4] if len(v_) >= 5 else 0, build_lanes=v_[5] if len(v_) >= 6 else 0,
                     half_list=v_[6] if len(v_) >= 7 else 0, layout=v_[7] if len(v_) >= 8 else 0)
    prim = run_gpu(args.workload, steps, args.warmup, sched)
    print(f"# primary {args.workload}: {prim['value']:.4g} atom-steps/s, {prim['ms_per_step']:.4f} ms/step",
          file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": prim["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "tuning_steps": prim["tuning_steps"],
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded FCC lattice, SplitMix64 velocities)",
        "config": {"workload": WORKLOADS[args.workload]["name"], "n_atoms": prim["n"],
                   "neighbor_list": "half inside blocks" if prim["schedule"]["half_list"] else "full",
                   "max_neighbors": 128},
        "roofline": prim["roofline"],
        "kernel_avg_ms": prim["kernel_ms"],
        "build_rooflines": prim["build_rooflines"],
        "mean_list_length": prim["mean_list_length"],
        "schedule": prim["schedule"],
    }
    if not args.no_secondary and args.workload != "c2":
        sec = run_gpu("c2", WORKLOADS["c2"]["steps"], args.warmup)
        print(f"# secondary c2: {sec['value']:.4g} atom-steps/s", file=sys.stderr, flush=True)
        out["secondary"] = {"c2": {"workload": WORKLOADS["c2"]["name"], "value": sec["value"],
                                   "ms_per_step": sec["ms_per_step"], "steps": sec["steps"],
                                   "roofline": sec["roofline"], "kernel_avg_ms": sec["kernel_ms"],
                                   "build_rooflines": sec["build_rooflines"],
                                   "mean_list_length": sec["mean_list_length"], "schedule": sec["schedule"]}}
        bat = run_batched()
        print(f"# secondary batched: {bat['value']:.4g} atom-steps/s, {bat['speedup_vs_sequential']:.1f}x "
              "sequential", file=sys.stderr, flush=True)
        out["secondary"]["batched"] = bat
        print(f"# secondary batched per box class: {bat['per_class']['value']:.4g} atom-steps/s "
              f"({len(bat['per_class']['classes'])} classes)", file=sys.stderr, flush=True)
        adj = run_adjoint()
        print(f"# secondary adjoint: {adj['value']:.4g} atom-steps/s, {adj['adjoint_over_plain_time']:.2f}x plain "
              "time", file=sys.stderr, flush=True)
        out["secondary"]["adjoint"] = adj
        sd = run_spring_dashpot()
        print("# secondary spring-dashpot: " + ", ".join(f"{k} {v['value']:.4g} atom-steps/s" for k, v in sd.items()),
              file=sys.stderr, flush=True)
        out["secondary"]["spring_dashpot"] = sd
        out["secondary"]["schedule_axes"] = run_axes()
        print("# secondary schedule axes: " + "; ".join(
            f"{wl} E{r['block_edge']} {'half' if r['half_list'] else 'full'} {r['layout']} {r['us_per_step']:.1f} us"
            for wl, rows in out["secondary"]["schedule_axes"].items() for r in rows), file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = run_cpu_baseline(args.workload, args.cpu_steps, args.cpu_single_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
