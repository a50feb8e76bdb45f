#!/usr/bin/env python3
"""Throughput of the SPH solid-body right-hand side and its adjoint on one MI355X.

Default workload: the non-uniform three-body set (8,388,608 particles: a dense
sphere with about 250 partners per particle, a sphere with about 60 and a sparse
shell with about 20; h = 2.4 dx).  One step = one pass of the whole hot path over it:
  cell build (tiled cell numbering)                          sph_build_cells
  frozen pair list (the interaction list, skin 0)            sph_build_pairs
  partner lists (CSR, user order, rows ascending)            sph_neighbours
  FP64 right-hand side (writing its velocity gradient and   sph_rhs
  operand records)
  FP64 adjoint (vector-Jacobian product, random cotangent,   sph_rhs_adjoint
  reading them instead of forming them again)
The metric counts the ordered pair interactions (b != a, |x_a - x_b| < h) evaluated
by the right-hand side and by the adjoint: value = 2 nnz / step time.  Inputs are
resident on the GPU before timing starts.  Reported beside it: the FP32-compensated
right-hand side (speed and normwise error per output against the FP64 GPU path and
against the oracle on 4,096 sampled targets), each stage's time, the partner-count
histogram, the roofline of the step's dominant kernel, the oracle's CPU rate and, on
the two-sphere collision (262,144 particles), the 10-step leapfrog with its reverse
sweep and the extended forms (energy, artificial stress, XSPH, Tillotson, damage,
Barnes-Hut gravity).

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one GPU (the
multi-GPU decomposition is described in the design notes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair interactions/s for sph_rhs (FP64 vs FP32-comp) and adjoint, 1 MI355X"
UNIT = "pair interactions/s"
PEAK_FP64_TFLOPS = 78.6  # MI355X vector FP64
PEAK_HBM_GBS = 8000.0
CELLS_PER_H = 2  # cell edge (h + skin) / 2: fewer candidates per row sweep than edge h + skin

# Algorithmic FP64 operations per ordered pair, the scope's measurement unit: 95 for
# the right-hand side (distance, square root, kernel and gradient, density sum,
# velocity gradient, viscosity, stress bracket, acceleration) and 250 for the adjoint
# (both roles of the pair; the lower end of the 250-300 estimate).  The kernels' own
# operation counts (FMA = 2, square root and division = 1) are reported beside them:
# 83 + 10 on approaching pairs (right-hand side), 222 + 23 (adjoint), 45 (the adjoint's
# velocity-gradient pass).
FLOPS_PER_PAIR = {"pairs_fp64": 95.0, "adjoint_pairs": 250.0, "adjoint_L": 45.0}
IMPL_FLOPS = {"pairs_fp64": (83.0, 10.0), "adjoint_pairs": (222.0, 23.0), "adjoint_L": (45.0, 0.0)}
KERNEL_NAME = {"pairs_fp64": "k_pairs64_list", "adjoint_pairs": "k_adj_pairs_list",
               "adjoint_L": "k_adj_L_list"}
# gravity walk, per body taken: distance (3), r^2 (5), opening test (3), force with a
# refined reciprocal square root and the reciprocal of r + eps (11)
FLOPS_GRAV_TERM = 22


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="nonuniform", choices=["nonuniform", "bullet", "two_spheres"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-two-spheres", action="store_true", help="skip the two-sphere section")
    ap.add_argument("--form-reps", type=int, default=10)
    return ap.parse_args()


WORKLOADS = {"two_spheres": 1, "bullet": 2, "nonuniform": 4}

# Counter figures of the dominant kernel, from rocprofv3 runs of this script (profiles/):
# HBM bytes per launch (FETCH_SIZE, then WRITE_SIZE, each scaled by what the counter reads
# for the 1 GiB calibration copy) and the L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)).
# They hold only for the kernel sources they were taken on: the hash of those files is
# compared at run time and the figures are dropped on a mismatch.
COUNTERS = {
    "k_adj_pairs_list": {
        "profile": "profiles/hbm_traffic_nonuniform_8388608.md",
        "fetch_bytes": 17094807996.0, "write_bytes": 3465202176.0, "l2_hit_rate": 0.8376,
        "sources_sha256": "6fdbf3b70b0a9dd90d864db6d96d54e949b44a6c5898310a22431a4a8678c743"},
    "k_pairs64_list": {
        "profile": "profiles/hbm_traffic_nonuniform_8388608.md",
        "fetch_bytes": 13632843261.2, "write_bytes": 3370255176.0, "l2_hit_rate": 0.7724,
        "sources_sha256": "25aa29c4db090ac435c66e9ff0c6db71fc994bbec6143f0ef62c3f7e12718909"},
}

KERNEL_SOURCES = {"k_adj_pairs_list": ("adjoint.hip", "adjoint.hpp", "rhs_common.hpp", "common.hpp"),
                  "k_pairs64_list": ("rhs.hip", "rhs_common.hpp", "common.hpp"),
                  "k_adj_L_list": ("adjoint.hip", "adjoint.hpp", "rhs_common.hpp", "common.hpp")}


def sources_sha(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1604_03290_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


HIST_EDGES = [0, 10, 20, 30, 40, 50, 60, 80, 100, 150, 200, 250, 300, 400, 100000]


def log(msg):
    """Progress of the run, one line per stage, on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def approaching_fraction(st, row_ptr, col, torch, chunk=1 << 20):
    """Fraction of ordered pairs with (v_a - v_b) . (x_a - x_b) < 0, which also evaluate
    the artificial viscosity; computed over row blocks to bound memory."""
    n = row_ptr.numel() - 1
    neg, tot = 0, 0
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        a, b = int(row_ptr[r0]), int(row_ptr[r1])
        rows = torch.repeat_interleave(torch.arange(r0, r1, device=row_ptr.device),
                                       row_ptr[r0 + 1:r1 + 1] - row_ptr[r0:r1])
        cl = col[a:b].long()
        wab = ((st.vel[:, rows] - st.vel[:, cl]) * (st.pos[:, rows] - st.pos[:, cl])).sum(0)
        neg += int((wab < 0).sum())
        tot += b - a
    return neg / max(tot, 1)


def partner_stats(row_ptr, torch):
    n = row_ptr.numel() - 1
    dev = row_ptr.device
    deg = (row_ptr[1:] - row_ptr[:-1]).double()
    q = torch.quantile(deg[torch.randperm(n, device=dev)[:1 << 20]],
                       torch.tensor([0.01, 0.5, 0.99], dtype=torch.float64, device=dev))
    return {"min": int(deg.min()), "p01": float(q[0]), "p50": float(q[1]), "p99": float(q[2]),
            "max": int(deg.max()), "mean": float(deg.mean()), "histogram_edges": HIST_EDGES,
            "histogram": torch.bincount(torch.bucketize(deg, torch.tensor(
                HIST_EDGES[1:-1], dtype=torch.float64, device=dev), right=True),
                minlength=len(HIST_EDGES) - 1).tolist()}


def copy_calibration(torch, nbytes=1 << 30):
    """One plain device copy of a known size (read nbytes, write nbytes): under a
    counter run its FETCH_SIZE / WRITE_SIZE give the scale of those counters."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    return nbytes


def median_ms(fn, reps, torch):
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def normwise(got, ref):
    """max |got - ref| / max |ref| of one output field."""
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def oracle_targets(w, k=4096, seed=11):
    """k targets drawn uniformly (seeded) and their partner lists by the oracle's brute
    force (untimed)."""
    import workloads as W
    from oracle import native
    idx = W.subsample(w.n, k, seed)
    csr = native.neighbours(w.pos, w.h, idx)
    return idx, csr


def cpu_baseline(w, idx, csr, budget_s=12.0):
    """The oracle's right-hand side of the sampled targets over their precomputed partner
    lists, repeated until the budget is used, on all host threads and on one."""
    from oracle import native
    nnz = int(csr[0][-1])
    pv = w.param_vector()

    def run(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            native.rhs(w.pos, w.vel, w.rho, w.S, w.m, pv, targets=idx, csr=csr, want_L=False)
            reps += 1
            el = time.perf_counter() - t0
            if el > budget or reps >= 5000:
                return reps, el

    reps, el = run(budget_s)
    cores = native.threads()
    native.set_threads(1)
    reps1, el1 = run(budget_s / 3)
    native.set_threads(cores)
    return {"value": nnz * reps / el, "unit": UNIT, "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "single_core_value": nnz * reps1 / el1,
            "sample": f"{idx.size} targets drawn uniformly from {w.name} ({nnz} ordered pairs), FP64 "
                      f"C oracle right-hand side over partner lists precomputed by its brute force; "
                      f"{reps} repetitions in {el:.1f} s on {cores} threads, {reps1} in {el1:.1f} s on one"}


def cpu_gravity_baseline(w, targets=131072):
    """The gravity oracle beside the GPU form: its tree over every body (built serially)
    and the walks of a sample of bodies, on the host's threads."""
    from oracle import native
    idx = np.linspace(0, w.n - 1, min(targets, w.n)).astype(np.int64)
    t0 = time.perf_counter()
    out = native.gravity(w.pos, w.m, 6.674e-11, 0.5, 0.5 * w.dx, targets=idx)
    el = time.perf_counter() - t0
    terms = int(out["count"].sum())
    return {"terms_per_s": terms / el, "cores": native.threads(), "kind": "oracle",
            "sample": f"tree of all {w.n} bodies and the walks of {idx.size} evenly spaced "
                      f"bodies ({terms} terms) in {el:.2f} s, tree build included"}


def kernel_roofline(kern, nnz, f_app, pl_entries, steps, ms_step):
    """Roofline entry of the step's dominant kernel from the library's event timings."""
    dom = max(kern, key=lambda k: kern[k][0])
    tot_ms, launches = kern[dom]
    avg_ms = tot_ms / max(launches, 1)
    fpp = FLOPS_PER_PAIR[dom]
    impl = IMPL_FLOPS[dom][0] + IMPL_FLOPS[dom][1] * f_app
    achieved = fpp * nnz / (avg_ms * 1e-3) / 1e12
    kname = KERNEL_NAME[dom]
    ctr = COUNTERS.get(kname)
    ok = ctr is not None and ctr["sources_sha256"] == sources_sha(kname)
    roof = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": ctr["fetch_bytes"] + ctr["write_bytes"] if ok else None,
            "traffic_unit": "bytes per launch (HBM read + write, counter-scaled)",
            "traffic_source": ctr["profile"] if ok else None,
            "hbm_GBps": (ctr["fetch_bytes"] + ctr["write_bytes"]) / (avg_ms * 1e-3) / 1e9 if ok else None,
            "l2_hit_rate": ctr["l2_hit_rate"] if ok else None,
            "avg_launch_ms": avg_ms, "launches": launches,
            "flops_per_pair": fpp, "flops_per_pair_implemented": impl,
            "frac_at_implemented_flops": impl * nnz / (avg_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "ordered_pairs_per_launch": nnz,
            "share_of_step": tot_ms / steps / ms_step,
            "other": {k: {"avg_launch_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in kern.items()}}
    gather_b = {"adjoint_pairs": 224, "pairs_fp64": 128, "adjoint_L": 64}.get(dom)
    if gather_b:
        gb = gather_b * pl_entries
        roof["gather"] = {"bytes_per_launch": gb, "achieved_TBps": gb / (avg_ms * 1e-3) / 1e12,
                          "bytes_per_entry": gather_b, "list_entries": pl_entries}
    return roof


def single_state_step(args, w, torch, P, L):
    """The default step on a one-state workload: cells, list, CSR, FP64 RHS, adjoint."""
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, "cuda")
    n = w.n
    skin = 0.0  # one state: the list is the interaction list itself
    lo, hi = P.api.default_box(st.pos, w.h, skin)
    dims, ncells, _ = L.grid_geometry(lo, hi, w.h, skin, CELLS_PER_H)
    ws_build = P.workspace(L.SPH_OP_BUILD, n, ncells)
    ws_pairs = P.workspace(L.SPH_OP_PAIRS, n)
    ws_nb = P.workspace(L.SPH_OP_NEIGHBOURS, n)
    ws_rhs = P.workspace(L.SPH_OP_RHS, n)
    ws_adj = P.workspace(L.SPH_OP_ADJOINT, n)
    box = (lo, hi)
    grid = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=box, ws=ws_build)
    pl_cap = P.sph_build_pairs(grid, st.pos, ws=ws_pairs)
    row_ptr, col = P.sph_neighbours(grid, st.pos, w.h, ws=ws_nb)
    nnz = int(row_ptr[-1].item())
    col_cap = int(col.numel())
    cnt = grid.pairs[1].long()
    cand = int(cnt.sum())
    nbk = (n + 63) // 64
    padded = 64 * int(torch.nn.functional.pad(cnt, (0, nbk * 64 - n)).view(nbk, 64).max(1).values.sum())
    f_app = approaching_fraction(st, row_ptr, col, torch)
    partners = partner_stats(row_ptr, torch)
    del col
    out = P.api.new_deriv(n, vgrad=9, records=True)
    cot = {k: torch.randn(out[k].shape, dtype=torch.float64, device="cuda",
                          generator=torch.Generator("cuda").manual_seed(3)) for k in P.api.DERIV_KEYS}
    holder = {}

    def step():
        g = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=box, ws=ws_build)
        P.sph_build_pairs(g, st.pos, capacity=pl_cap, ws=ws_pairs)
        holder["csr"] = P.sph_neighbours(g, st.pos, w.h, col_cap=col_cap, ws=ws_nb)
        # the forward hands its velocity gradient and operand records to the adjoint (as
        # a reverse-mode caller keeps its forward's intermediates)
        P.sph_rhs(g, st, w.params, "fp64", out=out, ws=ws_rhs)
        holder["grad"] = P.sph_rhs_adjoint(g, st, w.params, cot, ws=ws_adj, vgrad=out["vgrad"],
                                           rec=out["rec"])
        holder["g"] = g

    log(f"{w.name}: {nnz} ordered pairs, list of {padded} entries ({pl_cap} of room); warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    calib = copy_calibration(torch)
    log(f"{w.name}: timing {args.steps} steps")
    L.timing_reset()
    L.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.timing_enable(False)
    ms_step = e0.elapsed_time(e1) / args.steps
    kern = {k: L.timing_read(k) for k in ("pairs_fp64", "adjoint_pairs", "adjoint_L")}
    for wsx in (ws_rhs, ws_adj, ws_nb):
        rc = P.workspace_status(wsx)
        if rc != 0:
            raise RuntimeError(f"device flag {rc}")
    log(f"{w.name}: {ms_step:.3f} ms per step; forms")
    g = holder["g"]
    reps = args.form_reps
    forms = {
        "build_cells": {"ms": median_ms(lambda: P.sph_build_cells(
            st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=box, ws=ws_build), reps, torch)},
        "build_pairs": {"ms": median_ms(lambda: P.sph_build_pairs(g, st.pos, capacity=pl_cap, ws=ws_pairs),
                                        reps, torch), "entries": pl_cap},
        "neighbours_csr": {"ms": median_ms(lambda: P.sph_neighbours(g, st.pos, w.h, col_cap=col_cap, ws=ws_nb),
                                           reps, torch)},
    }
    outs = {}
    for form in ("fp64", "fp32comp"):
        o = P.api.new_deriv(n)
        ms = median_ms(lambda: P.sph_rhs(g, st, w.params, form, out=o, ws=ws_rhs), reps, torch)
        forms[f"rhs_{form}"] = {"ms": ms, "pairs_per_s": nnz / (ms * 1e-3)}
        outs[form] = o
    ms = median_ms(lambda: P.sph_rhs_adjoint(g, st, w.params, cot, ws=ws_adj), reps, torch)
    forms["adjoint_fp64"] = {"ms": ms, "pairs_per_s": nnz / (ms * 1e-3),
                             "note": "forms the velocity gradient itself"}
    ms = median_ms(lambda: P.sph_rhs_adjoint(g, st, w.params, cot, ws=ws_adj, vgrad=out["vgrad"],
                                             rec=out["rec"]), reps, torch)
    forms["adjoint_fp64_vgrad"] = {"ms": ms, "pairs_per_s": nnz / (ms * 1e-3),
                                   "note": "reads the velocity gradient and the operand records "
                                           "sph_rhs wrote (the step's form)"}
    forms["fp32comp_speedup_vs_fp64"] = forms["rhs_fp64"]["ms"] / forms["rhs_fp32comp"]["ms"]
    forms["rhs_fp32comp"]["note"] = ("a second precision, not a speedup: without packed FP32 its "
                                     "vector instructions issue at the FP64 rate, and its 80-byte "
                                     "records fetch the same cache lines as the FP64 ones")
    fields = ("acc", "drho", "dS", "rho_sum")
    forms["rhs_fp32comp"]["normwise_error_vs_fp64_gpu"] = {
        k: float((outs["fp32comp"][k] - outs["fp64"][k]).abs().max() / outs["fp64"][k].abs().max())
        for k in fields}
    sample = None
    if not args.no_cpu_baseline:
        from oracle import native
        log(f"{w.name}: oracle on 4,096 targets")
        idx, csr = oracle_targets(w)
        ref = native.rhs(w.pos, w.vel, w.rho, w.S, w.m, w.param_vector(), targets=idx, csr=csr, want_L=False)
        it = torch.as_tensor(idx, device="cuda")
        for form in ("fp64", "fp32comp"):
            forms[f"rhs_{form}"]["normwise_error_vs_oracle_4096_targets"] = {
                k: normwise(outs[form][k][..., it].cpu().numpy(), ref[k]) for k in fields}
        sample = (idx, csr)
    result = {
        "ms_per_step": ms_step, "value": 2.0 * nnz / (ms_step * 1e-3), "wall_s": wall,
        "config": {"workload": w.name, "particles": n, "ordered_pairs_per_rhs": nnz,
                   "approaching_pair_fraction": f_app, "partners_per_particle": partners,
                   "pair_list": {"room_entries": pl_cap, "padded_entries": padded, "candidates": cand,
                                 "true_pairs_fraction": nnz / cand,
                                 "load_balance_mean_over_max_per_wave": cand / padded},
                   "skin_over_dx": skin / w.dx, "h_over_dx": 2.4, "cells_per_h": CELLS_PER_H,
                   "grid_dims": list(dims), "grid_cells": ncells,
                   "step": "cell build + pair list + partner CSR + FP64 sph_rhs (writing its velocity "
                           "gradient and operand records) + FP64 sph_rhs_adjoint (random cotangent, "
                           "reading them) on one state"},
        "roofline": kernel_roofline(kern, nnz, f_app, padded, args.steps, ms_step),
        "forms": forms,
        "copy_calibration_bytes": calib,
    }
    return result, sample


def fp32_accuracy_section(w, torch, P, reps=5):
    """The bullet-into-cube set: FP64 and FP32-compensated right-hand sides on the pair
    list, and the FP32 form's normwise error per output against the FP64 GPU path and
    against the oracle on 4,096 sampled targets (the FP64 path's error beside it)."""
    from oracle import native
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, "cuda")
    g = P.sph_build_cells(st.pos, w.h, skin=0.0, cells_per_h=CELLS_PER_H, pairs=True)
    ws = P.workspace(P.api.L.SPH_OP_RHS, w.n)
    outs, res = {}, {"particles": w.n, "state": w.name}
    for form in ("fp64", "fp32comp"):
        o = P.api.new_deriv(w.n)
        ms = median_ms(lambda: P.sph_rhs(g, st, w.params, form, out=o, ws=ws), reps, torch)
        outs[form] = o
        res[f"rhs_{form}_ms"] = ms
    fields = ("acc", "drho", "dS", "rho_sum")
    res["fp32comp_normwise_error_vs_fp64_gpu"] = {
        k: float((outs["fp32comp"][k] - outs["fp64"][k]).abs().max() / outs["fp64"][k].abs().max())
        for k in fields}
    idx, csr = oracle_targets(w)
    ref = native.rhs(w.pos, w.vel, w.rho, w.S, w.m, w.param_vector(), targets=idx, csr=csr, want_L=False)
    it = torch.as_tensor(idx, device="cuda")
    for form in ("fp64", "fp32comp"):
        res[f"{form}_normwise_error_vs_oracle_4096_targets"] = {
            k: normwise(outs[form][k][..., it].cpu().numpy(), ref[k]) for k in fields}
    return res


def two_spheres_section(args, w, torch, P, L, full_forms=True):
    """The two-sphere collision: cell build, list, CSR, 10-step leapfrog (11 FP64 right-
    hand sides) and its reverse sweep (11 adjoints) for d KE / d (v0, mu, Y0), with the
    extended forms on the same state."""
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, "cuda")
    dev = "cuda"
    n = w.n
    steps_lf = max(w.steps, 1)
    # skin of the frozen grid and list: three times the largest displacement of one
    # untimed trajectory (skin / 2 must cover every particle's movement), at least 0.02 dx
    g0 = P.sph_build_cells(st.pos, w.h, skin=w.dx, cells_per_h=CELLS_PER_H)
    f0, _ = P.sph_leapfrog(g0, st, w.params, w.dt, steps_lf, checkpoints=False)
    L.check(P.workspace_status(f0._ws))
    dmax = float(((f0.pos - st.pos) ** 2).sum(0).sqrt().max())
    del g0, f0
    skin = max(3.0 * dmax, 0.02 * w.dx)
    lo, hi = P.api.default_box(st.pos, w.h, skin)
    dims, ncells, _ = L.grid_geometry(lo, hi, w.h, skin, CELLS_PER_H)
    box = (lo, hi)
    ws_build = P.workspace(L.SPH_OP_BUILD, n, ncells)
    ws_nb = P.workspace(L.SPH_OP_NEIGHBOURS, n)
    ws_rhs = P.workspace(L.SPH_OP_RHS, n)
    ws_lf = P.workspace(L.SPH_OP_LEAPFROG, n)
    ws_lfa = P.workspace(L.SPH_OP_LEAPFROG_ADJOINT, n)
    ws_adj = P.workspace(L.SPH_OP_ADJOINT, n)
    ws_pairs = P.workspace(L.SPH_OP_PAIRS, n)
    ck = torch.empty(L.checkpoint_bytes(n, steps_lf) // 8, dtype=torch.float64, device=dev)
    fin = P.ParticleState(torch.empty_like(st.pos), torch.empty_like(st.vel), torch.empty_like(st.rho),
                          torch.empty_like(st.S), st.m)
    cot = {"vel": torch.empty_like(st.vel)}
    grad = P.api._fields(n, dev)
    grid = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=box, ws=ws_build)
    row_ptr, col = P.sph_neighbours(grid, st.pos, w.h, ws=ws_nb)
    nnz0 = int(row_ptr[-1].item())
    col_cap = int(col.numel()) + n  # room for pairs formed during the trajectory
    pl_cap = P.sph_build_pairs(grid, st.pos, ws=ws_pairs)

    def step():
        g = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=box, ws=ws_build)
        P.sph_build_pairs(g, st.pos, capacity=pl_cap, ws=ws_pairs)
        P.sph_neighbours(g, st.pos, w.h, col_cap=col_cap, ws=ws_nb)
        P.sph_leapfrog(g, st, w.params, w.dt, steps_lf, checkpoints=ck, out=fin, ws=ws_lf)
        torch.mul(fin.vel, fin.m, out=cot["vel"])  # d KE / d v_final
        P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps_lf, ck, cot, ws=ws_lfa, grad=grad)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    rp_end, _ = P.sph_neighbours(grid, fin.pos, w.h, ws=ws_nb)
    nnz = 0.5 * (nnz0 + int(rp_end[-1].item()))
    reps = max(args.steps, 3)
    ms_step = median_ms(step, reps, torch)
    for wsx in (ws_lf, ws_lfa):
        rc = P.workspace_status(wsx)
        if rc != 0:
            raise RuntimeError(f"device flag {rc}")
    res = {"workload": w.name, "particles": n, "ordered_pairs_per_rhs": nnz, "skin_over_dx": skin / w.dx,
           "leapfrog_step_ms": ms_step,
           "leapfrog_step_pairs_per_s": 2 * (steps_lf + 1) * nnz / (ms_step * 1e-3),
           "leapfrog_step": f"cell build + pair list + partner CSR + {steps_lf}-step leapfrog ({steps_lf + 1} "
                            f"FP64 right-hand sides) + reverse sweep ({steps_lf + 1} adjoints)"}
    if not full_forms:
        return res
    g = grid
    fr = args.form_reps
    forms = {}
    outs = {}
    for form in ("fp64", "fp32comp"):
        o = P.api.new_deriv(n)
        ms = median_ms(lambda: P.sph_rhs(g, st, w.params, form, out=o, ws=ws_rhs), fr, torch)
        forms[f"rhs_{form}"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
        outs[form] = o
    forms["rhs_fp32comp"]["normwise_error_vs_fp64_gpu"] = {
        k: float((outs["fp32comp"][k] - outs["fp64"][k]).abs().max() / outs["fp64"][k].abs().max())
        for k in ("acc", "drho", "dS", "rho_sum")}
    gc = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=box)
    oc = P.api.new_deriv(n)
    ms = median_ms(lambda: P.sph_rhs(gc, st, w.params, "fp64", out=oc, ws=ws_rhs), fr, torch)
    forms["rhs_fp64_cell_sweep"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    # energy equation, artificial stress (eps_s 0.2, n 4, on a copy whose densities are
    # spread by +-0.5 % so that half of the particles are in tension) and XSPH (0.5)
    sx = P.ParticleState(st.pos, st.vel, st.rho * (1.0 + 0.005 * (2.0 * torch.rand(
        n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(5)) - 1.0)),
        st.S, st.m)
    px = dict(w.params, eps_s=0.2, n_s=4.0, xsph=0.5)
    ox = P.api.new_deriv(n, extra=True)
    ms = median_ms(lambda: P.sph_rhs(g, sx, px, "fp64", out=ox, ws=ws_rhs), fr, torch)
    forms["rhs_fp64_energy_artstress_xsph"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3),
                                               "particles_in_tension": int((sx.rho < w.params["rho0"]).sum())}
    ox32 = P.api.new_deriv(n, extra=True)
    ms = median_ms(lambda: P.sph_rhs(g, sx, px, "fp32comp", out=ox32, ws=ws_rhs), fr, torch)
    forms["rhs_fp32comp_energy_artstress_xsph"] = {
        "ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3),
        "normwise_error_vs_fp64_gpu": {k: float((ox32[k] - ox[k]).abs().max() / ox[k].abs().max())
                                       for k in ("acc", "drho", "dS", "du")}}
    # Tillotson (aluminium constants) with u over its cold to vaporised range
    su = P.ParticleState(sx.pos, sx.vel, sx.rho, sx.S, sx.m, 2e7 * torch.rand(
        n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(6)))
    pt = dict(w.params, eos=2.0)
    ot = P.api.new_deriv(n)
    ms = median_ms(lambda: P.sph_rhs(g, su, pt, "fp64", out=ot, ws=ws_rhs), fr, torch)
    forms["rhs_fp64_tillotson"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    # Grady-Kipp damage: d uniform in [0, 1], basalt's Weibull flaws over the bodies
    import workloads as W
    fptr, feps = W.flaws(n, float(np.sum(w.m) / w.params["rho0"]), 1e61, 16.0, 7)
    sd = P.ParticleState(sx.pos, sx.vel, sx.rho, sx.S, sx.m, None, torch.rand(
        n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(8)),
        torch.as_tensor(fptr).to(dev), torch.as_tensor(feps).to(dev))
    od = P.api.new_deriv(n, damage=True)
    ms = median_ms(lambda: P.sph_rhs(g, sd, w.params, "fp64", out=od, ws=ws_rhs), fr, torch)
    forms["rhs_fp64_damage"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3), "flaws": int(fptr[-1]),
                                "particles_with_active_flaws": int((od["n_act"] > 0).sum())}
    cg = {k: torch.randn_like(outs["fp64"][k]) for k in ("acc", "drho", "dS", "rho_sum")}
    ms = median_ms(lambda: P.sph_rhs_adjoint(g, st, w.params, cg, ws=ws_adj), fr, torch)
    forms["adjoint_fp64"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    ms = median_ms(lambda: P.sph_rhs_adjoint(g, su, pt, cg, ws=ws_adj), fr, torch)
    forms["adjoint_fp64_tillotson"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    # Barnes-Hut monopole self-gravity (section 3.3), theta = 0.5, smoothing 0.5 dx
    wsg = P.workspace(P._lib.SPH_OP_GRAVITY, n, 0, dev)
    go = P.sph_gravity(st.pos, st.m, 6.674e-11, 0.5, 0.5 * w.dx, count=True, ws=wsg)
    terms = int(go["count"].to(torch.int64).sum())
    ms = median_ms(lambda: P.sph_gravity(st.pos, st.m, 6.674e-11, 0.5, 0.5 * w.dx, ws=wsg), fr, torch)
    forms["gravity_bh_theta0.5"] = {"ms": ms, "inner_nodes": go["nodes"], "terms": terms,
                                    "terms_per_s": terms / (ms * 1e-3),
                                    "tflops_algorithmic": terms * FLOPS_GRAV_TERM / (ms * 1e-3) / 1e12,
                                    "frac_of_fp64_peak": terms * FLOPS_GRAV_TERM / (ms * 1e-3) / 1e12
                                    / PEAK_FP64_TFLOPS}
    if not args.no_cpu_baseline:
        forms["gravity_bh_theta0.5"]["cpu_oracle"] = cpu_gravity_baseline(w)
    res["forms"] = forms
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the multi-GPU "
                                   "domain decomposition is design only)"}))
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1604_03290_amd as P
    from paper_1604_03290_amd import _lib as L

    k = WORKLOADS[args.workload]
    log(f"generating workload {args.workload}")
    w = W.config(k)
    if args.workload == "two_spheres":
        calib = copy_calibration(torch)
        sec = two_spheres_section(args, w, torch, P, L)
        result = {"metric": METRIC, "value": sec["leapfrog_step_pairs_per_s"], "unit": UNIT, "n_gpus": 1,
                  "steps": max(args.steps, 3), "warmup": args.warmup, "ms_per_step": sec["leapfrog_step_ms"],
                  "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                  "data": "synthetic", "config": {"workload": w.name, "step": sec["leapfrog_step"]},
                  "copy_calibration_bytes": calib, "two_spheres": sec}
        print(json.dumps(result), flush=True)
        return
    res, sample = single_state_step(args, w, torch, P, L)
    result = {
        "metric": METRIC, "value": res["value"], "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": res["config"], "roofline": res["roofline"],
        "forms": res["forms"], "copy_calibration_bytes": res["copy_calibration_bytes"],
        "wall_s": res["wall_s"],
    }
    if sample is not None:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(w, *sample)
        del w
        torch.cuda.empty_cache()
        log("bullet into cube: FP32-compensated accuracy")
        result["bullet_into_cube_2105344"] = {
            state: fp32_accuracy_section(W.config(2, state=state), torch, P)
            for state in ("impact", "random")}
    if not args.no_two_spheres:
        w = None
        torch.cuda.empty_cache()
        log("two-sphere collision section")
        result["two_spheres_262144"] = two_spheres_section(args, W.config(1), torch, P, L)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
