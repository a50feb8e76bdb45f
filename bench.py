#!/usr/bin/env python3
"""Throughput of the SPH solid-body right-hand side on one MI355X.

One step = one pass of the whole hot path over the two-sphere collision
(262,144 particles, 131,072 per sphere, h = 2.4 dx):
  cell build (grid frozen for the trajectory, with a skin)   sph_build_cells
  partner lists (CSR)                                        sph_neighbours
  10 leapfrog steps = 11 FP64 right-hand sides               sph_leapfrog
  reverse sweep: gradient of the final kinetic energy with
  respect to v0, mu and Y0 = 11 adjoint evaluations          sph_leapfrog_adjoint
The metric counts ordered pair interactions (b != a, |x_a - x_b| < h)
evaluated by the right-hand sides and by the adjoint.  Inputs are resident
on the GPU before timing starts.  Per-form rates (FP64 and FP32-compensated
right-hand side, adjoint) are measured on the same input and reported beside
the step.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one
GPU (the multi-GPU decomposition is described in the design notes).
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

# Algorithmic FP64 operations per ordered pair (FMA = 2, square root and division = 1):
# right-hand side = distance, square root, kernel, gradient, density sum, velocity
# gradient, stress bracket, acceleration (83) + the artificial viscosity on approaching
# pairs (10); adjoint pair pass = both roles of the pair (222) + viscosity terms (23).
FLOPS_RHS, FLOPS_RHS_APPROACH = 83.0, 10.0
FLOPS_ADJ, FLOPS_ADJ_APPROACH = 222.0, 23.0
FLOPS_ADJ_L = 45.0  # the adjoint's recomputation of the velocity gradient
# gravity walk, per body taken: distance (3), r^2 (5), opening test (3), force with a
# refined reciprocal square root and the reciprocal of r + eps (11)
FLOPS_GRAV_TERM = 22


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="two_spheres", choices=["two_spheres", "bullet", "nonuniform", "cube40"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form-reps", type=int, default=20)
    return ap.parse_args()


def load_workload(name):
    import workloads as W
    k = {"two_spheres": 1, "bullet": 2, "cube40": 3, "nonuniform": 4}[name]
    w = W.config(k)
    return k, w


# HBM bytes per launch of the dominant kernel, from two rocprofv3 counter runs of this
# script (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads for the
# 1 GiB calibration copy.  They hold only for the kernel sources they were taken on: the
# hash of those files is compared at run time and the figure is dropped on a mismatch.
TRAFFIC = {"kernel": "k_adj_pairs_list", "workload": "two_spheres_262144",
           "sources_sha256": "26e7b6401953907540c9f4b7caa1b19f9ca7aa10af2a02bdba544adfd466d034",
           "fetch_bytes": 806.9e6, "write_bytes": 30.5e6,
           "profile": "profiles/hbm_traffic_two_spheres_262144.md"}

KERNEL_SOURCES = {"k_adj_pairs_list": ("adjoint.hip", "adjoint.hpp", "rhs_common.hpp", "common.hpp"),
                  "k_pairs64_list": ("rhs.hip", "rhs_common.hpp", "common.hpp")}


def sources_sha(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1604_03290_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


HIST_EDGES = [0, 10, 20, 30, 40, 50, 60, 80, 100, 150, 200, 250, 300, 400, 100000]


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


def cpu_baseline(w, budget_s=12.0):
    """The oracle's right-hand side on a spatially contiguous sample of the workload
    (the particles nearest the sample centre), partner lists precomputed by the oracle's
    brute force (not timed), repeated until the budget is used."""
    from oracle import native
    n_sample = min(w.n, 32768)
    c = w.pos.mean(1)
    d2 = ((w.pos - c[:, None]) ** 2).sum(0)
    idx = np.sort(np.argpartition(d2, n_sample - 1)[:n_sample])
    sub = w.take(idx)
    csr = native.neighbours(sub.pos, sub.h)
    nnz = int(csr[0][-1])
    pv = sub.param_vector()
    reps, t0 = 0, time.perf_counter()
    while True:
        native.rhs(sub.pos, sub.vel, sub.rho, sub.S, sub.m, pv, csr=csr, want_L=False)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 5000:
            break
    rate = nnz * reps / el
    cores = native.threads()
    # one core, as the paper's own CPU comparison (a shorter budget)
    native.set_threads(1)
    reps1, t0 = 0, time.perf_counter()
    while True:
        native.rhs(sub.pos, sub.vel, sub.rho, sub.S, sub.m, pv, csr=csr, want_L=False)
        reps1 += 1
        el1 = time.perf_counter() - t0
        if el1 > budget_s / 3 or reps1 >= 5000:
            break
    native.set_threads(cores)
    return {"value": rate, "unit": UNIT, "cores": cores, "kind": "oracle",
            "single_core_value": nnz * reps1 / el1,
            "sample": f"{n_sample} particles nearest the centre of {w.name} ({nnz} ordered pairs), "
                      f"FP64 C oracle right-hand side over precomputed partner lists, {reps} repetitions "
                      f"in {el:.1f} s on {cores} threads; {reps1} repetitions in {el1:.1f} s on one"}


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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU "
                                   "domain decomposition is design-only)"}))
        sys.exit(2)
    import torch
    import paper_1604_03290_amd as P
    from paper_1604_03290_amd import _lib as L

    k, w = load_workload(args.workload)
    dev = "cuda"
    st = P.ParticleState.from_arrays(w.pos, w.vel, w.rho, w.S, w.m, dev)
    steps_lf = max(w.steps, 1)
    # Skin of the frozen grid and list: twice the largest displacement the trajectory makes,
    # with 50 % margin (skin / 2 must cover every particle's movement; the device flag
    # STALE_GRID would end the run otherwise), at least 0.02 dx.  The displacement is
    # measured on one untimed trajectory under a grid with a generous skin of one dx.
    g0 = P.sph_build_cells(st.pos, w.h, skin=w.dx, cells_per_h=CELLS_PER_H)  # cell sweeps, no list
    f0, _ = P.sph_leapfrog(g0, st, w.params, w.dt, steps_lf, checkpoints=False)
    L.check(P.workspace_status(f0._ws))
    dmax = float(((f0.pos - st.pos) ** 2).sum(0).sqrt().max())
    del g0, f0
    skin = max(3.0 * dmax, 0.02 * w.dx)
    lo, hi = P.api.default_box(st.pos, w.h, skin)
    dims, ncells, _ = L.grid_geometry(lo, hi, w.h, skin, CELLS_PER_H)
    n = w.n
    ws_build = P.workspace(L.SPH_OP_BUILD, n, ncells)
    ws_nb = P.workspace(L.SPH_OP_NEIGHBOURS, n)
    ws_rhs = P.workspace(L.SPH_OP_RHS, n)
    out = P.api.new_deriv(n)

    ws_lf = P.workspace(L.SPH_OP_LEAPFROG, n)
    ws_lfa = P.workspace(L.SPH_OP_LEAPFROG_ADJOINT, n)
    ws_adj = P.workspace(L.SPH_OP_ADJOINT, n)
    ck = torch.empty(L.checkpoint_bytes(n, steps_lf) // 8, dtype=torch.float64, device=dev)
    fin = P.ParticleState(torch.empty_like(st.pos), torch.empty_like(st.vel), torch.empty_like(st.rho),
                          torch.empty_like(st.S), st.m)
    cot = {"vel": torch.empty_like(st.vel)}
    grad = P.api._fields(n, dev)

    grid = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=(lo, hi), ws=ws_build)
    row_ptr, col = P.sph_neighbours(grid, st.pos, w.h, ws=ws_nb)
    nnz0 = int(row_ptr[-1].item())
    # fraction of ordered pairs that approach (w_ab < 0): they also evaluate Pi
    f_app = approaching_fraction(st, row_ptr, col, torch)
    deg = (row_ptr[1:] - row_ptr[:-1]).double()
    q = torch.quantile(deg[torch.randperm(n, device=dev)[:1 << 20]],
                       torch.tensor([0.01, 0.5, 0.99], dtype=torch.float64, device=dev))
    partners = {"min": int(deg.min()), "p01": float(q[0]), "p50": float(q[1]), "p99": float(q[2]),
                "max": int(deg.max()), "mean": float(deg.mean()),
                "histogram_edges": HIST_EDGES,
                "histogram": torch.bincount(torch.bucketize(deg, torch.tensor(
                    HIST_EDGES[1:-1], dtype=torch.float64, device=dev), right=True),
                    minlength=len(HIST_EDGES) - 1).tolist()}
    del deg
    col_cap = int(col.numel()) + n  # room for pairs formed during the trajectory

    ws_pairs = P.workspace(L.SPH_OP_PAIRS, n)
    pl_cap = P.sph_build_pairs(grid, st.pos, ws=ws_pairs)
    cand = int(grid.pairs[1].long().sum())
    # load balance = mean over max list length per wavefront, summed over wavefronts
    pair_list = {"entries": pl_cap, "candidates": cand, "true_pairs_fraction": nnz0 / cand,
                 "load_balance_mean_over_max_per_wave": cand / pl_cap}

    def step():
        g = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=(lo, hi), ws=ws_build)
        P.sph_build_pairs(g, st.pos, capacity=pl_cap, ws=ws_pairs)
        P.sph_neighbours(g, st.pos, w.h, col_cap=col_cap, ws=ws_nb)
        P.sph_leapfrog(g, st, w.params, w.dt, steps_lf, checkpoints=ck, out=fin, ws=ws_lf)
        torch.mul(fin.vel, fin.m, out=cot["vel"])  # d KE / d v_final
        P.sph_leapfrog_adjoint(g, st, w.params, w.dt, steps_lf, ck, cot, ws=ws_lfa, grad=grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rp_end, _ = P.sph_neighbours(grid, fin.pos, w.h, ws=ws_nb)
    nnz1 = int(rp_end[-1].item())
    nnz = 0.5 * (nnz0 + nnz1)
    pairs_per_step = 2 * (steps_lf + 1) * nnz
    step_desc = (f"cell build + frozen pair list + partner CSR + {steps_lf}-step leapfrog ({steps_lf + 1} "
                 f"FP64 right-hand sides) + reverse sweep ({steps_lf + 1} adjoints) for d KE / d (v0, mu, Y0)")

    calib = copy_calibration(torch)
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
    for wsx in (ws_lf, ws_lfa):
        rc = P.workspace_status(wsx)
        if rc != 0:
            raise RuntimeError(f"device flag {rc}")

    # per-form rates on the initial state (median of reps); the right-hand side and the
    # adjoint read the frozen pair list, the "cells" form sweeps the cell rows instead
    g = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=(lo, hi), ws=ws_build)
    forms = {"build_cells": {"ms": median_ms(
        lambda: P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=(lo, hi), ws=ws_build), args.form_reps, torch)}}
    forms["build_pairs"] = {"ms": median_ms(
        lambda: P.sph_build_pairs(g, st.pos, capacity=pl_cap, ws=ws_pairs), args.form_reps, torch),
        "entries": pl_cap}
    forms["neighbours_csr"] = {"ms": median_ms(
        lambda: P.sph_neighbours(g, st.pos, w.h, col_cap=col_cap, ws=ws_nb), args.form_reps, torch)}
    gc = P.sph_build_cells(st.pos, w.h, skin=skin, cells_per_h=CELLS_PER_H, box=(lo, hi))
    oc = P.api.new_deriv(n)
    ms = median_ms(lambda: P.sph_rhs(gc, st, w.params, "fp64", out=oc, ws=ws_rhs), args.form_reps, torch)
    forms["rhs_fp64_cell_sweep"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    outs = {}
    for form in ("fp64", "fp32comp"):
        o = P.api.new_deriv(n)
        ms = median_ms(lambda: P.sph_rhs(g, st, w.params, form, out=o, ws=ws_rhs), args.form_reps, torch)
        forms[f"rhs_{form}"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
        outs[form] = o
    fields = {"acc": 3, "drho": 1, "dS": 6, "rho_sum": 1}
    errs = {}
    for k in fields:
        ref = outs["fp64"][k]
        errs[k] = float((outs["fp32comp"][k] - ref).abs().max() / ref.abs().max())
    forms["rhs_fp32comp"]["normwise_error_vs_fp64"] = errs
    # the next rows of the pair loop: energy equation, artificial stress (eps_s 0.2, n 4,
    # on a copy of the state whose densities are spread by +-0.5 % so that half of the
    # particles are in tension) and XSPH (0.5), FP64, same list
    sx = P.ParticleState(st.pos, st.vel, st.rho * (1.0 + 0.005 * (2.0 * torch.rand(
        n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(5)) - 1.0)),
        st.S, st.m)
    px = dict(w.params, eps_s=0.2, n_s=4.0, xsph=0.5)
    ox = P.api.new_deriv(n, extra=True)
    ms = median_ms(lambda: P.sph_rhs(g, sx, px, "fp64", out=ox, ws=ws_rhs), args.form_reps, torch)
    forms["rhs_fp64_energy_artstress_xsph"] = {
        "ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3),
        "particles_in_tension": int((sx.rho < w.params["rho0"]).sum())}
    ox32 = P.api.new_deriv(n, extra=True)
    ms = median_ms(lambda: P.sph_rhs(g, sx, px, "fp32comp", out=ox32, ws=ws_rhs), args.form_reps, torch)
    forms["rhs_fp32comp_energy_artstress_xsph"] = {
        "ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3),
        "normwise_error_vs_fp64": {k: float((ox32[k] - ox[k]).abs().max() / ox[k].abs().max())
                                   for k in ("acc", "drho", "dS", "du")}}
    # Tillotson equation of state (aluminium constants) on the same spread densities with
    # specific internal energies drawn over its cold, partial and full vaporisation ranges
    su = P.ParticleState(sx.pos, sx.vel, sx.rho, sx.S, sx.m, 2e7 * torch.rand(
        n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(6)))
    pt = dict(w.params, eos=2.0)
    ot = P.api.new_deriv(n)
    ms = median_ms(lambda: P.sph_rhs(g, su, pt, "fp64", out=ot, ws=ws_rhs), args.form_reps, torch)
    forms["rhs_fp64_tillotson"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    # Grady-Kipp damage on the spread densities: damage uniform in [0, 1], flaws of
    # basalt's Weibull law (k = 1e61 m^-3, m = 16) over the bodies' volume, about
    # N ln N of them; the damaged stress in the pair loop and the damage rates
    import workloads as W
    fptr, feps = W.flaws(n, float(np.sum(w.m) / w.params["rho0"]), 1e61, 16.0, 7)
    sd = P.ParticleState(sx.pos, sx.vel, sx.rho, sx.S, sx.m, None, torch.rand(
        n, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(8)),
        torch.as_tensor(fptr).to(dev), torch.as_tensor(feps).to(dev))
    od = P.api.new_deriv(n, damage=True)
    ms = median_ms(lambda: P.sph_rhs(g, sd, w.params, "fp64", out=od, ws=ws_rhs), args.form_reps, torch)
    forms["rhs_fp64_damage"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3), "flaws": int(fptr[-1]),
                                "particles_with_active_flaws": int((od["n_act"] > 0).sum())}
    # Barnes-Hut monopole self-gravity (section 3.3) on the same bodies, theta = 0.5 (the
    # paper's bound), smoothing 0.5 dx: tree build and walk in one call (it synchronises
    # once to size the tree); terms = pseudo-particles and leaves summed over particles
    mt = st.m
    wsg = P.workspace(P._lib.SPH_OP_GRAVITY, n, 0, dev)
    go = P.sph_gravity(st.pos, mt, 6.674e-11, 0.5, 0.5 * w.dx, count=True, ws=wsg)
    terms = int(go["count"].to(torch.int64).sum())
    ms = median_ms(lambda: P.sph_gravity(st.pos, mt, 6.674e-11, 0.5, 0.5 * w.dx, ws=wsg),
                   args.form_reps, torch)
    forms["gravity_bh_theta0.5"] = {"ms": ms, "inner_nodes": go["nodes"], "terms": terms,
                                    "terms_per_s": terms / (ms * 1e-3),
                                    "tflops_algorithmic": terms * FLOPS_GRAV_TERM / (ms * 1e-3) / 1e12,
                                    "frac_of_fp64_peak": terms * FLOPS_GRAV_TERM / (ms * 1e-3) / 1e12
                                    / PEAK_FP64_TFLOPS}
    forms["fp32comp_speedup_vs_fp64"] = forms["rhs_fp64"]["ms"] / forms["rhs_fp32comp"]["ms"]
    cg = {k: torch.randn_like(outs["fp64"][k]) for k in fields}
    ms = median_ms(lambda: P.sph_rhs_adjoint(g, st, w.params, cg, ws=ws_adj), args.form_reps, torch)
    forms["adjoint_fp64"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}
    # the adjoint with the Tillotson equation (gradient of u too; cell-sweep pair kernel)
    ms = median_ms(lambda: P.sph_rhs_adjoint(g, su, pt, cg, ws=ws_adj), args.form_reps, torch)
    forms["adjoint_fp64_tillotson"] = {"ms": ms, "pairs_per_s": nnz0 / (ms * 1e-3)}

    # dominant kernel of the step
    dom = max(kern, key=lambda k: kern[k][0])
    tot_ms, launches = kern[dom]
    avg_ms = tot_ms / max(launches, 1)
    fpp = {"pairs_fp64": FLOPS_RHS + FLOPS_RHS_APPROACH * f_app,
           "adjoint_pairs": FLOPS_ADJ + FLOPS_ADJ_APPROACH * f_app,
           "adjoint_L": FLOPS_ADJ_L}[dom]
    achieved = fpp * nnz / (avg_ms * 1e-3) / 1e12
    kname = {"pairs_fp64": "k_pairs64_list", "adjoint_pairs": "k_adj_pairs_list", "adjoint_L": "k_adj_L_list"}[dom]
    traffic = None
    if TRAFFIC and TRAFFIC["kernel"] == kname and TRAFFIC["workload"] == w.name and \
            TRAFFIC["sources_sha256"] == sources_sha(kname):
        traffic = TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]
    roofline = {"bound": "alu",
                "kernel": kname,
                "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM read + write, counter-scaled)",
                "traffic_source": TRAFFIC["profile"] if traffic else None,
                "avg_launch_ms": avg_ms, "launches": launches, "flops_per_pair": fpp,
                "share_of_step": tot_ms / args.steps / ms_step,
                "other": {k: {"avg_launch_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in kern.items()}}
    # the gather view of the same launch: partner bytes moved through the L1 per launch
    # (every padded list entry loads its partner's chunks: 7 + 7 chunks of 16 B for the
    # adjoint, 8 for the forward), at the kernel's average duration
    gather_b = {"adjoint_pairs": 224, "pairs_fp64": 128}.get(dom)
    if gather_b:
        gb = gather_b * pl_cap
        roofline["gather"] = {"bytes_per_launch": gb, "achieved_TBps": gb / (avg_ms * 1e-3) / 1e12,
                              "bytes_per_entry": gather_b, "list_entries": pl_cap}

    result = {
        "metric": METRIC, "value": pairs_per_step / (ms_step * 1e-3), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "particles": n, "ordered_pairs_per_rhs": nnz,
                   "ordered_pairs_start_end": [nnz0, nnz1], "skin_over_dx": skin / w.dx,
                   "approaching_pair_fraction": f_app, "partners_per_particle": partners,
                   "pair_list": pair_list,
                   "h_over_dx": 2.4, "cells_per_h": CELLS_PER_H, "leapfrog_steps": steps_lf, "step": step_desc,
                   "grid_dims": list(dims)},
        "roofline": roofline,
        "forms": forms,
        "copy_calibration_bytes": calib,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w)
        forms["gravity_bh_theta0.5"]["cpu_oracle"] = cpu_gravity_baseline(w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
