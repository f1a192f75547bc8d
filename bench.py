"""Benchmark of the same-level M2L hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 4096 independent 8^3 sub-grids (24^3 frames, 8 point masses per
cell, lognormal masses, seeded synthetic inputs), expansion order p = 3
(C = 20), the 892-offset shell stencil, float64. A step is the forward hot
path on that batch with inputs resident in HBM: P2M (point masses -> cell
moments, over the frame rows that hold the reachable 20^3 window: the cells M2L
reads) then M2L (moments -> local coefficients of the 512 targets of every
sub-grid) in float64, computed in the harmonic (traceless) form: (p+1)^2 = 16
folded moment components against 16 local columns, then expanded to all 20.
Both run in one persistent launch (fmm_p2m_m2l), each workgroup computing a
sub-grid's moments during the M2L of the sub-grid before it. `value` is
cell-pair interactions per second over the whole step. The same step as two
launches (P2M, then the M2L-only kernel) and the dense 20 x 20 form of the
M2L are timed as extras.

The same run also measures, each on its own batch: the split-precision M2L
(float32 matrix cores, hi/lo products) on the step's moments, with its error
against the FP64 result; forward + backward (P2M, M2L, adjoint M2L, adjoint P2M)
on 2048 sub-grids; the evaluation at the particles (near field over the 33
cells with |d|^2 <= 4 plus L2P of the step's L); the multi-level iteration
on a 128^3 domain (16.8M particles); the uneven batch (6000 sub-grids, p in {2,3,4} as 1:2:1,
h in {1,1/2,1/4}, random boundary masks) in one persistent launch; and the
CPU oracle on a bounded sample of the step's workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402

METRIC = "M2L cell-pair interactions/s FP64 vs split-FP32 (<=1e-10 rel); fwd+bwd ms/batch"
FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
FP32_PEAK_TFLOPS = 157.3    # MI355X dense FP32 matrix peak
INT8_PEAK_TOPS = 5000.0     # MI355X dense int8 matrix peak
HBM_PEAK_GBS = 8000.0
# the step's kernel: the M2L kernel source and the moment phase it includes
STEP_SRCS = [os.path.join(ROOT, "paper_2304_11002_amd", "csrc", f) for f in ("m2l_mfma.hip", "p2m_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "p2m_m2l_fused_uniform4096_p3_traffic.txt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def flops_per_pair(p):
    """Dense form: 2 C^2 FLOP per (target, offset) pair."""
    C = (p + 1) * (p + 2) * (p + 3) // 6
    return 2 * C * C


def harmonic_flops_per_pair(p):
    """Harmonic form: 2 (p+1)^4 FLOP per pair (the executed matrix-core work)."""
    return 2 * (p + 1) ** 4


# ---------------------------------------------------------------------------
# device helpers
# ---------------------------------------------------------------------------

def upload_batch(torch, w):
    t0 = time.time()
    with synth.SharedBatch(w) as sb:
        pos = torch.from_numpy(sb.pos).to("cuda")
        mass = torch.from_numpy(sb.mass).to("cuda")
        torch.cuda.synchronize()
    log("generated + uploaded %s (%d sub-grids) in %.1f s" % (w.name, w.nsub, time.time() - t0))
    return pos, mass


def timed(torch, fn, steps, warmup, marks=1):
    """Run fn(events, i) warmup+steps times; fn records `marks`+1 events per step.
    Returns (wall seconds of the timed steps, per-segment event ms arrays)."""
    for i in range(warmup):
        fn(None, i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(marks + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn(evs[i], i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    seg = np.array([[evs[i][j].elapsed_time(evs[i][j + 1]) for j in range(marks)] for i in range(steps)])
    return wall, seg


# FP64 operations of one near-field pair as executed: 3 differences, r^2 (1 mul,
# 2 fma), the float estimate of 1/r refined by one second-order step (1 mul,
# 3 fma, 1 mul), m/r, 1/r^2, m/r^3, the potential add and 3 gradient fma:
# 19 operations, 8 of them fused multiply-adds, 27 FLOP (the float estimate and
# its two conversions are not counted).
NEAR_FLOPS_PER_PAIR = 27


def l2p_flops(p):
    """Contraction flops of L2P per particle: C fma for the potential and
    3 C(p-1) for the gradient."""
    C = (p + 1) * (p + 2) * (p + 3) // 6
    Cm = p * (p + 1) * (p + 2) // 6
    return 2 * (C + 3 * Cm)


def near_pair_count(desc, ppc):
    """Particle pairs of the near field over the batch: for every target
    particle, the particles of the present cells among the 33 with |d|^2 <= 4,
    less itself."""
    offs = [(dx, dy, dz) for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)
            if dx * dx + dy * dy + dz * dz <= 4]
    cache, total = {}, 0
    for m in desc["mask"]:
        m = int(m)
        if m not in cache:
            bits = np.array([(m >> b) & 1 for b in range(27)], bool).reshape(3, 3, 3)   # [bz][by][bx]
            pres = np.repeat(np.repeat(np.repeat(bits, 8, 0), 8, 1), 8, 2)             # [z][y][x]
            cells = 0
            for dx, dy, dz in offs:
                cells += int(pres[8 + dz:16 + dz, 8 + dy:16 + dy, 8 + dx:16 + dx].sum())
            cache[m] = cells * ppc * ppc - 512 * ppc
        total += cache[m]
    return total


def rel_to_component_max(L_test, L_ref, desc, fmm):
    """|L_test - L_ref| relative to the largest |L_ref| of the same component and
    sub-grid, max and median over all entries (both on the device)."""
    import torch
    rel = []
    for b in range(len(desc)):
        C = fmm.ncomp(int(desc["p"][b]))
        o = int(desc["l_off"][b])
        r = L_ref[o:o + C * 512].view(C, 512)
        d = (L_test[o:o + C * 512].view(C, 512) - r).abs() / r.abs().amax(dim=1, keepdim=True)
        rel.append(d.reshape(-1))
    rel = torch.cat(rel)
    return {"max": float(rel.max()), "median": float(rel.median())}


def tree_pairs(n):
    """(target cell, source cell) pairs of the multi-level M2L over all levels
    (sources inside the domain), and the executed matrix-core slots (every
    level's blocks x 512 targets x 232 list slots)."""
    sets = []
    for sig in range(8):
        sg = (sig & 1, (sig >> 1) & 1, sig >> 2)
        lst = []
        for dz in range(-6, 7):
            for dy in range(-6, 7):
                for dx in range(-6, 7):
                    d = (dx, dy, dz)
                    if dx * dx + dy * dy + dz * dz <= 4:
                        continue
                    D = [(a + b) // 2 for a, b in zip(sg, d)]
                    if D[0] ** 2 + D[1] ** 2 + D[2] ** 2 <= 4:
                        lst.append(d)
        sets.append((sg, lst))
    pairs, slots, m = 0, 0, n
    while m >= 4:
        for sg, lst in sets:
            for d in lst:
                c = 1
                for a in range(3):
                    c *= sum(1 for T in range(m // 2) if 0 <= 2 * T + sg[a] + d[a] < m)
                pairs += c
        slots += max(1, m // 8) ** 3 * 512 * 232
        m //= 2
    return pairs, slots


def bench_tree(torch, fmm, ctx, K, W):
    """Multi-level solve (P2M, M2M, interaction-list M2L on every level, L2L,
    near field + L2P) on a 128^3 domain with 8 particles per cell, p = 3."""
    n, ppc, p = 128, 8, 3
    tree = fmm.Tree(p, n, ppc, 0, 1)      # harmonic form of the level M2L
    dense = fmm.Tree(p, n, ppc, 0, 0)
    _, elems = fmm.tree_size(tree)
    t0 = time.time()
    pos_h, mass_h = synth.grid_particles(40, n, 1.0, ppc)
    pos, mass = torch.from_numpy(pos_h).to("cuda"), torch.from_numpy(mass_h).to("cuda")
    log("generated + uploaded tree_128_p3 in %.1f s" % (time.time() - t0))
    M = torch.empty(elems, dtype=torch.float64, device="cuda")
    L = torch.empty(elems, dtype=torch.float64, device="cuda")
    E = torch.empty(4 * n ** 3 * ppc, dtype=torch.float64, device="cuda")

    def step_tree(ev, i):
        if ev: ev[0].record()
        ctx.tree_upward(tree, pos, mass, M)
        if ev: ev[1].record()
        ctx.tree_m2l(tree, M, L)
        if ev: ev[2].record()
        ctx.tree_downward(tree, L)
        if ev: ev[3].record()
        ctx.tree_evaluate(tree, pos, mass, L, E)
        if ev: ev[4].record()

    wall, seg = timed(torch, step_tree, K, W, marks=4)
    up, m2l, down, ev = (float(seg[:, i].mean()) for i in range(4))
    Ld = torch.empty_like(L)

    def step_dense(ev_, i):
        if ev_: ev_[0].record()
        ctx.tree_m2l(dense, M, Ld)
        if ev_: ev_[1].record()

    _, seg_d = timed(torch, step_dense, K, W, marks=1)
    m2l_dense = float(seg_d[:, 0].mean())
    del Ld
    pairs, slots = tree_pairs(n)
    fl = slots * harmonic_flops_per_pair(p)
    fl_dense = slots * flops_per_pair(p)
    assert bool(torch.isfinite(E).all())
    nparts = n ** 3 * ppc
    ms = wall / K * 1e3
    res = {"workload": "tree_128_p3", "domain_cells": n ** 3, "levels": 6, "particles": nparts,
           "solve_ms": ms, "particles_per_s": nparts / (ms * 1e-3),
           "upward_ms": up, "m2l_ms": m2l, "downward_ms": down, "evaluate_ms": ev,
           "m2l_pairs": pairs, "m2l_pairs_per_s": pairs / (m2l * 1e-3), "m2l_form": "harmonic",
           "m2l_dense_ms": m2l_dense, "m2l_dense_tflops": fl_dense / (m2l_dense * 1e-3) / 1e12,
           "roofline_m2l": {"bound": "mfma", "kernel": "m2l_level_kernel<3, true, 2> (levels 128, 64) + m2l_level_kernel<3, true, 1> (levels 32..4), v_mfma_f64_4x4x4, harmonic form; time of the fmm_tree_m2l call",
                            "achieved": fl / (m2l * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": fl / (m2l * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "traffic": None,
                            "executed_flops": fl, "flops_per_slot": harmonic_flops_per_pair(p),
                            "fp64_dense_equivalent_tflops": fl_dense / (m2l * 1e-3) / 1e12,
                            "useful_slot_fraction": pairs / slots},
           "parity": "tests/test_gpu_tree.py, tests/test_gpu_fullsize.py::test_tree_128_solve"}
    log("tree 128^3: solve %.3f ms (upward %.3f, M2L %.3f, downward %.3f, evaluate %.3f), M2L %.1f TFLOP/s executed;"
        " dense-form M2L %.3f ms" % (ms, up, m2l, down, ev, fl / (m2l * 1e-3) / 1e12, m2l_dense))
    del pos, mass, M, L, E
    return res


# ---------------------------------------------------------------------------
# CPU baseline: the oracle itself on a bounded sample, one process per core
# ---------------------------------------------------------------------------

def _oracle_worker(args):
    """Oracle P2M + M2L over this worker's share of the step's sub-grids until
    `budget` seconds of oracle time are spent; input generation is not timed."""
    seed, ids, budget = args
    from threadpoolctl import threadpool_limits
    import oracle as O
    n, busy = 0, 0.0
    with threadpool_limits(1):
        for b in ids:
            pos, mass = synth.subgrid_particles(seed, b)
            t0 = time.perf_counter()
            M = O.p2m(pos, mass, 3, 1.0)
            O.m2l(M, 3, 1.0)
            busy += time.perf_counter() - t0
            n += 1
            if busy >= budget:
                break
    return n, busy


def cpu_baseline(nsub, budget, seed=2):
    from multiprocessing import get_context
    cores = min(16, len(os.sched_getaffinity(0)))
    jobs = [(seed, list(range(w, nsub, cores)), budget) for w in range(cores)]
    with get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_worker, [(seed, [w], 0.0) for w in range(cores)])   # warm imports
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    per_sub = 512 * 892
    value = sum(n * per_sub / t for n, t in res if t > 0)       # all cores run at once
    done = sum(n for n, _ in res)
    return {"value": value, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": "%d of the step's %d sub-grids (seed 2, p=3), P2M + M2L each, NumPy float64, "
                      "one process per core with 1 BLAS thread, about %.0f s of oracle time per core "
                      "(input generation untimed); value = sum over cores of pairs / busy seconds"
                      % (done, nsub, max(t for _, t in res))}


# ---------------------------------------------------------------------------

def read_traffic(launch_pairs):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in STEP_SRCS)).hexdigest()[:16]
    if kv.get("kernel_source_sha256_16") != sha:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_fwd_bwd(torch, fmm, ctx, K, W):
    """Forward (P2M + M2L, one launch) and backward (M2L adjoint + P2M adjoint, one
    launch) on the 2048-sub-grid gradient batch, harmonic forms, loss = sum w . L."""
    w5 = synth.config(5)
    d5, m5, l5 = fmm.make_descriptors(w5.p, w5.log2_inv_h, w5.mask)
    pairs5 = fmm.pair_count(d5)
    pos5, mass5 = upload_batch(torch, w5)
    wt = torch.from_numpy(synth.loss_weights(w5.seed, w5.nsub)).to("cuda").reshape(-1)
    M5 = torch.empty(m5, dtype=torch.float64, device="cuda")
    L5 = torch.empty(l5, dtype=torch.float64, device="cuda")
    dM5 = torch.empty_like(M5)
    dm5 = torch.empty_like(mass5)

    def step_fb(ev, i):
        if ev: ev[0].record()
        ctx.p2m_m2l(d5, pos5, mass5, 8, M5, L5, fmm.FMM_FP64_HARMONIC)
        if ev: ev[1].record()
        ctx.m2l_p2m_backward(d5, pos5, 8, wt, dM5, dm5)   # dLoss/dL = w for loss = sum w . L
        if ev: ev[2].record()

    ctx.p2m(d5, pos5, mass5, 8, M5)
    tuned5 = ctx.autotune(d5, M5, L5, fmm.FMM_FP64_HARMONIC)
    prev = ctx.get_option(fmm.FMM_OPT_ADJOINT_FORM)
    ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 1)      # harmonic adjoint with the harmonic forward
    try:
        wall_fb, seg_fb = timed(torch, step_fb, max(3, K // 2), W, marks=2)
        fwd_ms, bwd_ms = seg_fb[:, 0].mean(), seg_fb[:, 1].mean()

        # the M2L adjoint alone (no mass-gradient phase), on the same dL
        def step_adj(ev, i):
            if ev: ev[0].record()
            ctx.m2l_backward(d5, wt, dM5)
            if ev: ev[1].record()
        _, seg_adj = timed(torch, step_adj, max(3, K // 2), 1, marks=1)
        adj_ms = seg_adj[:, 0].mean()
        ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 0)
        _, seg_fbd = timed(torch, step_fb, max(3, K // 2), 1, marks=2)
        bwd_dense_ms = seg_fbd[:, 1].mean()
    finally:
        ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, prev)
    assert bool(torch.isfinite(dm5).all())
    fl_h = pairs5 * harmonic_flops_per_pair(3)       # executed matrix flops, each direction
    fl_d = pairs5 * flops_per_pair(3)
    out = {"workload": "grad_2048_p3", "subgrids": w5.nsub, "pairs": pairs5,
           "forward": "P2M + M2L (harmonic form), one launch (fmm_p2m_m2l)",
           "backward": "M2L adjoint (harmonic form) + P2M adjoint, one launch (fmm_m2l_p2m_backward)",
           "bwd_ms_dense_adjoint": float(bwd_dense_ms),
           "m2l_adjoint_only_ms": float(adj_ms),
           "fwd_ms": float(fwd_ms), "bwd_ms": float(bwd_ms),
           "fwd_bwd_ms_per_batch": float(fwd_ms + bwd_ms),
           "bwd_over_fwd": float(bwd_ms / fwd_ms),
           "forward_autotune_choice": tuned5,
           "roofline": {"bound": "mfma", "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "flops_per_launch": fl_h, "flops_per_pair": harmonic_flops_per_pair(3),
                        "fwd_achieved": fl_h / (fwd_ms * 1e-3) / 1e12,
                        "fwd_frac": fl_h / (fwd_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "bwd_achieved": fl_h / (bwd_ms * 1e-3) / 1e12,
                        "bwd_frac": fl_h / (bwd_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "bwd_dense_adjoint_frac": fl_d / (bwd_dense_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "m2l_adjoint_only_frac": fl_h / (adj_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "note": "executed matrix flops of the M2L (or its adjoint) over the whole launch, "
                                "which also holds the HBM-bound moment (or mass-gradient) phase"}}
    log("fwd+bwd 2048: fwd %.3f ms (%.1f%%), bwd %.3f ms (%.1f%%); M2L adjoint alone %.3f ms (%.1f%%)"
        % (fwd_ms, 100 * out["roofline"]["fwd_frac"], bwd_ms, 100 * out["roofline"]["bwd_frac"],
           adj_ms, 100 * out["roofline"]["m2l_adjoint_only_frac"]))
    del pos5, mass5, wt, M5, L5, dM5, dm5
    torch.cuda.empty_cache()
    return out


def bench_uneven(torch, fmm, ctx, K, W):
    """The 6000-sub-grid uneven batch (mixed p, masks, spacings) in one persistent
    launch, harmonic and dense forms, each with its autotuned configuration."""
    w3 = synth.config(3)
    d3, m3, l3 = fmm.make_descriptors(w3.p, w3.log2_inv_h, w3.mask)
    pairs3 = fmm.pair_count(d3)
    per = np.array([fmm.pair_count(d3[i:i + 1]) for i in range(w3.nsub)], dtype=np.float64)
    fl3 = float(sum(per[i] * flops_per_pair(int(w3.p[i])) for i in range(w3.nsub)))
    fl3h = float(sum(per[i] * harmonic_flops_per_pair(int(w3.p[i])) for i in range(w3.nsub)))
    pos3, mass3 = upload_batch(torch, w3)
    M3 = torch.empty(m3, dtype=torch.float64, device="cuda")
    L3 = torch.empty(l3, dtype=torch.float64, device="cuda")
    ctx.p2m(d3, pos3, mass3, 8, M3)
    del pos3, mass3
    torch.cuda.empty_cache()
    chosen = ctx.autotune(d3, M3, L3, fmm.FMM_FP64)

    def step_ud(ev, i):
        if ev: ev[0].record()
        ctx.m2l(d3, M3, L3)
        if ev: ev[1].record()

    _, seg_ud = timed(torch, step_ud, K, W, marks=1)
    ms_ud = seg_ud[:, 0].mean()
    L3d = L3.clone()
    chosen_h = ctx.autotune(d3, M3, L3, fmm.FMM_FP64_HARMONIC)

    def step_u(ev, i):
        if ev: ev[0].record()
        ctx.m2l(d3, M3, L3, fmm.FMM_FP64_HARMONIC)
        if ev: ev[1].record()

    wall_u, seg_u = timed(torch, step_u, K, W, marks=1)
    ms_u = seg_u[:, 0].mean()
    dev3 = rel_to_component_max(L3, L3d, d3, fmm)
    assert dev3["max"] <= 1e-12, dev3
    # per order: executed flops and the sub-grid count, for the tail estimate
    by_p = {}
    for p in (2, 3, 4):
        sel = w3.p == p
        by_p[str(p)] = {"subgrids": int(sel.sum()), "pairs": float(per[sel].sum()),
                        "harmonic_flops": float(per[sel].sum() * harmonic_flops_per_pair(p))}
    out = {"workload": "uneven_6000_mixed_p", "subgrids": w3.nsub, "pairs": pairs3,
           "form": "harmonic", "m2l_ms": float(ms_u), "pairs_per_s": pairs3 / (ms_u * 1e-3),
           "autotune_choice": chosen_h,
           "roofline": {"bound": "mfma", "achieved": fl3h / (ms_u * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": fl3h / (ms_u * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "flops_per_launch": fl3h,
                        "note": "executed-useful matrix flops: 2 (p+1)^4 per present pair"},
           "dense_equivalent_tflops": fl3 / (ms_u * 1e-3) / 1e12,
           "by_order": by_p,
           "dense_m2l_ms": float(ms_ud), "dense_tflops": fl3 / (ms_ud * 1e-3) / 1e12,
           "dense_frac": fl3 / (ms_ud * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
           "dense_autotune_choice": chosen, "harmonic_vs_dense": dev3,
           "parity": "tests/test_gpu_fullsize.py::test_uneven_6000"}
    log("uneven 6000: harmonic %.3f ms (%.4g pairs/s, %.1f%% executed), dense %.3f ms"
        % (ms_u, pairs3 / (ms_u * 1e-3), 100 * out["roofline"]["frac"], ms_ud))
    del M3, L3, L3d
    torch.cuda.empty_cache()
    return out


def slice_int8_ops(desc, slices):
    """Executed int8 matrix operations (2 per multiply-add) of the exact-slice M2L:
    per sub-grid 4 waves x 8 tiles x 223 offset quads x (kept slice pairs) instructions
    of 16 x 16 x 64 multiply-adds (no quad of a full-mask sub-grid is skipped)."""
    kept = sum(1 for i in range(slices) for j in range(slices) if i + j <= slices)
    return len(desc) * 4 * 8 * 223 * kept * 16 * 16 * 64 * 2


def bench_exact_slice(torch, fmm, ctx, desc, M, L_fp64, pairs, K, W, harmonic_ms):
    """The exact-slice M2L (int8 matrix cores, exact int32 sums) on the same moments
    as the step, at 6 and 7 slices; error against the float64 device result."""
    out = {}
    Lx = torch.empty_like(L_fp64)
    prev = ctx.get_option(fmm.FMM_OPT_SLICES)
    try:
        for S in (7, 6):
            ctx.set_option(fmm.FMM_OPT_SLICES, S)
            ctx.m2l(desc, M, Lx, fmm.FMM_EXACT_SLICE)          # slice buffers allocated, untimed

            def step_x(ev, i):
                if ev: ev[0].record()
                ctx.m2l(desc, M, Lx, fmm.FMM_EXACT_SLICE)
                if ev: ev[1].record()

            _, seg_x = timed(torch, step_x, K, W, marks=1)
            ms_x = seg_x[:, 0].mean()
            err = rel_to_component_max(Lx, L_fp64, desc, fmm)
            ops = slice_int8_ops(desc, S)
            out["slices_%d" % S] = {
                "m2l_ms": float(ms_x), "pairs_per_s": pairs / (ms_x * 1e-3),
                "speedup_vs_harmonic_fp64_m2l": float(harmonic_ms / ms_x),
                "int8_ops_per_launch": ops,
                "int8_tops_whole_call": ops / (ms_x * 1e-3) / 1e12,
                "frac_of_int8_peak_whole_call": ops / (ms_x * 1e-3) / 1e12 / INT8_PEAK_TOPS,
                "error_vs_fp64": dict(err, scale="largest |L| of the component in the sub-grid")}
            log("exact-slice M2L, %d slices: %.3f ms (x%.2f vs harmonic FP64), %.0f int8 TOPS over the call, "
                "max err %.3g of the component max" % (S, ms_x, harmonic_ms / ms_x, ops / (ms_x * 1e-3) / 1e12,
                                                         err["max"]))
    finally:
        ctx.set_option(fmm.FMM_OPT_SLICES, prev)
    out["what"] = ("fmm_m2l with FMM_EXACT_SLICE: slice_window_kernel (fold, exponent, int8 slices of the "
                   "20^3 window per sub-grid) + m2l_fwd_slice_kernel (v_mfma_i32_16x16x64_i8, exact int32 "
                   "sums, float64 across slice pairs)")
    out["error_vs_oracle"] = "tests/test_gpu_slice.py, tests/test_gpu_fullsize.py (sampled sub-grids, vs Labs)"
    del Lx
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle seconds per host core for cpu_baseline")
    ap.add_argument("--no-extras", action="store_true", help="only the step (for profiling)")
    ap.add_argument("--tree-only", action="store_true",
                    help="only the multi-level solve on 128^3 (for profiling)")
    ap.add_argument("--evaluate-only", action="store_true",
                    help="only the step and the evaluation at the particles (for profiling)")
    ap.add_argument("--uneven-only", action="store_true",
                    help="only the 6000-sub-grid uneven batch (for profiling)")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="only the 2048-sub-grid gradient batch (for profiling)")
    ap.add_argument("--slice-only", action="store_true",
                    help="only the step's moments and the exact-slice M2L (for profiling)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of this many GiB three times (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2 ** 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "repeats": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs its hot path on a single MI355X "
              "(sub-grids are independent, so a batch would shard by sub-grid across GPUs). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_11002_amd import fmm
    fmm.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = fmm.Context(0)
    # P2M writes only the frame rows holding the reachable 20^3 window, the cells M2L reads
    ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 1)
    K, W = args.steps, args.warmup
    if args.tree_only:
        print(json.dumps({"tree": bench_tree(torch, fmm, ctx, K, W)}), flush=True)
        ctx.close()
        return
    if args.uneven_only:
        print(json.dumps({"uneven": bench_uneven(torch, fmm, ctx, K, W)}), flush=True)
        ctx.close()
        return
    if args.fwd_bwd_only:
        print(json.dumps({"fwd_bwd": bench_fwd_bwd(torch, fmm, ctx, K, W)}), flush=True)
        ctx.close()
        return
    out = {"metric": METRIC, "unit": "pairs/s", "n_gpus": 1, "steps": K, "warmup": W,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic"}

    # ---------------- the step: P2M + FP64 M2L on 4096 uniform p=3 sub-grids, one launch
    w = synth.config(2)
    desc, m_el, l_el = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    pairs = fmm.pair_count(desc)
    pos, mass = upload_batch(torch, w)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.empty(l_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, pos, mass, 8, M)
    tuned = ctx.autotune(desc, M, L, fmm.FMM_FP64_HARMONIC)    # configuration for this batch
    if args.slice_only:
        def step_h(ev, i):
            if ev: ev[0].record()
            ctx.m2l(desc, M, L, fmm.FMM_FP64_HARMONIC)
            if ev: ev[1].record()

        _, seg_h = timed(torch, step_h, K, W, marks=1)
        print(json.dumps({"exact_slice": bench_exact_slice(torch, fmm, ctx, desc, M, L, pairs, K, W,
                                                           seg_h[:, 0].mean())}), flush=True)
        ctx.close()
        return
    ctx.p2m_m2l(desc, pos, mass, 8, M, L, fmm.FMM_FP64_HARMONIC)   # graph capture, untimed

    def step(ev, i):
        if ev: ev[0].record()
        ctx.p2m_m2l(desc, pos, mass, 8, M, L, fmm.FMM_FP64_HARMONIC)
        if ev: ev[1].record()

    wall, seg = timed(torch, step, K, W, marks=1)
    ms_step = wall / K * 1e3
    fused_ms = seg[:, 0].mean()
    out["value"] = pairs / (wall / K)
    out["ms_per_step"] = ms_step
    log("step %.3f ms (one launch, %.3f ms by events): %.4g pairs/s" % (ms_step, fused_ms, out["value"]))

    # the same step as two launches: P2M, then the M2L-only kernel (same bits)
    Lu = torch.empty_like(L)
    ctx.m2l(desc, M, Lu, fmm.FMM_FP64_HARMONIC)                # graph capture, untimed

    def step_two(ev, i):
        if ev: ev[0].record()
        ctx.p2m(desc, pos, mass, 8, M)
        if ev: ev[1].record()
        ctx.m2l(desc, M, Lu, fmm.FMM_FP64_HARMONIC)
        if ev: ev[2].record()

    wall_two, seg_two = timed(torch, step_two, K, W, marks=2)
    p2m_ms, m2l_ms = seg_two[:, 0].mean(), seg_two[:, 1].mean()
    assert bool(torch.equal(L, Lu)), "the one-launch step differs from P2M + M2L"
    del Lu
    import torch.version as tv
    out["config"] = {"workload": "uniform_4096_p3", "subgrids": w.nsub, "p": 3, "components": 20,
                     "h": 1.0, "particles_per_cell": 8, "stencil_offsets": 892,
                     "pairs_per_step": pairs,
                     "step": "P2M over the frame rows holding the reachable 20^3 window + M2L (float64, "
                             "harmonic form), one persistent launch (fmm_p2m_m2l)",
                     "step_kernel_ms": float(fused_ms),
                     "two_launch_step": {"p2m_ms": float(p2m_ms), "m2l_ms": float(m2l_ms),
                                         "step_ms": float(wall_two / K * 1e3),
                                         "m2l_ms_median": float(np.median(seg_two[:, 1])),
                                         "m2l_ms_min": float(seg_two[:, 1].min())},
                     "autotune_choice": tuned, "device": torch.cuda.get_device_name(0),
                     "hip": getattr(tv, "hip", None), "torch": torch.__version__}
    log("two launches: %.3f ms (P2M %.3f, M2L %.3f)" % (wall_two / K * 1e3, p2m_ms, m2l_ms))
    fl_exec = pairs * harmonic_flops_per_pair(3)      # executed matrix-core flops
    fl_dense = pairs * flops_per_pair(3)              # the dense 2 C^2 form
    achieved = fl_exec / (fused_ms * 1e-3) / 1e12
    traffic = read_traffic(pairs)
    out["roofline"] = {"bound": "mfma",
                       "kernel": "m2l_fwd_bl_kernel<PIPE, HARM, FUSE> (v_mfma_f64_4x4x4, harmonic form, "
                                 "configuration %d, with the P2M moment phase inside)" % tuned,
                       "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                       "flops_per_launch": fl_exec, "flops_per_pair": harmonic_flops_per_pair(3),
                       "fp64_dense_equivalent_tflops": fl_dense / (fused_ms * 1e-3) / 1e12,
                       "dense_flops_per_pair": flops_per_pair(3),
                       "m2l_only_kernel": {"ms": float(m2l_ms),
                                           "achieved": fl_exec / (m2l_ms * 1e-3) / 1e12,
                                           "frac": fl_exec / (m2l_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}}
    log("step kernel: %.2f executed TFLOP/s of M2L (%.1f%% of %.1f); M2L-only kernel %.2f (%.1f%%)"
        % (achieved, 100 * achieved / FP64_PEAK_TFLOPS, FP64_PEAK_TFLOPS,
           fl_exec / (m2l_ms * 1e-3) / 1e12, 100 * fl_exec / (m2l_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS))

    assert bool(torch.isfinite(L).all())
    out["parity"] = ("against the oracle in tests/test_gpu_fullsize.py (this workload, sampled sub-grids) "
                     "and tests/test_gpu_parity.py")

    if not args.evaluate_only:
        # ---------------- the dense form of the same M2L, on the same moments
        Ld = torch.empty_like(L)
        tuned_d = ctx.autotune(desc, M, Ld, fmm.FMM_FP64)

        def step_dense(ev, i):
            if ev: ev[0].record()
            ctx.m2l(desc, M, Ld, fmm.FMM_FP64)
            if ev: ev[1].record()

        _, seg_d = timed(torch, step_dense, K, W, marks=1)
        ms_d = seg_d[:, 0].mean()
        dev_d = rel_to_component_max(Ld, L, desc, fmm)
        assert dev_d["max"] <= 1e-12, dev_d
        out["dense_fp64"] = {"m2l_ms": float(ms_d), "pairs_per_s": pairs / (ms_d * 1e-3),
                             "tflops": fl_dense / (ms_d * 1e-3) / 1e12,
                             "frac_of_fp64_peak": fl_dense / (ms_d * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                             "autotune_choice": tuned_d, "vs_harmonic_form": dev_d,
                             "harmonic_speedup": float(ms_d / m2l_ms)}
        log("dense FP64 M2L %.3f ms (%.2f TFLOP/s), harmonic x%.2f" % (ms_d, fl_dense / (ms_d * 1e-3) / 1e12, ms_d / m2l_ms))
        del Ld

    if not args.no_extras and not args.evaluate_only:
        # ---------------- split precision on the same moments
        try:
            Ls = torch.empty_like(L)

            def step_split(ev, i):
                if ev: ev[0].record()
                ctx.m2l(desc, M, Ls, fmm.FMM_SPLIT_FP32)
                if ev: ev[1].record()

            wall_s, seg_s = timed(torch, step_split, K, W, marks=1)
            ms_s = seg_s[:, 0].mean()
            err = rel_to_component_max(Ls, L, desc, fmm)
            out["split_fp32"] = {"pairs_per_s": pairs / (ms_s * 1e-3), "m2l_ms": float(ms_s),
                                 "speedup_vs_dense_fp64_m2l": float(ms_d / ms_s),
                                 "speedup_vs_harmonic_fp64_m2l": float(m2l_ms / ms_s),
                                 "executed_fp32_tflops": 3 * fl_dense / (ms_s * 1e-3) / 1e12,
                                 "peak_fp32_tflops": FP32_PEAK_TFLOPS,
                                 "error_vs_fp64": dict(err, scale="largest |L| of the component in the sub-grid"),
                                 "error_vs_oracle": "tests/test_gpu_fullsize.py (sampled sub-grids, vs Labs)"}
            log("split-FP32 M2L %.3f ms (x%.2f vs dense FP64), max err %.3g of the component max" % (ms_s, ms_d / ms_s, err["max"]))
            del Ls
        except fmm.FMMError as e:
            out["split_fp32"] = {"error": str(e)}
        out["exact_slice"] = bench_exact_slice(torch, fmm, ctx, desc, M, L, pairs, K, W, m2l_ms)
    if not args.no_extras:
        # ---------------- evaluation at the particles (near field + L2P) from the step's L
        del M
        torch.cuda.empty_cache()
        n_part = w.nsub * 512 * 8
        npairs = near_pair_count(desc, 8)
        E = torch.empty(n_part * 4, dtype=torch.float64, device="cuda")

        def step_ev(ev, i):
            if ev: ev[0].record()
            ctx.evaluate(desc, pos, mass, 8, L, E)
            if ev: ev[1].record()

        _, seg_e = timed(torch, step_ev, K, W, marks=1)
        ms_e = seg_e[:, 0].mean()
        assert bool(torch.isfinite(E).all())
        fl_e = npairs * NEAR_FLOPS_PER_PAIR + n_part * l2p_flops(3)
        ach_e = fl_e / (ms_e * 1e-3) / 1e12
        out["evaluate"] = {
            "what": "potential and gradient at all 16.8M particles of the step: near field "
                    "(33 cells, |d|^2 <= 4, direct sums) + L2P of the step's L",
            "ms": float(ms_e), "particles_per_s": n_part / (ms_e * 1e-3),
            "near_pairs": npairs, "near_pairs_per_s": npairs / (ms_e * 1e-3),
            "same_level_solve_ms": float(ms_step + ms_e),
            "roofline": {"bound": "alu", "kernel": "evaluate_kernel (FP64 VALU)",
                         "achieved": ach_e, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": ach_e / FP64_PEAK_TFLOPS, "traffic": None,
                         "flops_per_near_pair": NEAR_FLOPS_PER_PAIR,
                         "l2p_flops_per_particle": l2p_flops(3)},
            "parity": "tests/test_gpu_evaluate.py, tests/test_gpu_fullsize.py::test_uniform_4096_evaluate"}
        log("evaluate %.3f ms: %.4g particles/s, %.4g near pairs/s, %.1f TFLOP/s executed"
            % (ms_e, n_part / (ms_e * 1e-3), npairs / (ms_e * 1e-3), ach_e))
        del pos, mass, L, E
        torch.cuda.empty_cache()

    if not args.no_extras and not args.evaluate_only:
        out["fwd_bwd"] = bench_fwd_bwd(torch, fmm, ctx, K, W)
        out["uneven"] = bench_uneven(torch, fmm, ctx, K, W)

        # ---------------- the multi-level iteration on a 128^3 domain
        out["tree"] = bench_tree(torch, fmm, ctx, K, W)
        torch.cuda.empty_cache()

        # ---------------- one sub-grid: the latency of the step (too small to fill the GPU)
        w1 = synth.config(1)
        d1, m1, l1 = fmm.make_descriptors(w1.p, w1.log2_inv_h, w1.mask)
        p1, ms1 = synth.subgrid_particles(w1.seed)
        pos1 = torch.from_numpy(p1).to("cuda")
        mass1 = torch.from_numpy(ms1).to("cuda")
        M1 = torch.empty(m1, dtype=torch.float64, device="cuda")
        L1 = torch.empty(l1, dtype=torch.float64, device="cuda")

        def step_one(ev, i):
            if ev: ev[0].record()
            ctx.p2m_m2l(d1, pos1, mass1, 8, M1, L1, fmm.FMM_FP64_HARMONIC)
            if ev: ev[1].record()

        _, seg1 = timed(torch, step_one, K, W, marks=1)
        # the same with the rounds of the sub-grid spread over workgroups
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, 1)
        try:
            _, seg1s = timed(torch, step_one, K, W, marks=1)
        finally:
            ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
        out["single_subgrid"] = {"workload": "single_subgrid_p3", "pairs": fmm.pair_count(d1),
                                 "step_ms_median": float(np.median(seg1[:, 0])),
                                 "step_ms_min": float(seg1[:, 0].min()),
                                 "round_split_step_ms_median": float(np.median(seg1s[:, 0])),
                                 "round_split_step_ms_min": float(seg1s[:, 0].min())}
        log("single sub-grid step %.3f ms (median), %.3f ms with the rounds split over workgroups"
            % (np.median(seg1[:, 0]), np.median(seg1s[:, 0])))
        del pos1, mass1, M1, L1

        # ---------------- a small uneven batch (128 sub-grids drawn like the uneven
        # workload): M2L with one workgroup per sub-grid and with the rounds split
        w128 = synth.config(3, nsub=128)
        d128, m128, l128 = fmm.make_descriptors(w128.p, w128.log2_inv_h, w128.mask)
        p128, ms128 = upload_batch(torch, w128)
        M128 = torch.empty(m128, dtype=torch.float64, device="cuda")
        L128 = torch.empty(l128, dtype=torch.float64, device="cuda")
        ctx.p2m(d128, p128, ms128, 8, M128)

        def step_small(ev, i):
            if ev: ev[0].record()
            ctx.m2l(d128, M128, L128, fmm.FMM_FP64_HARMONIC)
            if ev: ev[1].record()

        _, seg_sw = timed(torch, step_small, K, W, marks=1)
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, 1)
        try:
            _, seg_ss = timed(torch, step_small, K, W, marks=1)
        finally:
            ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
        # and as the autotuner leaves it (it times the round split too at this size)
        Lt128 = torch.empty_like(L128)
        tuned128 = ctx.autotune(d128, M128, Lt128, fmm.FMM_FP64_HARMONIC)
        del Lt128
        _, seg_st = timed(torch, step_small, K, W, marks=1)
        out["small_uneven_batch"] = {"workload": "uneven_128_mixed_p (p 1:2:1, random masks, three spacings)",
                                     "pairs": fmm.pair_count(d128),
                                     "form": "harmonic", "m2l_ms": float(np.median(seg_sw[:, 0])),
                                     "round_split_m2l_ms": float(np.median(seg_ss[:, 0])),
                                     "autotuned_m2l_ms": float(np.median(seg_st[:, 0])),
                                     "autotune_choice": tuned128}
        log("uneven 128: M2L %.3f ms, %.3f ms with the rounds split over workgroups, %.3f ms autotuned"
            % (np.median(seg_sw[:, 0]), np.median(seg_ss[:, 0]), np.median(seg_st[:, 0])))
        del p128, ms128, M128, L128

        # ---------------- CPU baseline (the oracle on the host cores)
        out["cpu_baseline"] = cpu_baseline(w.nsub, args.cpu_seconds)
        log("cpu_baseline %.4g pairs/s on %d cores" % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))

    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
