"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerance (float64 paths): per entry |x_gpu - x_oracle| <= 1e-12 * x_abs,
where x_abs is the same sum taken over absolute values (Labs for L, Gabs
for dM). Relative-to-|L| tolerances would fail correct code, because
orders >= 1 cancel heavily.
"""
import numpy as np
import pytest

import oracle as O
import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import (descriptors, ensure_library, moment_abs_scale, oracle_subgrid,
                          particles, split_views, to_dev)

pytestmark = pytest.mark.gpu
TOL = 1e-12
REF, MFMA = 1, 2


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    ensure_library()
    c = fmm.Context(0)
    yield c
    c.close()


def forward(ctx, torch, w, idx, kernel, prec=fmm.FMM_FP64, poison=False, graph=1):
    desc, m_el, l_el = descriptors(w, idx)
    pos, mass = particles(w, idx)
    dpos, dmass = to_dev(pos), to_dev(mass)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.p2m(desc, dpos, dmass, w.ppc, M)
    if poison:
        Mh = M.cpu().numpy()
        for d, v in zip(desc, split_views(Mh, desc, "M")):
            v[:, ~O.present_cells(int(d["mask"]))] = np.nan
        M = to_dev(Mh)
    ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, kernel)
    ctx.set_option(fmm.FMM_OPT_USE_GRAPH, graph)
    ctx.m2l(desc, M, L, prec)
    torch.cuda.synchronize()
    return desc, pos, mass, M, L


def assert_close(got, want, scale, tol=TOL, what=""):
    err = np.abs(got - want)
    bad = ~(err <= tol * scale)
    assert not bad.any(), "%s: %d entries off, worst ratio %.3g" % (
        what, bad.sum(), np.nanmax(err / np.maximum(scale, 1e-300)))


# ---------------------------------------------------------------------------

def _order_scale(T, p):
    ks = O.multi_indices(p)
    order = np.array([sum(k) for k in ks])
    tot = order[:, None] + order[None, :]
    scale = np.zeros_like(T)
    for m in range(2 * p + 1):
        sel = tot == m
        scale[:, sel] = np.abs(T[:, sel]).max(axis=1, keepdims=True)
    return scale


def test_stencil_tables_match_exact_and_oracle(ctx, torch):
    from oracle.exact import dtensor_exact
    eps = np.finfo(float).eps
    S = O.stencil()
    tables = {}
    for p in (2, 3, 4):
        C = fmm.ncomp(p)
        out = torch.empty(892 * C * C, dtype=torch.float64, device="cuda")
        ctx.stencil_tables(p, out)
        torch.cuda.synchronize()
        T = out.cpu().numpy().reshape(892, C, C)
        tables[p] = T
        To = O.stencil_tensors(p, 1.0)
        # the oracle's closed form (Hobson) rounds its alternating sums: ~150 ulp of the order scale
        assert_close(T, To, _order_scale(To, p), 512 * eps, "T p=%d vs closed form" % p)
        # transposition symmetry T_{-d} = T_d^T holds exactly on the device tables
        idx = {d: i for i, d in enumerate(S)}
        for i in range(0, 892, 37):
            a, b, c = S[i]
            assert np.array_equal(T[idx[(-a, -b, -c)]], T[i].T)
    # the lower orders' tables are the leading blocks of the p = 4 ones (graded order)
    for p in (2, 3):
        C = fmm.ncomp(p)
        assert np.array_equal(tables[p], tables[4][:, :C, :C])
    # p = 4 holds every derivative up to order 8: at every offset and entry within
    # 2 units in the last place of the exact value (exact zeros exactly zero)
    ks = O.multi_indices(4)
    T4 = tables[4]
    worst = 0.0
    for s, d in enumerate(S):
        R = tuple(-v for v in d)
        cache = {}
        for ik, k in enumerate(ks):
            for jn, n in enumerate(ks):
                m = (k[0] + n[0], k[1] + n[1], k[2] + n[2])
                if m not in cache:
                    cache[m] = dtensor_exact(m, R)
                e = (-1) ** sum(k) * cache[m]
                g = T4[s, ik, jn]
                if e == 0.0:
                    assert g == 0.0, (d, k, n, g)
                else:
                    ulps = abs(g - e) / np.spacing(abs(e))
                    assert ulps <= 2, (d, k, n, g, e, ulps)
                    worst = max(worst, ulps)
    print("device tables: worst %.1f ulp against the exact derivatives" % worst)


def test_p2m_single_subgrid(ctx, torch):
    w = synth.config(1)
    desc, pos, mass, M, L = forward(ctx, torch, w, [0], MFMA)
    Mo = O.p2m(pos[0], mass[0], 3, 1.0)
    scale = moment_abs_scale(pos[0], mass[0], 3, 1.0, synth.FULL_MASK)
    assert_close(M.cpu().numpy().reshape(Mo.shape), Mo, scale, 1e-14, "M")


@pytest.mark.parametrize("kernel", [REF, MFMA])
def test_m2l_single_subgrid(ctx, torch, kernel):
    w = synth.config(1)
    desc, pos, mass, M, L = forward(ctx, torch, w, [0], kernel)
    _, Lo, La = oracle_subgrid(w, 0, pos[0], mass[0])
    Lg = L.cpu().numpy().reshape(Lo.shape)
    assert_close(Lg, Lo, La, TOL, "L kernel %d" % kernel)
    print("one p = 3 sub-grid, kernel %d: max |dL|/Labs %.3g" % (kernel, float(np.max(np.abs(Lg - Lo) / La))))
    assert 2600 < Lg[0].min() and Lg[0].max() < 2800


@pytest.mark.parametrize("kernel", [REF, MFMA])
def test_m2l_uneven_batch_with_poisoned_absent_blocks(ctx, torch, kernel):
    # mixed p, h and random masks; absent blocks hold NaN and must never be read
    w = synth.config(3, nsub=9)
    idx = list(range(9))
    desc, pos, mass, M, L = forward(ctx, torch, w, idx, kernel, poison=True)
    Lg = split_views(L.cpu().numpy(), desc, "L")
    assert sorted(set(w.p.tolist())) == [2, 3, 4] and len(set(w.log2_inv_h.tolist())) > 1
    for b in idx:
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "sub-grid %d (p=%d, h=%g)" % (b, w.p[b], w.h(b)))


def test_edge_cases(ctx, torch):
    # empty batch, centre block only, and the largest order at the smallest spacing
    ctx.m2l(np.zeros(0, fmm.DESC_DTYPE), None, None)
    w = synth.Workload("edge", 17, np.array([4, 3, 2], np.int32), np.array([2, 0, 1], np.int32),
                       np.array([1 << 13, synth.FULL_MASK, (1 << 13) | (1 << 0) | (1 << 26)], np.uint32))
    for kernel in (REF, MFMA):
        desc, pos, mass, M, L = forward(ctx, torch, w, [0, 1, 2], kernel, poison=True)
        Lg = split_views(L.cpu().numpy(), desc, "L")
        for b in range(3):
            _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
            assert_close(Lg[b], Lo, La, TOL, "edge %d kernel %d" % (b, kernel))


def test_determinism_and_slot_independence(ctx, torch):
    w = synth.config(3, nsub=6)
    _, _, _, M, L1 = forward(ctx, torch, w, range(6), MFMA)
    desc, _, _ = descriptors(w, range(6))
    L2 = torch.full_like(L1, float("nan"))
    ctx.m2l(desc, M, L2)
    torch.cuda.synchronize()
    assert torch.equal(L1, L2)
    # the same sub-grid in another slot of a differently ordered batch
    order = [5, 2, 0, 4, 1, 3]
    desc_r, m_el, l_el = descriptors(w, order)
    Mv = split_views(M.cpu().numpy(), desc, "M")
    Mr = np.concatenate([Mv[b].ravel() for b in order])
    Lr = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.m2l(desc_r, to_dev(Mr), Lr)
    torch.cuda.synchronize()
    a = split_views(L1.cpu().numpy(), desc, "L")
    bb = split_views(Lr.cpu().numpy(), desc_r, "L")
    for i, b in enumerate(order):
        assert np.array_equal(a[b], bb[i])


def test_graph_replays_match_plain_launches(ctx, torch):
    w = synth.config(3, nsub=5)
    _, _, _, M, L_plain = forward(ctx, torch, w, range(5), MFMA, graph=0)
    desc, _, _ = descriptors(w, range(5))
    ctx.set_option(fmm.FMM_OPT_USE_GRAPH, 1)
    for rep in range(4):
        L = torch.full_like(L_plain, float("nan"))
        ctx.m2l(desc, M, L)
        x = torch.ones(1000, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(L, L_plain), rep
        assert x.item() == 1000


@pytest.mark.parametrize("kernel", [REF, MFMA])
def test_backward_matches_oracle_adjoint(ctx, torch, kernel):
    w = synth.config(3, nsub=6)
    idx = list(range(6))
    desc, m_el, l_el = descriptors(w, idx)
    pos, mass = particles(w, idx)
    rng = np.random.default_rng(77)
    W = rng.standard_normal(l_el)
    dM = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
    dmass = torch.full((len(idx) * fmm.NCELL * 8,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, kernel)
    ctx.m2l_backward(desc, to_dev(W), dM)
    ctx.p2m_backward(desc, to_dev(pos), 8, dM, dmass)
    torch.cuda.synchronize()
    Gg = split_views(dM.cpu().numpy(), desc, "M")
    Wv = split_views(W, desc, "L")
    gm = dmass.cpu().numpy().reshape(len(idx), fmm.NCELL, 8)
    for b in idx:
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        Go = O.m2l_adjoint(Wv[b], p, h, mask)
        Ga = O.m2l_adjoint_abs(Wv[b], p, h, mask)
        assert_close(Gg[b], Go, Ga, TOL, "dM sub-grid %d kernel %d" % (b, kernel))
        go = O.p2m_adjoint(pos[b], Go, p, h, mask)
        c = O.cell_centres(h)[:, None, :]
        gscale = O.p2m_adjoint(c + np.abs(pos[b] - c), Ga, p, h, mask)
        assert_close(gm[b], go, gscale, TOL, "dmass sub-grid %d" % b)


def test_adjoint_dot_product_on_device(ctx, torch):
    w = synth.config(3, nsub=4)
    desc, pos, mass, M, L = forward(ctx, torch, w, range(4), MFMA)
    rng = np.random.default_rng(3)
    W = rng.standard_normal(L.numel())
    dM = torch.empty_like(M)
    ctx.m2l_backward(desc, to_dev(W), dM)
    torch.cuda.synchronize()
    lhs = float(np.dot(W, L.cpu().numpy()))
    rhs = float(np.dot(dM.cpu().numpy(), M.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + abs(rhs))


def test_split_fp32_error_bounds(ctx, torch):
    # split precision is not bitwise reproducible against any CPU model (matrix-core
    # float32 summation order is the hardware's); its error is bounded instead:
    # float32 block sums cap it near 2^-24 of Labs
    w = synth.config(3, nsub=6)
    desc, pos, mass, M, L = forward(ctx, torch, w, range(6), MFMA, prec=fmm.FMM_SPLIT_FP32,
                                    poison=True)
    Lg = split_views(L.cpu().numpy(), desc, "L")
    rel = []
    for b in range(6):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        r = np.abs(Lg[b] - Lo) / La
        assert np.all(np.isfinite(Lg[b]))
        rel.append(r.ravel())
    rel = np.concatenate(rel)
    assert rel.max() < 1e-6, rel.max()
    assert np.median(rel) < 5e-8, np.median(rel)


def test_split_fp32_matches_expectation_model_scale(ctx, torch):
    w = synth.config(1)
    desc, pos, mass, M, L = forward(ctx, torch, w, [0], MFMA, prec=fmm.FMM_SPLIT_FP32)
    Mo, Lo, La = oracle_subgrid(w, 0, pos[0], mass[0])
    Lg = L.cpu().numpy().reshape(Lo.shape)
    Le = O.m2l_split32_emulated(Mo, 3, 1.0)
    gpu = np.abs(Lg - Lo) / La
    emu = np.abs(Le - Lo) / La
    assert gpu.max() < 10 * emu.max() and np.median(gpu) < 10 * np.median(emu)
    # and it is far from float64 agreement: the split really ran in float32
    assert gpu.max() > 1e-11


def test_p2m_generic_particle_count_and_adjoint(ctx, torch):
    # 3 particles per cell takes the general P2M kernels (8 takes the LDS-staged ones)
    w = synth.Workload("ppc3", 23, np.array([4, 2], np.int32), np.array([1, 0], np.int32),
                       np.array([synth.FULL_MASK, (1 << 13) | (1 << 4) | (1 << 22)], np.uint32), ppc=3)
    desc, pos, mass, M, L = forward(ctx, torch, w, [0, 1], MFMA)
    Mg = split_views(M.cpu().numpy(), desc, "M")
    rng = np.random.default_rng(5)
    G = rng.standard_normal(M.numel())
    dmass = torch.full((2 * fmm.NCELL * 3,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.p2m_backward(desc, to_dev(pos), 3, to_dev(G), dmass)
    torch.cuda.synchronize()
    gm = dmass.cpu().numpy().reshape(2, fmm.NCELL, 3)
    Gv = split_views(G, desc, "M")
    for b in range(2):
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        Mo = O.p2m(pos[b], mass[b], p, h, mask)
        assert_close(Mg[b], Mo, moment_abs_scale(pos[b], mass[b], p, h, mask), 1e-14, "M ppc3")
        go = O.p2m_adjoint(pos[b], Gv[b], p, h, mask)
        c = O.cell_centres(h)[:, None, :]
        scale = O.p2m_adjoint(c + np.abs(pos[b] - c), np.abs(Gv[b]), p, h, mask)
        assert_close(gm[b], go, scale, 1e-14, "dmass ppc3")


def test_every_tile_configuration_agrees_bitwise(ctx, torch):
    # all FP64 configurations do the same products in the same order: identical L
    w = synth.config(3, nsub=5)
    desc, pos, mass, M, L0 = forward(ctx, torch, w, range(5), MFMA)
    Lg = split_views(L0.cpu().numpy(), desc, "L")
    for b in range(5):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "sub-grid %d" % b)
    cfg = 0
    while True:
        try:
            ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, cfg)
        except fmm.FMMError:
            break
        L = torch.full_like(L0, float("nan"))
        try:
            ctx.m2l(desc, M, L, fmm.FMM_FP64)
        except fmm.FMMError as e:
            assert e.status == fmm.FMM_EINVAL   # a split-precision configuration
            cfg += 1
            continue
        torch.cuda.synchronize()
        assert torch.equal(L, L0), cfg
        cfg += 1
    ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, -1)
    assert cfg >= 4
    # the harmonic form's configurations (pipelined or not, chunk lengths) likewise
    Lh0 = torch.full_like(L0, float("nan"))
    ctx.m2l(desc, M, Lh0, fmm.FMM_FP64_HARMONIC)
    tried = 0
    for c in range(cfg):
        ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, c)
        L = torch.full_like(L0, float("nan"))
        try:
            ctx.m2l(desc, M, L, fmm.FMM_FP64_HARMONIC)
        except fmm.FMMError as e:
            assert e.status == fmm.FMM_EINVAL
            continue
        torch.cuda.synchronize()
        assert torch.equal(L, Lh0), c
        tried += 1
    ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, -1)
    assert tried >= 3


def test_backward_is_deterministic(ctx, torch):
    # the adjoint sums into LDS in a fixed order: bitwise identical run to run
    w = synth.config(3, nsub=6)
    desc, m_el, l_el = descriptors(w, range(6))
    W = to_dev(np.random.default_rng(9).standard_normal(l_el))
    ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, MFMA)
    outs = []
    for _ in range(3):
        dM = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.m2l_backward(desc, W, dM)
        torch.cuda.synchronize()
        outs.append(dM)
    assert torch.isfinite(outs[0]).all()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


# ---------------------------------------------------------------------------
# harmonic (traceless) form, against the dense oracle
# ---------------------------------------------------------------------------

HARM = fmm.FMM_FP64_HARMONIC


def test_harmonic_form_matches_oracle(ctx, torch):
    # one full sub-grid; mixed p, h and masks with absent blocks poisoned; the edge set
    w = synth.config(1)
    desc, pos, mass, M, L = forward(ctx, torch, w, [0], MFMA, prec=HARM)
    _, Lo, La = oracle_subgrid(w, 0, pos[0], mass[0])
    assert_close(L.cpu().numpy().reshape(Lo.shape), Lo, La, TOL, "harmonic single")
    w = synth.config(3, nsub=9)
    desc, pos, mass, M, L = forward(ctx, torch, w, range(9), MFMA, prec=HARM, poison=True)
    Lg = split_views(L.cpu().numpy(), desc, "L")
    for b in range(9):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "harmonic sub-grid %d (p=%d, h=%g)" % (b, w.p[b], w.h(b)))
    w = synth.Workload("edge", 17, np.array([4, 3, 2], np.int32), np.array([2, 0, 1], np.int32),
                       np.array([1 << 13, synth.FULL_MASK, (1 << 13) | (1 << 0) | (1 << 26)], np.uint32))
    desc, pos, mass, M, L = forward(ctx, torch, w, [0, 1, 2], MFMA, prec=HARM, poison=True)
    Lg = split_views(L.cpu().numpy(), desc, "L")
    for b in range(3):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "harmonic edge %d" % b)


def test_harmonic_form_full_blocks_every_order(ctx, torch):
    # every neighbour present (the branch-free loops), p = 2, 3, 4 at each spacing
    w = synth.Workload("full", 23, np.array([2, 3, 4, 4], np.int32), np.array([1, 0, 0, 2], np.int32),
                       np.full(4, synth.FULL_MASK, np.uint32))
    desc, pos, mass, M, L = forward(ctx, torch, w, range(4), MFMA, prec=HARM)
    Lg = split_views(L.cpu().numpy(), desc, "L")
    for b in range(4):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "harmonic full sub-grid %d (p=%d, h=%g)" % (b, w.p[b], w.h(b)))


def test_harmonic_form_deterministic_graphs_and_autotune(ctx, torch):
    w = synth.config(3, nsub=5)
    _, _, _, M, L_plain = forward(ctx, torch, w, range(5), MFMA, prec=HARM, graph=0)
    desc, _, _ = descriptors(w, range(5))
    ctx.set_option(fmm.FMM_OPT_USE_GRAPH, 1)
    for rep in range(3):
        L = torch.full_like(L_plain, float("nan"))
        ctx.m2l(desc, M, L, HARM)
        x = torch.ones(1000, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(L, L_plain), rep
        assert x.item() == 1000
    # the autotuner, on a context of its own (its choice is kept per descriptor
    # set): with FMM_OPT_ROUND_SPLIT = 0 the tuned call gives the same bits; at its
    # default (-1) five sub-grids, far too few to fill the GPU, take the round
    # split, which it times too: the bits of FMM_OPT_ROUND_SPLIT = 1
    c2 = fmm.Context(0)
    try:
        Lt = torch.empty_like(L_plain)
        chosen = c2.autotune(desc, M, Lt, HARM)
        L = torch.full_like(L_plain, float("nan"))
        c2.m2l(desc, M, L, HARM)
        outs = {}
        for opt in (0, 1):
            c2.set_option(fmm.FMM_OPT_ROUND_SPLIT, opt)
            outs[opt] = torch.full_like(L_plain, float("nan"))
            c2.m2l(desc, M, outs[opt], HARM)
        c2.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
        torch.cuda.synchronize()
    finally:
        c2.close()
    assert chosen >= 0 and torch.equal(outs[0], L_plain)
    assert torch.equal(L, outs[1])
    scale = torch.abs(L_plain).max()
    assert (torch.abs(L - L_plain) <= 1e-13 * scale).all()


def test_harmonic_adjoint_matches_oracle_and_is_deterministic(ctx, torch):
    # the harmonic adjoint against the dense oracle adjoint; mixed p, h and masks
    w = synth.config(3, nsub=9)
    idx = list(range(9))
    desc, m_el, l_el = descriptors(w, idx)
    W = np.random.default_rng(78).standard_normal(l_el)
    dW = to_dev(W)
    ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, MFMA)
    ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 1)
    try:
        dM = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.m2l_backward(desc, dW, dM)
        dM2 = torch.full_like(dM, float("nan"))
        ctx.m2l_backward(desc, dW, dM2)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 0)
    assert torch.equal(dM, dM2)
    Gg = split_views(dM.cpu().numpy(), desc, "M")
    Wv = split_views(W, desc, "L")
    assert sorted(set(w.p.tolist())) == [2, 3, 4]
    for b in idx:
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        Go = O.m2l_adjoint(Wv[b], p, h, mask)
        Ga = O.m2l_adjoint_abs(Wv[b], p, h, mask)
        assert_close(Gg[b], Go, Ga, TOL, "harmonic dM sub-grid %d (p=%d)" % (b, p))


def test_harmonic_adjoint_dot_product(ctx, torch):
    # <W, L(M)> = <dM(W), M> between the harmonic forward and the harmonic adjoint
    w = synth.config(3, nsub=4)
    desc, pos, mass, M, L = forward(ctx, torch, w, range(4), MFMA, prec=HARM)
    W = np.random.default_rng(4).standard_normal(L.numel())
    dM = torch.empty_like(M)
    ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 1)
    try:
        ctx.m2l_backward(desc, to_dev(W), dM)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 0)
    lhs = float(np.dot(W, L.cpu().numpy()))
    rhs = float(np.dot(dM.cpu().numpy(), M.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + abs(rhs))


def test_p2m_window_option(ctx, torch):
    # FMM_OPT_P2M_WINDOW = 1: the moments of the frame rows holding the reachable
    # window bitwise as in the full P2M, every other cell of M untouched, and the
    # same M2L; also the generic kernel
    for ppc in (8, 5):
        w = synth.config(3, nsub=4)
        w.ppc = ppc
        desc, m_el, l_el = descriptors(w, range(4))
        pos, mass = particles(w, range(4))
        dpos, dmass = to_dev(pos), to_dev(mass)
        Mf = torch.empty(m_el, dtype=torch.float64, device="cuda")
        Mw = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.p2m(desc, dpos, dmass, ppc, Mf)
        ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 1)
        try:
            ctx.p2m(desc, dpos, dmass, ppc, Mw)
        finally:
            ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 0)
        torch.cuda.synchronize()
        rows = np.zeros((24, 24, 24), bool)          # [z][y][x]: rows (y, z) in [2, 22)^2, every x
        rows[2:22, 2:22, :] = True
        for vf, vw in zip(split_views(Mf.cpu().numpy(), desc, "M"), split_views(Mw.cpu().numpy(), desc, "M")):
            assert np.array_equal(vf[:, rows], vw[:, rows])
            assert np.isnan(vw[:, ~rows]).all()
        if ppc == 8:
            ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, MFMA)
            L1 = torch.empty(l_el, dtype=torch.float64, device="cuda")
            L2 = torch.empty_like(L1)
            ctx.m2l(desc, Mf, L1, fmm.FMM_FP64_HARMONIC)
            ctx.m2l(desc, Mw, L2, fmm.FMM_FP64_HARMONIC)
            torch.cuda.synchronize()
            assert torch.equal(L1, L2)



@pytest.mark.parametrize("prec,cfg", [(HARM, 7), (fmm.FMM_FP64, 0), (fmm.FMM_FP64, 1)])
def test_round_split_option(ctx, torch, prec, cfg):
    # FMM_OPT_ROUND_SPLIT: one workgroup per (sub-grid, round), rounds added in
    # order by a second kernel; mixed orders, spacings and masks, one full
    # sub-grid; against the oracle and, up to rounding, the whole-sub-grid path.
    # Above 256 sub-grids the option does not apply (bitwise the usual path).
    w = synth.config(3, nsub=9)
    desc, m_el, l_el = descriptors(w, range(9))
    pos, mass = particles(w, range(9))
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, to_dev(pos), to_dev(mass), 8, M)
    L0 = torch.empty(l_el, dtype=torch.float64, device="cuda")
    L1 = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, cfg)
    try:
        ctx.m2l(desc, M, L0, prec)
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, 1)
        ctx.m2l(desc, M, L1, prec)
        L2 = torch.full_like(L1, float("nan"))
        ctx.m2l(desc, M, L2, prec)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
        ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, -1)
    assert torch.equal(L1, L2)                       # deterministic
    Lg, L0v = split_views(L1.cpu().numpy(), desc, "L"), split_views(L0.cpu().numpy(), desc, "L")
    for b in range(9):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "round split sub-grid %d (p=%d)" % (b, w.p[b]))
        assert_close(Lg[b], L0v[b], La, 1e-13, "round split vs whole sub-grid %d" % b)
    w1 = synth.config(1)
    desc1, m1, l1 = descriptors(w1, [0])
    p1, ms1 = particles(w1, [0])
    M1 = torch.empty(m1, dtype=torch.float64, device="cuda")
    ctx.p2m(desc1, to_dev(p1), to_dev(ms1), 8, M1)
    L1s = torch.empty(l1, dtype=torch.float64, device="cuda")
    ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, 1)
    try:
        ctx.m2l(desc1, M1, L1s, prec)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
    _, Lo, La = oracle_subgrid(w1, 0, p1[0], ms1[0])
    assert_close(L1s.cpu().numpy().reshape(Lo.shape), Lo, La, TOL, "round split single sub-grid")
    w = synth.config(3, nsub=257)
    desc, m_el, l_el = descriptors(w, range(257))
    pos, mass = particles(w, range(257))
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, to_dev(pos), to_dev(mass), 8, M)
    La_, Lb_ = torch.empty(l_el, dtype=torch.float64, device="cuda"), torch.empty(l_el, dtype=torch.float64, device="cuda")
    ctx.m2l(desc, M, La_, prec)
    ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, 1)
    try:
        ctx.m2l(desc, M, Lb_, prec)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
    assert torch.equal(La_, Lb_)


def test_round_split_mid_size_uneven_batch(ctx, torch):
    # 200 uneven sub-grids (thousands of round slots): the split path against the
    # whole-sub-grid path everywhere (1e-12 of each component's largest |L| in
    # the sub-grid) and against the oracle on sampled sub-grids of every order
    n = 200
    w = synth.config(3, nsub=n)
    desc, m_el, l_el = descriptors(w, range(n))
    pos, mass = particles(w, range(n))
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, to_dev(pos), to_dev(mass), 8, M)
    L0 = torch.empty(l_el, dtype=torch.float64, device="cuda")
    L1 = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.m2l(desc, M, L0, HARM)
    ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, 1)
    try:
        ctx.m2l(desc, M, L1, HARM)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ROUND_SPLIT, -1)
    Lg, L0v = split_views(L1.cpu().numpy(), desc, "L"), split_views(L0.cpu().numpy(), desc, "L")
    for b in range(n):
        scale = np.abs(L0v[b]).reshape(L0v[b].shape[0], -1).max(axis=1)[:, None, None, None]
        assert (np.abs(Lg[b] - L0v[b]) <= 1e-12 * scale).all(), "sub-grid %d" % b
    for p in (2, 3, 4):
        b = int(np.flatnonzero(w.p == p)[-1])
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        assert_close(Lg[b], Lo, La, TOL, "round split mid-size sub-grid %d (p=%d)" % (b, p))
