"""GPU parity of the fused P2M + M2L entry point (fmm_p2m_m2l) through the C ABI.

The single launch must give, bit for bit, what fmm_p2m over the rows holding
the reachable window followed by fmm_m2l gives: the same L, the same moments
in those rows, and no write to any other cell of M. It is checked in every
form it runs in (harmonic, and the two float64 configurations with staged
tables) on batches with more sub-grids than the GPU has compute units, where
workgroups compute the next sub-grid's moments in the middle of the current
one's M2L, and on uneven batches, where the next sub-grid's order, spacing and
mask differ from the current one's. Sampled sub-grids are checked against the
oracle as well, at the tolerance of the other parity tests, and the cases that
run as two launches (ppc != 8, split precision, the reference kernel) against
the two separate calls.
"""
import numpy as np
import pytest

import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import (descriptors, ensure_library, moment_abs_scale, oracle_subgrid,
                          particles, split_views, to_dev)

pytestmark = pytest.mark.gpu
TOL = 1e-12
ROWS = np.zeros((24, 24, 24), bool)          # [z][y][x]: rows (y, z) in [2, 22)^2, every x
ROWS[2:22, 2:22, :] = True
HARM_CFG, FP64_CFGS = 7, (0, 1)               # staged-table configurations


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


def separate(ctx, torch, desc, dpos, dmass, ppc, m_el, l_el, prec):
    M = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
    L = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 1)
    try:
        ctx.p2m(desc, dpos, dmass, ppc, M)
    finally:
        ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 0)
    ctx.m2l(desc, M, L, prec)
    return M, L


def fused(ctx, torch, desc, dpos, dmass, ppc, m_el, l_el, prec):
    M = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
    L = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.p2m_m2l(desc, dpos, dmass, ppc, M, L, prec)
    return M, L


def assert_same(desc, Ms, Ls, Mf, Lf, what):
    assert torch_equal(Ls, Lf), "%s: L differs" % what
    for b, (vs, vf) in enumerate(zip(split_views(Ms.cpu().numpy(), desc, "M"),
                                     split_views(Mf.cpu().numpy(), desc, "M"))):
        assert np.array_equal(vs[:, ROWS], vf[:, ROWS]), "%s: M rows of sub-grid %d differ" % (what, b)
        assert np.isnan(vf[:, ~ROWS]).all(), "%s: M written outside the rows, sub-grid %d" % (what, b)


def torch_equal(a, b):
    import torch as t
    return bool(t.equal(a, b))


def run_forms(ctx, torch, w, idx, forms):
    desc, m_el, l_el = descriptors(w, idx)
    pos, mass = particles(w, idx)
    dpos, dmass = to_dev(pos), to_dev(mass)
    out = {}
    for prec, cfg in forms:
        ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, cfg)
        try:
            Ms, Ls = separate(ctx, torch, desc, dpos, dmass, w.ppc, m_el, l_el, prec)
            Mf, Lf = fused(ctx, torch, desc, dpos, dmass, w.ppc, m_el, l_el, prec)
            torch.cuda.synchronize()
        finally:
            ctx.set_option(fmm.FMM_OPT_TILE_CONFIG, -1)
        assert_same(desc, Ms, Ls, Mf, Lf, "prec %d cfg %d" % (prec, cfg))
        out[(prec, cfg)] = (Mf, Lf)
    return desc, pos, mass, out


def test_fused_uneven_batch_matches_the_separate_calls(ctx, torch):
    # 600 sub-grids, p in {2,3,4}, h in {1,1/2,1/4}, random masks: more items than
    # compute units, and consecutive items of different orders
    w = synth.config(3, nsub=600)
    assert len(set(w.p.tolist())) == 3
    forms = [(fmm.FMM_FP64_HARMONIC, HARM_CFG)] + [(fmm.FMM_FP64, c) for c in FP64_CFGS]
    desc, pos, mass, out = run_forms(ctx, torch, w, range(600), forms)
    # and against the oracle on sampled sub-grids of every order
    Lh = out[(fmm.FMM_FP64_HARMONIC, HARM_CFG)][1].cpu().numpy()
    Mh = out[(fmm.FMM_FP64_HARMONIC, HARM_CFG)][0].cpu().numpy()
    picks = [int(np.flatnonzero(w.p == p)[k]) for p in (2, 3, 4) for k in (0, -1)]
    Lv, Mv = split_views(Lh, desc, "L"), split_views(Mh, desc, "M")
    for b in picks:
        Mo, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        err = np.abs(Lv[b] - Lo)
        assert (err <= TOL * La).all(), "L of sub-grid %d (p=%d): worst %.3g" % (
            b, w.p[b], np.max(err / np.maximum(La, 1e-300)))
        Ma = moment_abs_scale(pos[b], mass[b], int(w.p[b]), w.h(b), int(w.mask[b]))
        assert (np.abs(Mv[b][:, ROWS] - Mo[:, ROWS]) <= 1e-13 * Ma[:, ROWS]).all()


def test_fused_uniform_batch_against_the_oracle(ctx, torch):
    # 300 uniform p = 3 sub-grids of the 4096 workload (more than the compute units)
    w = synth.config(2, nsub=300)
    forms = [(fmm.FMM_FP64_HARMONIC, HARM_CFG), (fmm.FMM_FP64, 0)]
    desc, pos, mass, out = run_forms(ctx, torch, w, range(300), forms)
    for (prec, cfg), (_, Lf) in out.items():
        Lv = split_views(Lf.cpu().numpy(), desc, "L")
        for b in (0, 171, 299):
            _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
            err = np.abs(Lv[b] - Lo)
            assert (err <= TOL * La).all(), "prec %d cfg %d sub-grid %d: worst %.3g" % (
                prec, cfg, b, np.max(err / np.maximum(La, 1e-300)))


@pytest.mark.parametrize("p", [2, 4])
def test_fused_full_blocks_other_orders(ctx, torch, p):
    # 300 sub-grids of one order with every neighbour present (the branch-free
    # loops, and at p = 4 the harmonic form's pipelined one)
    n = 300
    w = synth.Workload("full_p%d" % p, 40 + p, np.full(n, p, np.int32), np.zeros(n, np.int32),
                       np.full(n, synth.FULL_MASK, np.uint32))
    forms = [(fmm.FMM_FP64_HARMONIC, HARM_CFG), (fmm.FMM_FP64, 0)]
    desc, pos, mass, out = run_forms(ctx, torch, w, range(n), forms)
    Lv = split_views(out[(fmm.FMM_FP64_HARMONIC, HARM_CFG)][1].cpu().numpy(), desc, "L")
    for b in (0, n - 1):
        _, Lo, La = oracle_subgrid(w, b, pos[b], mass[b])
        err = np.abs(Lv[b] - Lo)
        assert (err <= TOL * La).all(), "p=%d sub-grid %d: worst %.3g" % (p, b, np.max(err / np.maximum(La, 1e-300)))


def test_fused_graph_replays(ctx, torch):
    # replays of the cached graph of the single launch: plain launches give the
    # same bits, and doubled masses give exactly doubled moments and L (a power of
    # two scales exactly)
    w = synth.config(3, nsub=300)
    desc, m_el, l_el = descriptors(w, range(300))
    pos, mass = particles(w, range(300))
    dpos, dmass = to_dev(pos), to_dev(mass)
    prec = fmm.FMM_FP64_HARMONIC
    Ms, Ls = separate(ctx, torch, desc, dpos, dmass, 8, m_el, l_el, prec)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.empty(l_el, dtype=torch.float64, device="cuda")
    results = []
    for rep in range(3):
        M.fill_(float("nan"))
        L.fill_(float("nan"))
        ctx.p2m_m2l(desc, dpos, dmass, 8, M, L, prec)
        torch.cuda.synchronize()
        results.append((M.clone(), L.clone()))
    for Mf, Lf in results:
        assert_same(desc, Ms, Ls, Mf, Lf, "graph replay")
    ctx.set_option(fmm.FMM_OPT_USE_GRAPH, 0)
    try:
        Mn, Ln = fused(ctx, torch, desc, dpos, dmass, 8, m_el, l_el, prec)
    finally:
        ctx.set_option(fmm.FMM_OPT_USE_GRAPH, 1)
    torch.cuda.synchronize()
    assert_same(desc, Ms, Ls, Mn, Ln, "plain launch")
    dmass.mul_(2.0)
    M.fill_(float("nan"))
    ctx.p2m_m2l(desc, dpos, dmass, 8, M, L, prec)
    torch.cuda.synchronize()
    assert torch.equal(L, 2.0 * Ls)
    assert torch.equal(torch.nan_to_num(M, 0.0), torch.nan_to_num(2.0 * results[0][0], 0.0))


@pytest.mark.parametrize("case", ["small", "ppc5", "split", "reference"])
def test_fused_entry_point_two_launch_cases(ctx, torch, case):
    # the cases without the single launch give what the two calls give: a batch
    # no larger than the compute-unit count, ppc != 8, split precision, the
    # reference kernel (the others on 300 sub-grids)
    n = 6 if case == "small" else 300
    w = synth.config(3, nsub=n)
    if case == "ppc5":
        w.ppc = 5
    desc, m_el, l_el = descriptors(w, range(n))
    pos, mass = particles(w, range(n))
    dpos, dmass = to_dev(pos), to_dev(mass)
    prec = {"small": fmm.FMM_FP64_HARMONIC, "ppc5": fmm.FMM_FP64_HARMONIC, "split": fmm.FMM_SPLIT_FP32,
            "reference": fmm.FMM_FP64}[case]
    if case == "reference":
        ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, 1)
    try:
        Ms, Ls = separate(ctx, torch, desc, dpos, dmass, w.ppc, m_el, l_el, prec)
        Mf, Lf = fused(ctx, torch, desc, dpos, dmass, w.ppc, m_el, l_el, prec)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, 0)
    assert_same(desc, Ms, Ls, Mf, Lf, case)


# ---------------------------------------------------------------------------
# the adjoints in one launch (fmm_m2l_p2m_backward)
# ---------------------------------------------------------------------------

def backward_both(ctx, torch, desc, dpos, ppc, dL, m_el, n_part):
    dM1 = torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda")
    dm1 = torch.full((n_part,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.m2l_backward(desc, dL, dM1)
    ctx.p2m_backward(desc, dpos, ppc, dM1, dm1)
    dM2 = torch.full_like(dM1, float("nan"))
    dm2 = torch.full_like(dm1, float("nan"))
    ctx.m2l_p2m_backward(desc, dpos, ppc, dL, dM2, dm2)
    torch.cuda.synchronize()
    return dM1, dm1, dM2, dm2


@pytest.mark.parametrize("form", [0, 1])
def test_fused_backward_matches_the_separate_calls(ctx, torch, form):
    # 600 uneven sub-grids (every order, spacing and random masks), dense and
    # harmonic adjoint: dM and the mass gradients bit for bit as the two calls,
    # and sampled sub-grids of every order against the oracle
    w = synth.config(3, nsub=600)
    n = 600
    desc, m_el, l_el = descriptors(w, range(n))
    pos, mass = particles(w, range(n))
    dpos = to_dev(pos)
    W = np.random.default_rng(91).standard_normal(l_el)
    ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, form)
    try:
        dM1, dm1, dM2, dm2 = backward_both(ctx, torch, desc, dpos, 8, to_dev(W), m_el, n * fmm.NCELL * 8)
        # replayed graph-free launches of the same call give the same bits
        dM3, dm3 = torch.empty_like(dM2), torch.empty_like(dm2)
        ctx.m2l_p2m_backward(desc, dpos, 8, to_dev(W), dM3, dm3)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 0)
    assert torch.equal(dM1, dM2) and torch.equal(dm1, dm2)
    assert torch.equal(dM2, dM3) and torch.equal(dm2, dm3)
    import oracle as O
    Gv, Wv = split_views(dM2.cpu().numpy(), desc, "M"), split_views(W, desc, "L")
    gm = dm2.cpu().numpy().reshape(n, fmm.NCELL, 8)
    picks = [int(np.flatnonzero(w.p == p)[k]) for p in (2, 3, 4) for k in (0, -1)]
    for b in picks:
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        Go, Ga = O.m2l_adjoint(Wv[b], p, h, mask), O.m2l_adjoint_abs(Wv[b], p, h, mask)
        assert (np.abs(Gv[b] - Go) <= TOL * Ga).all(), "dM of sub-grid %d (p=%d)" % (b, p)
        go = O.p2m_adjoint(pos[b], Go, p, h, mask)
        c = O.cell_centres(h)[:, None, :]
        gscale = O.p2m_adjoint(c + np.abs(pos[b] - c), Ga, p, h, mask)
        assert (np.abs(gm[b] - go) <= TOL * gscale).all(), "dmass of sub-grid %d (p=%d)" % (b, p)


@pytest.mark.parametrize("case", ["small", "ppc5", "reference"])
def test_fused_backward_two_launch_cases(ctx, torch, case):
    n = 6 if case == "small" else 300
    w = synth.config(3, nsub=n)
    if case == "ppc5":
        w.ppc = 5
    desc, m_el, l_el = descriptors(w, range(n))
    pos, mass = particles(w, range(n))
    W = to_dev(np.random.default_rng(5).standard_normal(l_el))
    if case == "reference":
        ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, 1)
    try:
        dM1, dm1, dM2, dm2 = backward_both(ctx, torch, desc, to_dev(pos), w.ppc, W, m_el, n * fmm.NCELL * w.ppc)
    finally:
        ctx.set_option(fmm.FMM_OPT_M2L_KERNEL, 0)
    assert torch.equal(dM1, dM2) and torch.equal(dm1, dm2)


# seeded compositions: batch size just above and well above the compute-unit
# count, order mix, spacings and masks drawn per sub-grid (full blocks included)
def _random_batch(seed, n):
    rng = np.random.default_rng([seed, 1234])
    p = rng.choice(np.array([2, 3, 4], np.int32), size=n, p=[0.3, 0.4, 0.3]).astype(np.int32)
    lh = rng.integers(0, 3, n).astype(np.int32)
    masks = np.array([synth.FULL_MASK if rng.random() < 0.3 else synth.random_mask(rng) for _ in range(n)],
                     np.uint32)
    return synth.Workload("sweep_%d" % seed, 60 + seed, p, lh, masks)


@pytest.mark.parametrize("seed,n", [(1, 257), (2, 333), (3, 520)])
def test_one_launch_sweep(ctx, torch, seed, n):
    w = _random_batch(seed, n)
    forms = [(fmm.FMM_FP64_HARMONIC, HARM_CFG), (fmm.FMM_FP64, 0)]
    desc, pos, mass, out = run_forms(ctx, torch, w, range(n), forms)
    W = to_dev(np.random.default_rng(seed).standard_normal(int(desc["l_off"][-1]) + 512 * fmm.ncomp(int(w.p[-1]))))
    m_el = int(desc["m_off"][-1]) + fmm.NCELL * fmm.ncomp(int(w.p[-1]))
    ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 1)
    try:
        dM1, dm1, dM2, dm2 = backward_both(ctx, torch, desc, to_dev(pos), 8, W, m_el, n * fmm.NCELL * 8)
    finally:
        ctx.set_option(fmm.FMM_OPT_ADJOINT_FORM, 0)
    assert torch.equal(dM1, dM2) and torch.equal(dm1, dm2)


def test_same_descriptor_set_on_two_streams(ctx, torch):
    # calls with one descriptor set share its work-list counter: enqueued on two
    # streams without host synchronisation, they must still give the results of
    # the same calls made one after the other
    n = 600
    w = synth.config(2, nsub=n)
    assert w.ppc == 8
    desc, m_el, l_el = descriptors(w, range(n))
    pos, mass = particles(w, range(n))
    dpos = to_dev(pos)
    dmass = [to_dev(mass), to_dev(mass * 0.75 + 0.125)]
    prec = fmm.FMM_FP64_HARMONIC
    want = [fused(ctx, torch, desc, dpos, dm, 8, m_el, l_el, prec) for dm in dmass]
    want_m2l = []
    for Mw, _ in want:
        L = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.m2l(desc, Mw, L, prec)
        want_m2l.append(L)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[torch.full((m_el,), float("nan"), dtype=torch.float64, device="cuda"),
             torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda"),
             torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")] for _ in range(2)]
    torch.cuda.synchronize()
    for _ in range(3):
        for i in (0, 1):
            M, L, L2 = outs[i]
            ctx.p2m_m2l(desc, dpos, dmass[i], 8, M, L, prec, streams[i])
            ctx.m2l(desc, M, L2, prec, streams[i])
    torch.cuda.synchronize()
    for i in (0, 1):
        M, L, L2 = outs[i]
        assert torch.equal(L, want[i][1]), "stream %d: one-launch L differs" % i
        assert torch.equal(L2, want_m2l[i]), "stream %d: M2L-only L differs" % i
        assert torch.equal(L, L2), "stream %d: the two forms differ" % i


def test_binding_rejects_host_and_short_buffers(ctx, torch):
    # raised by the binding before the library is called: nothing is enqueued
    w = synth.config(2, nsub=2)
    desc, m_el, l_el = descriptors(w, range(2))
    M = torch.zeros(m_el, dtype=torch.float64, device="cuda")
    L = torch.zeros(l_el, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="cuda:0"):
        ctx.m2l(desc, M.cpu(), L)
    with pytest.raises(ValueError, match="elements"):
        ctx.m2l(desc, M, L[:-512])
    with pytest.raises(TypeError, match="float64"):
        ctx.m2l(desc, M, L.float())
    ctx.m2l(desc, M, L)
    torch.cuda.synchronize()
    assert torch.count_nonzero(L) == 0      # zero moments give zero expansions


def test_cache_eviction_over_two_streams(ctx, torch):
    # 12 descriptor sets (more than the 8 a context holds) and 24 distinct graphs
    # (more than the 16 it keeps), enqueued alternately on two streams without
    # host synchronisation: evicting a set drops only its own graphs, a released
    # graph has finished its last launch, and every result equals, bit for bit,
    # that of plain launches made one at a time on a fresh context
    rng = np.random.default_rng(77)
    sets = []
    for i in range(12):
        p = rng.integers(2, 5, size=3)
        masks = [synth.random_mask(rng) for _ in range(3)]
        desc, m_el, l_el = fmm.make_descriptors(p, rng.integers(0, 3, size=3), masks)
        M = torch.from_numpy(rng.standard_normal(m_el)).to("cuda")
        sets.append((desc, M, l_el))
    prec = fmm.FMM_FP64_HARMONIC
    with fmm.Context(0) as ref:
        ref.set_option(fmm.FMM_OPT_USE_GRAPH, 0)
        want = []
        for desc, M, l_el in sets:
            L = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
            ref.m2l(desc, M, L, prec)
            torch.cuda.synchronize()
            want.append(L)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda") for _, _, l_el in sets]
            for _ in range(2)]
    torch.cuda.synchronize()
    for r in range(2):
        for i, (desc, M, _) in enumerate(sets):
            ctx.m2l(desc, M, outs[r][i], prec, streams[(i + r) % 2])
    torch.cuda.synchronize()
    for r in range(2):
        for i in range(len(sets)):
            assert torch.equal(outs[r][i], want[i]), "pass %d, set %d" % (r, i)
