"""GPU parity of the multi-level iteration on a uniform octree (fmm_tree_*)
through the C ABI against oracle/tree.py.

Each step is checked on oracle inputs (the oracle's M for the M2L, the
oracle's per-level L for the downward pass, the oracle's finest L for the
evaluation), per entry within 1e-12 of the step's rounding scale (the same
sums over absolute values). The whole solve is checked against the oracle's
solve within 1e-12 of the chained scale, and bitwise against the device
steps run one by one.
"""
import numpy as np
import pytest

import oracle.tree as T
import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import ensure_library, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


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


def split_levels(flat, p, n):
    C = fmm.ncomp(p)
    out, off = [], 0
    for m in T.tree_levels(n):
        out.append(flat[off:off + C * m ** 3].reshape(C, m, m, m))
        off += C * m ** 3
    return out


def flatten(levels):
    return np.concatenate([v.ravel() for v in levels])


def check(got, want, scale, what):
    err = np.abs(got - want)
    bad = ~(err <= TOL * scale)
    assert not bad.any(), "%s: %d entries off, worst ratio %.3g" % (
        what, bad.sum(), np.nanmax(err / np.maximum(scale, 1e-300)))


# (p, n, ppc, log2_h): orders 2-4, one to five levels below the top, and more
# than 8 particles per cell (the evaluation's particle chunks); every level of
# these domains runs in the one-block launch of the level M2L
CASES = [(2, 16, 2, 0), (3, 16, 3, -1), (4, 8, 2, 1), (3, 32, 1, 0), (3, 8, 11, 0)]


@pytest.mark.parametrize("p,n,ppc,lh", CASES)
def test_tree_steps_match_oracle(ctx, torch, p, n, ppc, lh):
    h = 2.0 ** lh
    tree = fmm.Tree(p, n, ppc, lh)
    nl, elems = fmm.tree_size(tree)
    assert nl == len(T.tree_levels(n))
    pos, mass = synth.grid_particles(10 + p, n, h, ppc)
    dpos, dmass = to_dev(pos), to_dev(mass)
    # upward: P2M + M2M
    M = torch.full((elems,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.tree_upward(tree, dpos, dmass, M)
    torch.cuda.synchronize()
    Mo, Ma = T.upward(pos, mass, p, n, h), T.upward(pos, mass, p, n, h, absolute=True)
    for lvl, (g, w, s) in enumerate(zip(split_levels(M.cpu().numpy(), p, n), Mo, Ma)):
        check(g, w, s, "M level %d" % lvl)
    # every level's M2L, on the oracle's moments, in the dense and the harmonic form
    Lo, La = T.m2l_levels(Mo, p, h), T.m2l_levels(Mo, p, h, absolute=True)
    for harmonic in (0, 1):
        th = fmm.Tree(p, n, ppc, lh, harmonic)
        L = torch.full((elems,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.tree_m2l(th, to_dev(flatten(Mo)), L)
        torch.cuda.synchronize()
        for lvl, (g, w, s) in enumerate(zip(split_levels(L.cpu().numpy(), p, n), Lo, La)):
            check(g, w, s, "L level %d (harmonic %d)" % (lvl, harmonic))
    # downward, on the oracle's per-level expansions
    Ld = to_dev(flatten(Lo))
    ctx.tree_downward(tree, Ld)
    torch.cuda.synchronize()
    Lt, Lta = T.downward(Lo, p, h), T.downward(Lo, p, h, absolute=True)
    for lvl, (g, w, s) in enumerate(zip(split_levels(Ld.cpu().numpy(), p, n), Lt, Lta)):
        check(g, w, s, "L total level %d" % lvl)
    # evaluation at the particles, on the oracle's finest-level total
    out = torch.full((4 * n ** 3 * ppc,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.tree_evaluate(tree, dpos, dmass, to_dev(flatten(Lt)), out)
    torch.cuda.synchronize()
    want = T.l2p_grid(Lt[0], pos, p, n, h) + T.near_grid(pos, mass, n, h)
    scale = T.l2p_grid_abs(Lt[0], pos, p, n, h) + T.near_grid(pos, mass, n, h, absolute=True)
    check(out.cpu().numpy().reshape(4, n ** 3, ppc), want, scale, "evaluation")


@pytest.mark.parametrize("p,n,ppc,lh,harmonic", [(3, 16, 2, 0, 0), (4, 16, 1, -2, 0), (3, 16, 2, 0, 1),
                                                   (4, 16, 1, -2, 1), (2, 32, 1, 1, 1)])
def test_tree_solve_matches_oracle_and_the_steps(ctx, torch, p, n, ppc, lh, harmonic):
    h = 2.0 ** lh
    tree = fmm.Tree(p, n, ppc, lh, harmonic)
    _, elems = fmm.tree_size(tree)
    pos, mass = synth.grid_particles(20 + p, n, h, ppc)
    dpos, dmass = to_dev(pos), to_dev(mass)
    M = torch.empty(elems, dtype=torch.float64, device="cuda")
    L = torch.empty(elems, dtype=torch.float64, device="cuda")
    out = torch.empty(4 * n ** 3 * ppc, dtype=torch.float64, device="cuda")
    ctx.tree_solve(tree, dpos, dmass, M, L, out)
    # the same steps one by one: bitwise equal
    M2, L2, out2 = torch.empty_like(M), torch.empty_like(L), torch.empty_like(out)
    ctx.tree_upward(tree, dpos, dmass, M2)
    ctx.tree_m2l(tree, M2, L2)
    ctx.tree_downward(tree, L2)
    ctx.tree_evaluate(tree, dpos, dmass, L2, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2) and torch.equal(L, L2)
    want = T.solve(pos, mass, p, n, h)
    Ma = T.upward(pos, mass, p, n, h, absolute=True)
    Lta = T.downward(T.m2l_levels(Ma, p, h, absolute=True), p, h, absolute=True)
    scale = T.l2p_grid_abs(Lta[0], pos, p, n, h) + T.near_grid(pos, mass, n, h, absolute=True)
    check(out.cpu().numpy().reshape(4, n ** 3, ppc), want, scale, "solve")


def test_tree_solve_accuracy_against_the_direct_sum(ctx, torch):
    # a property at any size: the FMM truncation error of the whole iteration
    n, ppc, p = 16, 2, 4
    tree = fmm.Tree(p, n, ppc, 0)
    _, elems = fmm.tree_size(tree)
    pos, mass = synth.grid_particles(30, n, 1.0, ppc)
    M = torch.empty(elems, dtype=torch.float64, device="cuda")
    L = torch.empty(elems, dtype=torch.float64, device="cuda")
    out = torch.empty(4 * n ** 3 * ppc, dtype=torch.float64, device="cuda")
    ctx.tree_solve(tree, to_dev(pos), to_dev(mass), M, L, out)
    torch.cuda.synchronize()
    E = out.cpu().numpy().reshape(4, -1)
    ex = T.direct_all(pos, mass)
    assert np.max(np.abs(E[0] - ex[0]) / ex[0]) < 5e-4
    assert np.median(np.abs(E[1:] - ex[1:]).max(axis=0) / np.abs(ex[1:]).max(axis=0)) < 1.5e-3


def test_tree_m2l_wide_and_narrow_launches(ctx, torch):
    # 64^3: the 64 level goes in the launch of two-block workgroups, the 32 .. 4
    # levels in the one-block launch; every level of both forms against the oracle
    p, n, ppc, h = 2, 64, 1, 1.0
    pos, mass = synth.grid_particles(12, n, h, ppc)
    Mo = T.upward(pos, mass, p, n, h)
    Lo, La = T.m2l_levels(Mo, p, h), T.m2l_levels(Mo, p, h, absolute=True)
    for harmonic in (0, 1):
        tree = fmm.Tree(p, n, ppc, 0, harmonic)
        _, elems = fmm.tree_size(tree)
        L = torch.full((elems,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.tree_m2l(tree, to_dev(flatten(Mo)), L)
        torch.cuda.synchronize()
        for lvl, (g, w, s) in enumerate(zip(split_levels(L.cpu().numpy(), p, n), Lo, La)):
            check(g, w, s, "64^3 L level %d (harmonic %d)" % (lvl, harmonic))


# a seeded sweep over order, spacing (the extremes of log2_h), form and particle count
SWEEP = [(p, lh, harm, ppc) for p, lh, harm, ppc in
         zip([2, 3, 4, 2, 3, 4, 3, 2], [-4, 4, 2, -3, -2, 3, 1, 0], [1, 0, 1, 0, 1, 0, 1, 1], [1, 2, 1, 9, 1, 1, 4, 2])]


@pytest.mark.parametrize("p,lh,harmonic,ppc", SWEEP)
def test_tree_solve_sweep(ctx, torch, p, lh, harmonic, ppc):
    n, h = 8, 2.0 ** lh
    tree = fmm.Tree(p, n, ppc, lh, harmonic)
    _, elems = fmm.tree_size(tree)
    pos, mass = synth.grid_particles(50 + p + 10 * ppc, n, h, ppc)
    M = torch.empty(elems, dtype=torch.float64, device="cuda")
    L = torch.empty(elems, dtype=torch.float64, device="cuda")
    out = torch.empty(4 * n ** 3 * ppc, dtype=torch.float64, device="cuda")
    ctx.tree_solve(tree, to_dev(pos), to_dev(mass), M, L, out)
    torch.cuda.synchronize()
    want = T.solve(pos, mass, p, n, h)
    Ma = T.upward(pos, mass, p, n, h, absolute=True)
    Lta = T.downward(T.m2l_levels(Ma, p, h, absolute=True), p, h, absolute=True)
    scale = T.l2p_grid_abs(Lta[0], pos, p, n, h) + T.near_grid(pos, mass, n, h, absolute=True)
    check(out.cpu().numpy().reshape(4, n ** 3, ppc), want, scale, "sweep p=%d lh=%d harmonic=%d ppc=%d" % (p, lh, harmonic, ppc))
