"""Pins of the multi-level oracle (oracle/tree.py): interaction lists by
enumeration, exact re-expansion identities of M2M and L2L, agreement of the
level M2L, near field and L2P with the single-level oracle on an interior
block, and convergence of the whole iteration to the brute-force sum."""
from itertools import product
from math import factorial

import numpy as np
import pytest

import oracle as O
import oracle.tree as T
import synth


def test_interaction_lists():
    S = set(O.stencil())
    lists = {sig: T.interaction_list(sig) for sig in product((0, 1), repeat=3)}
    union = set().union(*map(set, lists.values()))
    assert all(len(v) == 231 for v in lists.values()) and len(union) == 418
    assert union <= S and set(T.top_list()) <= union and len(T.top_list()) == 7 ** 3 - 33
    for sig, v in lists.items():
        # mirror symmetry: d in IL_sigma <=> -d in IL_(1 - sigma)
        mirror = tuple(1 - s for s in sig)
        assert {tuple(-x for x in d) for d in v} == set(lists[mirror])


def test_every_pair_of_finest_cells_is_counted_once():
    n = 16
    levels = T.tree_levels(n)
    g = np.arange(n)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    lists = {sig: set(T.interaction_list(sig)) for sig in product((0, 1), repeat=3)}
    top = set(T.top_list())
    for t in cells[::37]:
        count = np.zeros(len(cells), int)
        d0 = cells - t
        count += (np.sum(d0 * d0, axis=1) <= 4)
        for lvl in range(len(levels)):
            a_t, a_s = t >> lvl, cells >> lvl
            d = a_s - a_t
            keys = map(tuple, d)
            ref = top if lvl == len(levels) - 1 else lists[tuple(int(v) for v in a_t & 1)]
            count += np.fromiter((k in ref for k in keys), bool, len(cells))
        assert np.all(count == 1), (t, np.unique(count))


def test_m2m_is_p2m_about_the_parent_centres():
    n, h = 8, 0.5
    pos, mass = synth.grid_particles(3, n, h, 2)
    for p in (2, 4):
        Mc = T.p2m_grid(pos, mass, p, n, h)
        Mp = T.m2m(Mc, p, h)
        # parents' particles, moments taken directly about the parent centres
        P = pos.reshape(n, n, n, 2, 3)
        Mm = mass.reshape(n, n, n, 2)
        q = n // 2
        pp = P.reshape(q, 2, q, 2, q, 2, 2, 3).transpose(0, 2, 4, 1, 3, 5, 6, 7).reshape(q ** 3, 16, 3)
        mp = Mm.reshape(q, 2, q, 2, q, 2, 2).transpose(0, 2, 4, 1, 3, 5, 6).reshape(q ** 3, 16)
        want = T.p2m_grid(pp, mp, p, q, 2 * h)
        c = T._centres(q, 2 * h)[:, None, :]
        scale = T.p2m_grid(c + np.abs(pp - c), mp, p, q, 2 * h)
        assert np.all(np.abs(Mp - want) <= 1e-13 * scale)


def test_l2l_keeps_the_local_polynomial():
    rng = np.random.default_rng(4)
    for p, hc in ((3, 1.0), (4, 0.25)):
        C = O.ncomp(p)
        Lp = rng.standard_normal((C, 4, 4, 4))
        Lc = T.l2l(Lp, p, hc)
        ks = O.multi_indices(p)
        for _ in range(20):
            j = rng.integers(0, 8, 3)
            x = (j + rng.random(3)) * hc
            cc = (j + 0.5) * hc
            J = j // 2
            cp = (J + 0.5) * 2 * hc
            mono = lambda b: np.array([b[0] ** k[0] * b[1] ** k[1] * b[2] ** k[2] /
                                       (factorial(k[0]) * factorial(k[1]) * factorial(k[2])) for k in ks])
            vp = Lp[:, J[2], J[1], J[0]] @ mono(x - cp)
            vc = Lc[:, j[2], j[1], j[0]] @ mono(x - cc)
            assert abs(vp - vc) <= 1e-12 * (np.abs(Lp[:, J[2], J[1], J[0]]) @ np.abs(mono(x - cp)))


@pytest.mark.parametrize("p", [2, 3])
def test_level_m2l_matches_the_single_level_oracle(p):
    # an interior 8^3 block of a 32^3 level, seen as the centre of a 24^3 frame
    n, h = 32, 2.0
    rng = np.random.default_rng(7)
    C = O.ncomp(p)
    M = rng.standard_normal((C, n, n, n))
    L = T.m2l_level(M, p, h)
    frame = M[:, 4:28, 4:28, 4:28]
    for sig in product((0, 1), repeat=3):
        Lf = O.m2l(frame, p, h, offsets=T.interaction_list(sig))
        sub = (slice(None), slice(sig[2], 8, 2), slice(sig[1], 8, 2), slice(sig[0], 8, 2))
        got = L[:, 12:20, 12:20, 12:20][sub]
        scale = O.m2l_abs(frame, p, h, offsets=T.interaction_list(sig))[sub]
        assert np.all(np.abs(got - Lf[sub]) <= 1e-13 * scale)


def test_near_grid_and_l2p_grid_match_the_single_level_oracle():
    n, h, ppc = 32, 1.0, 2
    pos, mass = synth.grid_particles(5, n, h, ppc)
    P = pos.reshape(n, n, n, ppc, 3)[4:28, 4:28, 4:28].reshape(-1, ppc, 3) - 4 * h
    Mm = mass.reshape(n, n, n, ppc)[4:28, 4:28, 4:28].reshape(-1, ppc)
    near = T.near_grid(pos, mass, n, h).reshape(4, n, n, n, ppc)[:, 12:20, 12:20, 12:20]
    want = O.near_field(P, Mm, h).reshape(4, 8, 8, 8, ppc)
    scale = O.near_field_abs(P, Mm, h).reshape(4, 8, 8, 8, ppc)
    assert np.all(np.abs(near - want) <= 1e-13 * scale)
    L0 = np.random.default_rng(8).standard_normal((20, n, n, n))
    got = T.l2p_grid(L0, pos, 3, n, h).reshape(4, n, n, n, ppc)[:, 12:20, 12:20, 12:20]
    want = O.l2p(L0[:, 12:20, 12:20, 12:20], P, 3, h).reshape(4, 8, 8, 8, ppc)
    scale = O.l2p_abs(L0[:, 12:20, 12:20, 12:20], P, 3, h).reshape(4, 8, 8, 8, ppc)
    assert np.all(np.abs(got - want) <= 1e-13 * scale)


@pytest.mark.parametrize("n,ppc", [(8, 2), (16, 1)])
def test_solve_converges_to_the_direct_sum(n, ppc):
    pos, mass = synth.grid_particles(1, n, 1.0, ppc)
    ex = T.direct_all(pos, mass)
    err = {}
    for p in (2, 4):
        E = T.solve(pos, mass, p, n, 1.0).reshape(4, -1)
        phi = np.abs(E[0] - ex[0]) / ex[0]
        grad = np.abs(E[1:] - ex[1:]).max(axis=0) / np.abs(ex[1:]).max(axis=0)
        err[p] = (phi.max(), np.median(grad))
    assert err[4][0] < 5e-4 and err[4][0] < err[2][0] / 5, err
    assert err[4][1] < 1.5e-3 and err[4][1] < err[2][1] / 5, err


def test_coarsest_level_lists_agree_and_scales_bound_values():
    # on the 4-per-axis level every parent is near every other: the top list and
    # the interaction lists give the same sums there
    rng = np.random.default_rng(12)
    M = rng.standard_normal((20, 4, 4, 4))
    a, b = T.m2l_level(M, 3, 4.0, top=True), T.m2l_level(M, 3, 4.0, top=False)
    assert np.all(np.abs(a - b) <= 1e-14 * T.m2l_level(M, 3, 4.0, top=True, absolute=True))
    # the absolute variants bound the values they scale
    pos, mass = synth.grid_particles(2, 8, 1.0, 2)
    Ms, Ma = T.upward(pos, mass, 3, 8, 1.0), T.upward(pos, mass, 3, 8, 1.0, absolute=True)
    assert all(np.all(np.abs(x) <= y * (1 + 1e-12)) for x, y in zip(Ms, Ma))
    Ls, La = T.m2l_levels(Ms, 3, 1.0), T.m2l_levels(Ma, 3, 1.0, absolute=True)
    assert all(np.all(np.abs(x) <= y * (1 + 1e-12)) for x, y in zip(Ls, La))
    Lt, Lta = T.downward(Ls, 3, 1.0), T.downward(La, 3, 1.0, absolute=True)
    assert all(np.all(np.abs(x) <= y * (1 + 1e-12)) for x, y in zip(Lt, Lta))


def test_one_cell_path_matches_the_whole_iteration():
    # the per-cell route (direct moments of each source cell, direct shift to the
    # target) against the level-by-level iteration, at cells of every kind
    n, h, ppc, p = 16, 0.5, 2, 3
    pos, mass = synth.grid_particles(6, n, h, ppc)
    E = T.solve(pos, mass, p, n, h).reshape(4, n, n, n, ppc)
    Lt = T.downward(T.m2l_levels(T.upward(pos, mass, p, n, h), p, h), p, h)[0]
    for t in [(0, 0, 0), (7, 8, 9), (15, 3, 12), (5, 15, 15)]:
        lv, la = T.local_at(pos, mass, p, n, h, t), T.local_at(pos, mass, p, n, h, t, absolute=True)
        assert np.all(np.abs(lv - Lt[:, t[2], t[1], t[0]]) <= 1e-12 * la)
        ev, ea = T.evaluate_at(pos, mass, p, n, h, t), T.evaluate_at(pos, mass, p, n, h, t, absolute=True)
        assert np.all(np.abs(ev - E[:, t[2], t[1], t[0]]) <= 1e-12 * ea)
