"""Pins of the CPU oracle against facts fixed by mathematics, not by itself.

Each test ties one part of the oracle to something independent of its code:
the Legendre addition theorem (scipy), exact symbolic derivatives stored in
tests/golden/, textbook closed forms of the first derivatives of 1/r, the
direct Newtonian sum, the rigorous truncation bound, exact symmetries of the
stencil and of the Laplace kernel, and the adjoint identities.
"""
import os
from itertools import product
from math import factorial

import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dtensor_integer_points.txt")
EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------------------
# index set and stencil
# ---------------------------------------------------------------------------

def test_index_set_graded_order():
    ks = O.multi_indices(3)
    assert len(ks) == O.ncomp(3) == 20
    assert [O.ncomp(p) for p in (0, 1, 2, 3, 4)] == [1, 4, 10, 20, 35]
    assert ks[:4] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    assert ks[4:10] == [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]
    assert ks[10] == (3, 0, 0) and ks[-1] == (0, 0, 3)
    assert len(set(ks)) == len(ks)


def test_stencil_shell():
    S = O.stencil()
    assert len(S) == 892
    q = [dx * dx + dy * dy + dz * dz for dx, dy, dz in S]
    assert min(q) == 5 and max(q) == 36
    assert max(max(abs(c) for c in d) for d in S) == 6
    per_dz = [sum(1 for d in S if d[2] == z) for z in range(-6, 7)]
    assert per_dz == [1, 37, 69, 89, 100, 100, 100, 100, 100, 89, 69, 37, 1]
    Sset = set(S)
    assert all((-a, -b, -c) in Sset for a, b, c in S)          # symmetric
    assert O.pair_count(O.FULL_MASK) == 512 * 892


# ---------------------------------------------------------------------------
# derivative tensors of 1/r
# ---------------------------------------------------------------------------

def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#"):
                continue
            v = line.split()
            rows.append((tuple(int(x) for x in v[0:3]), tuple(int(x) for x in v[3:6]), float(v[7])))
    return rows


def test_dtensor_matches_exact_integer_points():
    rows = _golden_rows()
    assert len(rows) > 1000
    by_order = {}
    for d, m, val in rows:
        by_order.setdefault((d, sum(m)), []).append(abs(val))
    worst = 0.0
    for d, m, exact in rows:
        got = float(O.dtensor(m, np.array(d, dtype=np.float64)))
        scale = max(by_order[(d, sum(m))])
        err = abs(got - exact) / scale
        worst = max(worst, err)
    # Hobson's sum has alternating terms: bound relative to the order's largest entry
    assert worst < 64 * EPS, worst


def test_dtensor_legendre_addition_theorem():
    rng = np.random.default_rng(11)
    R = rng.normal(size=(64, 3)) * 3.0
    a = rng.normal(size=(64, 3))
    a *= (0.7 * np.linalg.norm(R, axis=1) / np.linalg.norm(a, axis=1) * rng.random(64))[:, None]
    rn, an = np.linalg.norm(R, axis=1), np.linalg.norm(a, axis=1)
    cos = np.sum(a * R, axis=1) / (an * rn)
    for j in range(0, 9):
        lhs = np.zeros(64)
        for k in O.multi_indices(j):
            if sum(k) != j:
                continue
            kf = factorial(k[0]) * factorial(k[1]) * factorial(k[2])
            lhs += (-a[:, 0]) ** k[0] * (-a[:, 1]) ** k[1] * (-a[:, 2]) ** k[2] / kf * O.dtensor(k, R)
        rhs = an ** j * eval_legendre(j, cos) / rn ** (j + 1)
        scale = an ** j / rn ** (j + 1)
        assert np.max(np.abs(lhs - rhs) / scale) < 1e-13, j


def test_dtensor_laplace_traceless():
    rng = np.random.default_rng(3)
    R = rng.normal(size=(32, 3)) * 4
    for m in O.multi_indices(8):
        lap = sum(O.dtensor((m[0] + e[0], m[1] + e[1], m[2] + e[2]), R)
                  for e in ((2, 0, 0), (0, 2, 0), (0, 0, 2)))
        scale = max(np.max(np.abs(O.dtensor(mm, R))) for mm in
                    [(m[0] + 2, m[1], m[2]), (m[0], m[1] + 2, m[2]), (m[0], m[1], m[2] + 2)])
        assert np.max(np.abs(lap)) <= 1e-13 * scale


def test_tensor_transpose_symmetry_and_h_scaling():
    S = O.stencil()
    idx = {d: i for i, d in enumerate(S)}
    for p in (2, 3):
        T = O.stencil_tensors(p, 1.0)
        for i, (a, b, c) in enumerate(S):
            assert np.array_equal(T[idx[(-a, -b, -c)]], T[i].T)
        order = np.array([sum(k) for k in O.multi_indices(p)], dtype=np.float64)
        for h in (0.5, 0.25):
            Th = O.stencil_tensors(p, h)
            scaled = T * (h ** -order)[None, :, None] * (h ** (-1.0 - order))[None, None, :]
            assert np.array_equal(Th, scaled)


# ---------------------------------------------------------------------------
# P2M
# ---------------------------------------------------------------------------

def _one_particle_frame(cell_xyz, offset, m=1.0, h=1.0, ppc=1):
    pos = O.cell_centres(h)[:, None, :].copy()
    mass = np.zeros((O.NCELL, ppc))
    x, y, z = cell_xyz
    cell = x + 24 * y + 576 * z
    pos[cell, 0] += np.asarray(offset, dtype=np.float64) * h
    mass[cell, 0] = m
    return pos, mass, cell


def test_p2m_single_particle_by_hand():
    a = (0.25, -0.125, 0.375)
    pos, mass, cell = _one_particle_frame((10, 11, 12), a, m=2.0)
    M = O.p2m(pos, mass, 3, 1.0).reshape(20, -1)[:, cell]
    ks = O.multi_indices(3)
    want = {(0, 0, 0): 2.0, (1, 0, 0): 0.5, (0, 1, 0): -0.25, (0, 0, 1): 0.75,
            (2, 0, 0): 2.0 * 0.0625 / 2, (1, 1, 0): 2.0 * 0.25 * -0.125,
            (0, 0, 2): 2.0 * 0.140625 / 2, (2, 1, 0): 2.0 * 0.0625 * -0.125 / 2,
            (0, 0, 3): 2.0 * 0.052734375 / 6, (1, 1, 1): 2.0 * 0.25 * -0.125 * 0.375}
    for k, v in want.items():
        assert M[ks.index(k)] == pytest.approx(v, rel=1e-15, abs=1e-18)
    assert np.count_nonzero(O.p2m(pos, mass, 3, 1.0)) == 20


def test_p2m_mask_zeroes_absent_blocks(cfg1_inputs):
    pos, mass = cfg1_inputs
    mask = O.FULL_MASK & ~(1 << 0) & ~(1 << 26)
    M = O.p2m(pos, mass, 2, 1.0, mask)
    assert np.all(M[:, :8, :8, :8] == 0) and np.all(M[:, 16:, 16:, 16:] == 0)
    assert np.all(M[0, 8:16, 8:16, 8:16] > 0)


# ---------------------------------------------------------------------------
# M2L against closed forms and the direct sum
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("h", [1.0, 0.5])
def test_single_pair_closed_forms(h):
    d = (3, -2, 1)
    t = (4, 4, 4)
    src = tuple(t[i] + 8 + d[i] for i in range(3))
    pos, mass, _ = _one_particle_frame(src, (0, 0, 0), h=h)
    L = O.m2l(O.p2m(pos, mass, 2, h), 2, h)[:, t[2], t[1], t[0]]
    R = -np.array(d, dtype=np.float64) * h
    r = np.linalg.norm(R)
    ks = O.multi_indices(2)
    want = {(0, 0, 0): 1 / r}
    for i, e in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        want[e] = -R[i] / r ** 3
    for i in range(3):
        for j in range(i, 3):
            k = [0, 0, 0]
            k[i] += 1
            k[j] += 1
            want[tuple(k)] = 3 * R[i] * R[j] / r ** 5 - (1 / r ** 3 if i == j else 0.0)
    for k, v in want.items():
        assert L[ks.index(k)] == pytest.approx(v, rel=1e-14), k


@pytest.mark.parametrize("p", [0, 2, 3])
def test_monopole_leaves_are_exact(p):
    # the paper's leaf case: each cell's mass as a monopole at its centre
    _, mass = synth.subgrid_particles(7, ppc=2)
    pos = np.repeat(O.cell_centres(1.0)[:, None, :], 2, axis=1)
    M = O.p2m(pos, mass, p, 1.0)
    L = O.m2l(M, p, 1.0)
    La = O.m2l_abs(M, p, 1.0)
    targets = [(0, 0, 0), (7, 7, 7), (3, 5, 2)]
    ex = O.direct_sum(pos, mass, 1.0, p, targets=targets)
    for it, (x, y, z) in enumerate(targets):
        assert np.all(np.abs(L[:, z, y, x] - ex[it]) <= 1e-13 * La[:, z, y, x])


def test_truncation_bound_and_decay():
    # one target, a handful of offsets, random particles: the L_0 error is
    # within the rigorous Legendre tail bound for every p, and aggregate
    # errors of every component fall with p.
    offs = [(3, 0, 0), (-2, 1, 0), (0, -2, -2), (1, 1, 3), (2, 2, 1), (-4, 0, 1)]
    pos, mass = synth.subgrid_particles(5)
    t = (3, 4, 2)
    ct = (np.array(t) + 8 + 0.5)
    ex = O.direct_sum(pos, mass, 1.0, 2, offsets=offs, targets=[t])[0]
    jt = np.array(t) + 8
    bound_terms = []
    for d in offs:
        js = jt + np.array(d)
        cell = js[0] + 24 * js[1] + 576 * js[2]
        cs = js + 0.5
        a = np.linalg.norm(pos[cell] - cs, axis=1)
        Rn = np.linalg.norm(ct - cs)
        bound_terms.append((mass[cell], a, Rn))
    errs = []
    for p in range(0, 9):
        L = O.m2l(O.p2m(pos, mass, p, 1.0), p, 1.0, offsets=offs)[:, t[2], t[1], t[0]]
        bound = sum(np.sum(m * (a / Rn) ** (p + 1) / (Rn - a)) for m, a, Rn in bound_terms)
        err0 = abs(L[0] - ex[0])
        assert err0 <= bound * (1 + 1e-12) + 1e-13 * abs(ex[0]), (p, err0, bound)
        errs.append(np.abs(L[:min(len(L), 10)] - ex[:min(len(L), 10)]).max())
    # not strictly monotone step by step; monotone every two orders
    for p in range(0, 7):
        assert errs[p + 2] < errs[p], errs


def test_error_falls_with_p_on_aggregate():
    offs = O.stencil(5, 12)
    pos, mass = synth.subgrid_particles(9)
    targets = [(x, y, z) for z in (2, 5) for y in (1, 6) for x in range(8)]
    ex = O.direct_sum(pos, mass, 1.0, 1, offsets=offs, targets=targets)
    errs = []
    for p in range(1, 6):
        L = O.m2l(O.p2m(pos, mass, p, 1.0), p, 1.0, offsets=offs)
        got = np.stack([L[:4, z, y, x] for (x, y, z) in targets])
        errs.append(np.mean(np.abs(got - ex) / np.abs(ex).max(axis=0)))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


# ---------------------------------------------------------------------------
# invariants of M2L
# ---------------------------------------------------------------------------

def _random_moments(seed, C, shape=(24, 24, 24)):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(C,) + shape)


def test_linearity():
    p, C = 2, 10
    M1, M2 = _random_moments(1, C), _random_moments(2, C)
    L = O.m2l(2.5 * M1 - 0.75 * M2, p, 1.0)
    La = O.m2l_abs(2.5 * np.abs(M1) + 0.75 * np.abs(M2), p, 1.0)
    ref = 2.5 * O.m2l(M1, p, 1.0) - 0.75 * O.m2l(M2, p, 1.0)
    assert np.all(np.abs(L - ref) <= 1e-13 * La)


def test_translation_invariance():
    p, C = 2, 10
    F = _random_moments(4, C, (25, 24, 24))          # [C][z][y][x], 25 planes in z
    A = F[:, 0:24]
    B = F[:, 1:25]
    LA, LB = O.m2l(A, p, 1.0), O.m2l(B, p, 1.0)
    La = O.m2l_abs(A, p, 1.0)
    # target z in B equals target z+1 in A
    assert np.all(np.abs(LA[:, 1:] - LB[:, :-1]) <= 1e-13 * La[:, 1:])


def _cubic_map(A, ks, perm, signs):
    """Apply the cubic symmetry (reflect axis i where signs[i] < 0, then new axis i =
    old axis perm[i]) to a component-major field A [C][z][y][x]: cells move with the
    map, component k picks up prod (-1)^k_i over reflected axes and is relabelled
    k'_i = k_perm[i]."""
    B = np.array(A, dtype=np.float64)
    for ax in range(3):
        if signs[ax] < 0:
            B = np.flip(B, axis=3 - ax)
            B = B * np.array([(-1.0) ** k[ax] for k in ks])[:, None, None, None]
    # [C][z][y][x] -> axes in x, y, z order, permute, back
    Bx = np.transpose(B, (0, 3, 2, 1))
    Bx = np.transpose(Bx, (0,) + tuple(1 + q for q in perm))
    B = np.transpose(Bx, (0, 3, 2, 1))
    src_of = [ks.index(tuple(k[perm[i]] for i in range(3))) for k in ks]
    out = np.empty_like(B)
    for c, s in enumerate(src_of):
        out[s] = B[c]
    return out


def test_cubic_group_equivariance():
    # all 48 symmetries of the cube (6 axis permutations x 8 reflections) map the
    # shell stencil to itself, so M2L commutes with each of them; they include the
    # z reflection and the permutations that move z, not only x reflection and x<->y
    from itertools import permutations
    p = 3
    ks = O.multi_indices(p)
    M = _random_moments(5, len(ks))
    L = O.m2l(M, p, 1.0)
    La = O.m2l_abs(M, p, 1.0)
    count = 0
    for perm in permutations(range(3)):
        for signs in product((1, -1), repeat=3):
            Lg = O.m2l(_cubic_map(M, ks, perm, signs), p, 1.0)
            want = _cubic_map(L, ks, perm, signs)
            scale = np.abs(_cubic_map(La, ks, perm, signs))
            assert np.all(np.abs(Lg - want) <= 1e-13 * scale), (perm, signs)
            count += 1
    assert count == 48
    # the map itself is not trivial: a z reflection changes a generic field
    assert not np.allclose(_cubic_map(M, ks, (0, 1, 2), (1, 1, -1)), M)
    assert not np.allclose(_cubic_map(M, ks, (2, 1, 0), (1, 1, 1)), M)


def test_local_expansion_is_traceless_and_ignores_trace_moments():
    p = 3
    ks = O.multi_indices(p)
    M = _random_moments(6, len(ks))
    L = O.m2l(M, p, 1.0)
    La = O.m2l_abs(M, p, 1.0)
    for n in ks:
        if sum(n) > p - 2:
            continue
        tr = [ks.index((n[0] + e[0], n[1] + e[1], n[2] + e[2])) for e in ((2, 0, 0), (0, 2, 0), (0, 0, 2))]
        s = L[tr[0]] + L[tr[1]] + L[tr[2]]
        assert np.all(np.abs(s) <= 1e-13 * (La[tr[0]] + La[tr[1]] + La[tr[2]]))
    M2 = M.copy()
    for k in ((2, 0, 0), (0, 2, 0), (0, 0, 2)):
        M2[ks.index(k)] += 3.0
    L2 = O.m2l(M2, p, 1.0)
    assert np.all(np.abs(L2 - L) <= 1e-13 * O.m2l_abs(np.abs(M2) + np.abs(M), p, 1.0))


def test_masks_zero_nan_poison_and_block_superposition():
    p, C = 2, 10
    M = _random_moments(8, C)
    rng = np.random.default_rng(8)
    mask = synth.random_mask(rng)
    pres = O.present_cells(mask)
    poisoned = np.where(pres[None], M, np.nan)
    L = O.m2l(poisoned, p, 1.0, mask)
    assert np.all(np.isfinite(L))
    L0 = O.m2l(np.where(pres[None], M, 0.0), p, 1.0)
    assert np.array_equal(L, L0)
    # the 27 single-block results add up to the full result
    full = O.m2l(M, p, 1.0)
    La = O.m2l_abs(M, p, 1.0)
    acc = sum(O.m2l(M, p, 1.0, 1 << b) for b in range(27))
    assert np.all(np.abs(acc - full) <= 1e-13 * La)


def test_h_scaling_of_m2l():
    p = 3
    ks = O.multi_indices(p)
    order = np.array([sum(k) for k in ks], dtype=np.float64)
    M = _random_moments(12, len(ks))
    for h in (0.5, 0.25):
        Lh = O.m2l(M, p, h)
        L1 = O.m2l(M * (h ** -order)[:, None, None, None], p, 1.0) * (h ** (-1 - order))[:, None, None, None]
        La = O.m2l_abs(M, p, h)
        assert np.all(np.abs(Lh - L1) <= 1e-14 * La)


# ---------------------------------------------------------------------------
# adjoints
# ---------------------------------------------------------------------------

def test_m2l_adjoint_dot_product_and_transpose_form():
    p = 3
    ks = O.multi_indices(p)
    C = len(ks)
    rng = np.random.default_rng(21)
    mask = synth.random_mask(rng)
    M = _random_moments(22, C)
    W = rng.normal(size=(C, 8, 8, 8))
    for h in (1.0, 0.5):
        L = O.m2l(M, p, h, mask)
        G = O.m2l_adjoint(W, p, h, mask)
        lhs, rhs = np.sum(W * L), np.sum(G * M)
        scale = np.sum(np.abs(W) * O.m2l_abs(M, p, h, mask))
        assert abs(lhs - rhs) <= 1e-13 * scale
    # the adjoint equals the forward operator on zero-padded W with the
    # tables of the opposite offset, G_k(s) = sum_e sum_n W_n(s + e) T_e[n][k]
    S = O.stencil()
    T = O.stencil_tensors(p, 1.0)
    Wpad = np.zeros((C, 24, 24, 24))
    Wpad[:, 8:16, 8:16, 8:16] = W
    G = O.m2l_adjoint(W, p, 1.0)
    Ga = O.m2l_adjoint_abs(W, p, 1.0)
    pres = O.present_cells(O.FULL_MASK)
    for s in [(2, 2, 2), (9, 12, 14), (21, 3, 11), (15, 15, 8)]:
        sx, sy, sz = s
        g = np.zeros(C)
        for (ex, ey, ez), Te in zip(S, T):
            x, y, z = sx + ex, sy + ey, sz + ez
            if 0 <= x < 24 and 0 <= y < 24 and 0 <= z < 24:
                g += Te.T @ Wpad[:, z, y, x]
        assert pres[sz, sy, sx]
        assert np.all(np.abs(g - G[:, sz, sy, sx]) <= 1e-13 * Ga[:, sz, sy, sx])
    assert np.all(G[:, :2] == 0) and np.all(G[:, :, :, 22:] == 0)


def test_p2m_adjoint_dot_product(cfg1_inputs):
    pos, mass = cfg1_inputs
    p = 3
    rng = np.random.default_rng(31)
    mask = synth.random_mask(rng)
    G = rng.normal(size=(20, 24, 24, 24))
    M = O.p2m(pos, mass, p, 1.0, mask)
    g = O.p2m_adjoint(pos, G, p, 1.0, mask)
    assert np.sum(G * M) == pytest.approx(np.sum(g * mass), rel=1e-12)
    pres = O.present_cells(mask).reshape(-1)
    assert np.all(g[~pres] == 0)


def test_mass_gradient_matches_central_differences():
    # loss = sum w . L is linear in the masses, so central differences are
    # exact up to rounding; the difference is taken entry-wise before the sum
    p, h = 3, 1.0
    pos, mass = synth.subgrid_particles(5, 0)
    rng = np.random.default_rng(41)
    w = rng.normal(size=(20, 8, 8, 8))
    grad = O.p2m_adjoint(pos, O.m2l_adjoint(w, p, h), p, h)
    eps = 1e-6
    for cell, i in [(9 + 24 * 10 + 576 * 11, 3), (2 + 24 * 21 + 576 * 5, 0), (14 + 24 * 8 + 576 * 19, 7)]:
        mp, mm = mass.copy(), mass.copy()
        mp[cell, i] += eps
        mm[cell, i] -= eps
        Lp = O.m2l(O.p2m(pos, mp, p, h), p, h)
        Lm = O.m2l(O.p2m(pos, mm, p, h), p, h)
        fd = np.sum(w * (Lp - Lm)) / (2 * eps)
        gmax = np.max(np.abs(grad))
        assert abs(fd - grad[cell, i]) <= 1e-5 * max(abs(grad[cell, i]), 1e-3 * gmax)


def test_split32_expectation_model_error_scale(cfg1_inputs):
    pos, mass = cfg1_inputs
    M = O.p2m(pos, mass, 3, 1.0)
    L = O.m2l(M, 3, 1.0)
    La = O.m2l_abs(M, 3, 1.0)
    Ls = O.m2l_split32_emulated(M, 3, 1.0)
    rel = np.abs(Ls - L) / La
    # FP32 accumulation per block caps the error near 2^-24 of Labs
    assert 1e-10 < np.max(rel) < 1e-6
    assert np.median(rel) < 1e-7


def test_half_spacing_frame_geometry_against_direct_sum():
    # particles drawn inside cells [j h, (j+1) h) at h = 1/2: moments about the
    # centres have |a| <= h/2 per axis, and M2L agrees with the direct sum to
    # the truncation level
    h = 0.5
    pos, mass = synth.subgrid_particles(13, h=h)
    a = pos - O.cell_centres(h)[:, None, :]
    assert np.all(np.abs(a) <= h / 2)
    M = O.p2m(pos, mass, 4, h)
    assert np.all(np.abs(M[1:4]) <= (h / 2) * M[0][None] + 1e-15)
    offs = O.stencil(5, 9)
    targets = [(1, 2, 3), (6, 6, 0)]
    ex = O.direct_sum(pos, mass, h, 2, offsets=offs, targets=targets)
    L = O.m2l(M, 4, h, offsets=offs)
    for it, (x, y, z) in enumerate(targets):
        assert np.max(np.abs(L[:10, z, y, x] - ex[it]) / np.abs(ex[it]).max()) < 2e-3


# ---------------------------------------------------------------------------
# harmonic (traceless) form
# ---------------------------------------------------------------------------

def test_harmonic_fold_structure_and_trace_annihilation():
    for p in range(0, 7):
        hs = O.harmonic_indices(p)
        assert len(hs) == (p + 1) ** 2
        assert all(k[2] <= 1 for k in hs)
        ks = O.multi_indices(p)
        F = O.harmonic_fold(p)
        assert np.array_equal(F, np.round(F))              # integer coefficients
        for row, k in enumerate(ks):
            nz = np.nonzero(F[row])[0]
            assert all(sum(hs[c]) == sum(k) for c in nz)   # folding keeps the order
            if k in hs:
                assert list(nz) == [hs.index(k)] and F[row, nz[0]] == 1.0
        # a pure trace (sum_i delta_{m + 2 e_i}) carries no field: it folds to zero exactly
        for m in O.multi_indices(p - 2) if p >= 2 else []:
            Mt = np.zeros(len(ks))
            for e in ((2, 0, 0), (0, 2, 0), (0, 0, 2)):
                Mt[ks.index((m[0] + e[0], m[1] + e[1], m[2] + e[2]))] += 1.0
            assert np.array_equal(F.T @ Mt, np.zeros(len(hs)))


def test_harmonic_fold_reproduces_derivative_tensors():
    # D_{k+n}(R) is harmonic in k (Laplace, via Hobson's formula): the fold must
    # rebuild every D_{k+n} from the k_z <= 1 ones
    rng = np.random.default_rng(7)
    R = rng.normal(size=3) * 3.0
    for p in (2, 3, 4):
        ks = O.multi_indices(p)
        F = O.harmonic_fold(p)
        hs = O.harmonic_indices(p)
        D = O.dtensor_all(2 * p, R)
        for n in ks:
            col = np.array([D[(k[0] + n[0], k[1] + n[1], k[2] + n[2])] for k in ks])
            colh = np.array([D[(k[0] + n[0], k[1] + n[1], k[2] + n[2])] for k in hs])
            scale = np.abs(col).max()
            assert np.max(np.abs(F @ colh - col)) <= 1e-12 * scale


@pytest.mark.parametrize("p,h,seed,masked", [(2, 1.0, 0, False), (3, 1.0, 0, False),
                                              (3, 0.5, 11, True), (4, 0.25, 12, True)])
def test_harmonic_m2l_equals_dense(p, h, seed, masked):
    pos, mass = synth.subgrid_particles(seed, h=h)
    mask = synth.random_mask(np.random.default_rng(seed)) if masked else O.FULL_MASK
    M = O.p2m(pos, mass, p, h, mask)
    Ld = O.m2l(M, p, h, mask)
    Lh = O.m2l_harmonic(M, p, h, mask)
    La = O.m2l_abs(M, p, h, mask)
    assert np.max(np.abs(Lh - Ld) / La) <= 1e-13


# ---------------------------------------------------------------------------
# evaluation at the particles: near field and L2P
# ---------------------------------------------------------------------------

def _exact_same_level(pos, mass, h, tcells, mask=O.FULL_MASK):
    """Brute force: potential and gradient at the particles of the given target
    cells from every particle of the cells with |d|^2 <= 36 (present blocks),
    excluding the particle itself; explicit loops over particles."""
    pres = O.present_cells(mask)
    out = []
    for (tx, ty, tz) in tcells:
        j = (tx + 8, ty + 8, tz + 8)
        ct = j[0] + 24 * j[1] + 576 * j[2]
        phis, grads = [], []
        for i in range(pos.shape[1]):
            y = pos[ct, i]
            phi, g = 0.0, np.zeros(3)
            for dz in range(-6, 7):
                for dy in range(-6, 7):
                    for dx in range(-6, 7):
                        if dx * dx + dy * dy + dz * dz > 36:
                            continue
                        js = (j[0] + dx, j[1] + dy, j[2] + dz)
                        if not pres[js[2], js[1], js[0]]:
                            continue
                        cs = js[0] + 24 * js[1] + 576 * js[2]
                        for k in range(pos.shape[1]):
                            if cs == ct and k == i:
                                continue
                            v = y - pos[cs, k]
                            r = np.sqrt(v @ v)
                            phi += mass[cs, k] / r
                            g -= mass[cs, k] * v / r ** 3
            phis.append(phi)
            grads.append(g)
        out.append((np.array(phis), np.array(grads)))
    return out


def test_near_stencil_complements_the_shell():
    N, S = set(O.near_stencil()), set(O.stencil())
    assert len(N) == 33 and (0, 0, 0) in N and not (N & S)
    assert N | S == set(O.stencil(0, 36))


def test_near_field_against_pair_loop():
    # independent explicit loops over particle pairs, ppc = 2, absent blocks
    pos, mass = synth.subgrid_particles(21, ppc=2)
    mask = O.FULL_MASK & ~(1 << 4) & ~(1 << 14)     # blocks next to the centre removed
    nf = O.near_field(pos, mass, 1.0, mask)
    pres = O.present_cells(mask)
    for (tx, ty, tz) in [(0, 0, 0), (7, 3, 0), (2, 7, 7), (4, 4, 4)]:
        t = tx + 8 * ty + 64 * tz
        j = (tx + 8, ty + 8, tz + 8)
        ct = j[0] + 24 * j[1] + 576 * j[2]
        for i in range(2):
            phi, g = 0.0, np.zeros(3)
            for z in range(j[2] - 2, j[2] + 3):
                for y in range(j[1] - 2, j[1] + 3):
                    for x in range(j[0] - 2, j[0] + 3):
                        if (x - j[0]) ** 2 + (y - j[1]) ** 2 + (z - j[2]) ** 2 > 4 or not pres[z, y, x]:
                            continue
                        cs = x + 24 * y + 576 * z
                        for k in range(2):
                            if cs == ct and k == i:
                                continue
                            v = pos[ct, i] - pos[cs, k]
                            r = np.sqrt(v @ v)
                            phi += mass[cs, k] / r
                            g -= mass[cs, k] * v / r ** 3
            assert abs(nf[0, t, i] - phi) <= 1e-13 * phi
            assert np.max(np.abs(nf[1:, t, i] - g)) <= 1e-12 * np.abs(g).max()


def test_l2p_is_the_taylor_polynomial_of_far_sources():
    # L from exact derivatives of a far shell of sources: L2P at the particles must
    # approach the sources' exact potential and field as p grows (|b| / R <= 0.2)
    h = 1.0
    pos, mass = synth.subgrid_particles(22)
    far = O.stencil(25, 36)
    targets = [(0, 0, 0), (5, 2, 7)]
    errs = []
    for p in (2, 4):
        Lx = O.direct_sum(pos, mass, h, p, offsets=far, targets=targets)     # [2, C]
        L = np.zeros((O.ncomp(p), 512))
        for it, (x, y, z) in enumerate(targets):
            L[:, x + 8 * y + 64 * z] = Lx[it]
        ev = O.l2p(L.reshape(-1, 8, 8, 8), pos, p, h)
        worst = 0.0
        for (x, y, z) in targets:
            t = x + 8 * y + 64 * z
            ct = (x + 8) + 24 * (y + 8) + 576 * (z + 8)
            for i in range(8):
                yv = pos[ct, i]
                phi, g = 0.0, np.zeros(3)
                for d in far:
                    cs = (x + 8 + d[0]) + 24 * (y + 8 + d[1]) + 576 * (z + 8 + d[2])
                    v = yv[None, :] - pos[cs]
                    r = np.sqrt(np.sum(v * v, axis=1))
                    phi += np.sum(mass[cs] / r)
                    g -= np.sum((mass[cs] / r ** 3)[:, None] * v, axis=0)
                worst = max(worst, abs(ev[0, t, i] - phi) / phi,
                            np.max(np.abs(ev[1:, t, i] - g)) / np.abs(g).max())
        errs.append(worst)
    assert errs[1] < 2e-3 and errs[1] < errs[0] / 5, errs


def test_l2p_gradient_is_the_derivative_of_the_potential():
    # central differences of phi in each coordinate of one particle (phi is a
    # polynomial in the position for fixed L)
    rng = np.random.default_rng(9)
    pos, _ = synth.subgrid_particles(23)
    L = rng.standard_normal((20, 8, 8, 8))
    ev = O.l2p(L, pos, 3, 1.0)
    cell = 9 + 24 * 10 + 576 * 11
    t = 1 + 8 * 2 + 64 * 3
    eps = 1e-5
    for ax in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[cell, 0, ax] += eps
        pm[cell, 0, ax] -= eps
        fd = (O.l2p(L, pp, 3, 1.0)[0, t, 0] - O.l2p(L, pm, 3, 1.0)[0, t, 0]) / (2 * eps)
        assert abs(fd - ev[1 + ax, t, 0]) <= 1e-7 * (abs(ev[1 + ax, t, 0]) + 1.0)


def test_evaluation_converges_to_the_direct_sum():
    # near field + L2P of the M2L local expansion against brute force over every
    # particle with |d| <= 6: the error falls with p
    pos, mass = synth.subgrid_particles(0)
    tcells = [(0, 0, 0), (3, 4, 5), (7, 7, 7)]
    ex = _exact_same_level(pos, mass, 1.0, tcells)
    worst = {}
    for p in (2, 4):
        E = O.evaluate(pos, mass, p, 1.0)
        ep, eg = 0.0, 0.0
        for k, (x, y, z) in enumerate(tcells):
            t = x + 8 * y + 64 * z
            ep = max(ep, np.max(np.abs(E[0, t] - ex[k][0]) / ex[k][0]))
            eg = max(eg, np.max(np.abs(E[1:, t].T - ex[k][1]).max(axis=1) / np.abs(ex[k][1]).max(axis=1)))
        worst[p] = (ep, eg)
    assert worst[4][0] < 3e-5 and worst[4][0] < worst[2][0] / 5, worst
    assert worst[4][1] < 0.05 and worst[4][1] < worst[2][1] / 3, worst
