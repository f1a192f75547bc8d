"""Pins of the oracle's tolerance scales from above.

Every GPU parity test bounds |x_gpu - x_oracle| by 1e-12 times a scale the
oracle computes: the same sum as the value, taken over the absolute values
of its terms (m2l_abs, m2l_adjoint_abs, near_field_abs, l2p_abs and the
absolute=True variants of oracle.tree). |x| <= x_abs is a triangle
inequality and is checked elsewhere; an inflated scale would pass that check
and silently loosen every parity test. These tests pin each scale to a value
computed independently of its code:

* inputs with a single non-zero term, where the scale must equal that term
  written out by hand (tables from the exact integer-point derivatives of
  oracle.exact, monomials by hand, the binomial theorem for shifts);
* inputs whose terms are all positive, where the scale must equal the value;
* masked inputs, where the scale must equal that of the zeroed input.

Planted mistakes (a doubled scale, a scale taken before masking, at the
wrong spacing, or over the near offsets as well) each fail at least one pin.
"""
from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np
import pytest

import oracle as O
import oracle.tree as T
import synth
from oracle.exact import dtensor_exact

TOL = 1e-13


@lru_cache(maxsize=None)
def _d_exact(d):
    """D_m(-d) for |m| <= 8 at the integer point -d, correctly rounded."""
    md = tuple(-v for v in d)
    return {m: dtensor_exact(m, md) for m in O.multi_indices(8)}


def _tables_exact(d, p, h):
    """(-1)^|k| D_{k+n}(-d h) for k, n in I_p from the exact integer-point
    derivatives (D_m(-d h) = h^(-1-|m|) D_m(-d), exact for powers of two), and
    the largest |D_m(-d h)| of each order |m|."""
    ks = O.multi_indices(p)
    D = {m: v * h ** (-1 - sum(m)) for m, v in _d_exact(tuple(d)).items() if sum(m) <= 2 * p}
    Tt = np.array([[(-1) ** sum(k) * D[(k[0] + n[0], k[1] + n[1], k[2] + n[2])] for n in ks] for k in ks])
    omax = {}
    for m, v in D.items():
        omax[sum(m)] = max(omax.get(sum(m), 0.0), abs(v))
    return Tt, omax


def _order_scale(omax, p, k):
    return np.array([omax[sum(k) + sum(n)] for n in O.multi_indices(p)])


# ---------------------------------------------------------------------------
# m2l_abs
# ---------------------------------------------------------------------------

def _pin_m2l_single_entry(fn, p, k, src, h, mask, v=-2.5):
    """One moment entry M_k(src) = v: Labs_n(t) = |v| |T_{src-t}[k][n]| for every
    target t with src - t in the shell, zero elsewhere (and zero everywhere if
    src lies in an absent block)."""
    ks = O.multi_indices(p)
    ik = ks.index(k)
    M = np.zeros((len(ks), 24, 24, 24))
    M[ik, src[2], src[1], src[0]] = v
    got = fn(M, p, h, mask)
    present = O.present_cells(mask)[src[2], src[1], src[0]]
    S = set(O.stencil())
    want = np.zeros_like(got)
    bound = np.zeros_like(got)
    for tz, ty, tx in product(range(8), repeat=3):
        d = (src[0] - 8 - tx, src[1] - 8 - ty, src[2] - 8 - tz)
        if present and d in S:
            Tt, omax = _tables_exact(d, p, h)
            want[:, tz, ty, tx] = abs(v) * np.abs(Tt[ik])
            bound[:, tz, ty, tx] = abs(v) * _order_scale(omax, p, k)
    return np.all(got[bound == 0] == 0) and np.all(np.abs(got - want) <= TOL * bound)


def _pin_m2l_masked(fn, p, h, mask, seed=3):
    """Absent blocks count as zero: NaN-poisoned, zeroed and unmasked-zeroed inputs agree."""
    rng = np.random.default_rng(seed)
    C = O.ncomp(p)
    M = rng.standard_normal((C, 24, 24, 24))
    pres = O.present_cells(mask)[None]
    Mz = np.where(pres, M, 0.0)
    Mn = np.where(pres, M, np.nan)
    a = fn(Mn, p, h, mask)
    b = fn(Mz, p, h, O.FULL_MASK)
    return np.array_equal(a, b)


def _pin_m2l_positive_masses(fn):
    """cfg1-like frame, positive masses: Labs_0 >= L_0 and Labs_0 <= 1.1 L_0 (the
    monopole term dominates, |a| / |R| <= 0.39)."""
    pos, mass = synth.subgrid_particles(0)
    M = O.p2m(pos, mass, 3, 1.0)
    L0 = O.m2l(M, 3, 1.0)[0]
    La0 = fn(M, 3, 1.0, O.FULL_MASK)[0]
    return np.all(La0 >= L0 * (1 - 1e-14)) and np.all(La0 <= 1.1 * L0)


def _pin_m2l_monopole_leaves(fn, h=0.5):
    """Particles at the cell centres (the paper's leaf case): only M_0 is non-zero,
    so Labs_n(t) = sum over the shell of M_0(t + d) |D_n(-d h)|, for every n."""
    _, mass = synth.subgrid_particles(7, ppc=2)
    pos = np.repeat(O.cell_centres(h)[:, None, :], 2, axis=1)
    mask = O.FULL_MASK & ~(1 << 14) & ~(1 << 4)
    M = O.p2m(pos, mass, 3, h, mask)
    got = fn(M, 3, h, mask)
    ks = O.multi_indices(3)
    ok = True
    for t in [(0, 0, 0), (7, 3, 5), (4, 7, 1)]:
        want, bound = np.zeros(len(ks)), np.zeros(len(ks))
        for d in O.stencil():
            s = (t[0] + 8 + d[0], t[1] + 8 + d[1], t[2] + 8 + d[2])
            m0 = M[0, s[2], s[1], s[0]]
            if m0 == 0:
                continue
            Tt, omax = _tables_exact(d, 3, h)
            want += m0 * np.abs(Tt[0])
            bound += m0 * _order_scale(omax, 3, (0, 0, 0))
        ok = ok and np.all(np.abs(got[:, t[2], t[1], t[0]] - want) <= TOL * bound)
    return ok


M2L_CASES = [
    (3, (0, 0, 0), (12, 9, 5), 1.0, O.FULL_MASK),
    (3, (2, 0, 1), (17, 3, 20), 0.5, O.FULL_MASK),
    (2, (0, 1, 1), (4, 13, 10), 0.25, O.FULL_MASK & ~(1 << 12)),
    (3, (1, 1, 0), (4, 13, 10), 1.0, O.FULL_MASK & ~(1 << 12)),     # source block absent
]


def _m2l_abs_pins_hold(fn):
    return (all(_pin_m2l_single_entry(fn, *c) for c in M2L_CASES)
            and _pin_m2l_masked(fn, 3, 0.5, O.FULL_MASK & ~(1 << 22) & ~(1 << 0))
            and _pin_m2l_positive_masses(fn) and _pin_m2l_monopole_leaves(fn))


def test_m2l_abs_pins():
    assert _m2l_abs_pins_hold(lambda M, p, h, mask: O.m2l_abs(M, p, h, mask))


M2L_ABS_MUTANTS = {
    "doubled": lambda M, p, h, mask: 2.0 * O.m2l_abs(M, p, h, mask),
    "unmasked": lambda M, p, h, mask: O.m2l_abs(np.nan_to_num(M), p, h, O.FULL_MASK),
    "unit spacing": lambda M, p, h, mask: O.m2l_abs(M, p, 1.0, mask),
    "twice the spacing": lambda M, p, h, mask: O.m2l_abs(M, p, 2.0 * h, mask),
    "near offsets too": lambda M, p, h, mask: O.m2l_abs(M, p, h, mask, O.stencil(1, 36)),
    "only |d|^2 >= 6": lambda M, p, h, mask: O.m2l_abs(M, p, h, mask, O.stencil(6, 36)),
}


@pytest.mark.parametrize("name", sorted(M2L_ABS_MUTANTS))
def test_m2l_abs_pins_catch_planted_mistakes(name):
    assert not _m2l_abs_pins_hold(M2L_ABS_MUTANTS[name]), name


# ---------------------------------------------------------------------------
# m2l_adjoint_abs
# ---------------------------------------------------------------------------

def _pin_adjoint_single_entry(fn, p, n, tgt, h, mask, v=-1.75):
    """One entry W_n(tgt) = v: Gabs_k(s) = |v| |T_{s-tgt}[k][n]| for every frame cell s
    with s - tgt in the shell and s in a present block, zero elsewhere."""
    ks = O.multi_indices(p)
    jn = ks.index(n)
    W = np.zeros((len(ks), 8, 8, 8))
    W[jn, tgt[2], tgt[1], tgt[0]] = v
    got = fn(W, p, h, mask)
    pres = O.present_cells(mask)
    want = np.zeros_like(got)
    bound = np.zeros_like(got)
    for d in O.stencil():
        s = (tgt[0] + 8 + d[0], tgt[1] + 8 + d[1], tgt[2] + 8 + d[2])
        if not pres[s[2], s[1], s[0]]:
            continue
        Tt, omax = _tables_exact(d, p, h)
        want[:, s[2], s[1], s[0]] = abs(v) * np.abs(Tt[:, jn])
        bound[:, s[2], s[1], s[0]] = abs(v) * np.array([omax[sum(k) + sum(n)] for k in ks])
    return np.all(got[bound == 0] == 0) and np.all(np.abs(got - want) <= TOL * bound)


def _pin_adjoint_pairing(fn, p=3, h=0.5, mask=O.FULL_MASK & ~(1 << 25)):
    """<|W|, m2l_abs(|M|)> = <m2l_adjoint_abs(|W|), |M|>: both are the sum of
    |W_n(t)| |M_k(t + d)| |T_d[k][n]| over every (t, d, k, n)."""
    rng = np.random.default_rng(9)
    C = O.ncomp(p)
    M = np.where(O.present_cells(mask)[None], rng.standard_normal((C, 24, 24, 24)), 0.0)
    W = rng.standard_normal((C, 8, 8, 8))
    lhs = np.sum(np.abs(W) * O.m2l_abs(M, p, h, mask))
    rhs = np.sum(fn(W, p, h, mask) * np.abs(M))
    return abs(lhs - rhs) <= 1e-13 * lhs


ADJ_CASES = [
    (3, (0, 0, 0), (3, 4, 5), 1.0, O.FULL_MASK),
    (3, (1, 0, 2), (0, 7, 7), 0.5, O.FULL_MASK & ~(1 << 15) & ~(1 << 24)),
    (2, (2, 0, 0), (7, 0, 2), 0.25, O.FULL_MASK),
]


def _adjoint_abs_pins_hold(fn):
    return all(_pin_adjoint_single_entry(fn, *c) for c in ADJ_CASES) and _pin_adjoint_pairing(fn)


def test_m2l_adjoint_abs_pins():
    assert _adjoint_abs_pins_hold(lambda W, p, h, mask: O.m2l_adjoint_abs(W, p, h, mask))


ADJ_ABS_MUTANTS = {
    "doubled": lambda W, p, h, mask: 2.0 * O.m2l_adjoint_abs(W, p, h, mask),
    "unmasked": lambda W, p, h, mask: O.m2l_adjoint_abs(W, p, h, O.FULL_MASK),
    "unit spacing": lambda W, p, h, mask: O.m2l_adjoint_abs(W, p, 1.0, mask),
    "near offsets too": lambda W, p, h, mask: O.m2l_adjoint_abs(W, p, h, mask, O.stencil(1, 36)),
}


@pytest.mark.parametrize("name", sorted(ADJ_ABS_MUTANTS))
def test_m2l_adjoint_abs_pins_catch_planted_mistakes(name):
    assert not _adjoint_abs_pins_hold(ADJ_ABS_MUTANTS[name]), name


# ---------------------------------------------------------------------------
# near_field_abs and l2p_abs
# ---------------------------------------------------------------------------

def _pin_near_positive(fn, h=0.5, mask=O.FULL_MASK & ~(1 << 12)):
    """Positive masses: the potential's scale is the potential itself."""
    pos, mass = synth.subgrid_particles(4, None, h, 2)
    a = fn(pos, mass, h, mask)[0]
    b = O.near_field(pos, mass, h, mask)[0]
    return np.all(np.abs(a - b) <= 1e-14 * b)


def _pin_near_two_sources(fn, h=1.0):
    """Two massive particles, every other particle massless at its cell centre:
    each target particle's scales are sum m_j / r (potential) and sum m_j / r^2
    (every gradient component) over the massive particles j != i in its near
    cells (|d|^2 <= 4), written out by hand."""
    pos = O.cell_centres(h)[:, None, :].copy()
    mass = np.zeros((O.NCELL, 1))
    src = {11 + 24 * 9 + 576 * 12: (np.array([0.1, -0.2, 0.3]), 2.0),     # target cell (3, 1, 4)
           12 + 24 * 10 + 576 * 12: (np.array([-0.25, 0.05, -0.4]), 3.0)}  # its near cell (4, 2, 4)
    for c, (a, m) in src.items():
        pos[c, 0] += a * h
        mass[c, 0] = m
    got = fn(pos, mass, h, O.FULL_MASK)
    want = np.zeros_like(got)
    for t in range(512):
        j = np.array([t % 8 + 8, (t // 8) % 8 + 8, t // 64 + 8])
        ct = j[0] + 24 * j[1] + 576 * j[2]
        for c in src:
            js = np.array([c % 24, (c // 24) % 24, c // 576])
            if c == ct or np.sum((js - j) ** 2) > 4:
                continue
            r = np.linalg.norm(pos[ct, 0] - pos[c, 0])
            want[0, t, 0] += mass[c, 0] / r
            want[1:, t, 0] += mass[c, 0] / r ** 2
    return np.count_nonzero(want[0]) > 20 and np.all(np.abs(got - want) <= 1e-15 * np.max(want))


def _near_abs_pins_hold(fn):
    return _pin_near_positive(fn) and _pin_near_two_sources(fn)


def test_near_field_abs_pins():
    assert _near_abs_pins_hold(lambda pos, mass, h, mask: O.near_field_abs(pos, mass, h, mask))


NEAR_ABS_MUTANTS = {
    "doubled": lambda pos, mass, h, mask: 2.0 * O.near_field_abs(pos, mass, h, mask),
    "unmasked": lambda pos, mass, h, mask: O.near_field_abs(pos, mass, h, O.FULL_MASK),
    "r instead of r^2": lambda pos, mass, h, mask: np.concatenate(
        [O.near_field_abs(pos, mass, h, mask)[:1]] * 4),
}


@pytest.mark.parametrize("name", sorted(NEAR_ABS_MUTANTS))
def test_near_field_abs_pins_catch_planted_mistakes(name):
    assert not _near_abs_pins_hold(NEAR_ABS_MUTANTS[name]), name


def _l2p_abs_by_hand(comps, b):
    """sum_n |v_n| |b|^n / n! and, per axis i, sum_{n_i >= 1} |v_n| |b|^(n - e_i) / (n - e_i)!
    for the components {n: v_n}; b [..., 3]."""
    b = np.abs(b)
    out = np.zeros((4,) + b.shape[:-1])
    for n, v in comps.items():
        nf = factorial(n[0]) * factorial(n[1]) * factorial(n[2])
        out[0] += abs(v) * b[..., 0] ** n[0] * b[..., 1] ** n[1] * b[..., 2] ** n[2] / nf
        for ax in range(3):
            if n[ax] == 0:
                continue
            m = list(n)
            m[ax] -= 1
            mf = factorial(m[0]) * factorial(m[1]) * factorial(m[2])
            out[1 + ax] += abs(v) * b[..., 0] ** m[0] * b[..., 1] ** m[1] * b[..., 2] ** m[2] / mf
    return out


def _pin_l2p_components(fn, p, comps, h):
    """Components {n: v_n} (mixed signs) at every target: the potential's scale is
    sum |v_n| |b|^n / n! and the gradient's along axis i is
    sum_{n_i >= 1} |v_n| |b|^(n - e_i) / (n - e_i)!, b = y - c_t, by hand."""
    ks = O.multi_indices(p)
    L = np.zeros((len(ks), 8, 8, 8))
    for n, v in comps.items():
        L[ks.index(n)] = v
    pos, _ = synth.subgrid_particles(6, None, h, 2)
    got = fn(L, pos, p, h)
    cs = O.cell_centres(h)
    want = np.zeros_like(got)
    for t in range(512):
        cell = (t % 8 + 8) + 24 * ((t // 8) % 8 + 8) + 576 * (t // 64 + 8)
        want[:, t] = _l2p_abs_by_hand(comps, pos[cell] - cs[cell])
    return np.all(np.abs(got - want) <= 1e-14 * np.maximum(want, 1e-300))


L2P_CASES = [(3, {(0, 0, 0): -3.0}, 1.0), (3, {(2, 1, 0): 2.5}, 0.5),
             (3, {(0, 0, 0): 1.5, (1, 0, 0): -2.0, (0, 1, 2): 0.75, (1, 1, 1): -4.0}, 1.0),
             (4, {(1, 1, 1): -3.0, (0, 3, 1): 1.25, (0, 0, 2): -0.5}, 0.25)]


def _l2p_abs_pins_hold(fn):
    return all(_pin_l2p_components(fn, *c) for c in L2P_CASES)


def test_l2p_abs_pins():
    assert _l2p_abs_pins_hold(lambda L, pos, p, h: O.l2p_abs(L, pos, p, h))


L2P_ABS_MUTANTS = {
    "doubled": lambda L, pos, p, h: 2.0 * O.l2p_abs(L, pos, p, h),
    "unit spacing": lambda L, pos, p, h: O.l2p_abs(L, pos, p, 1.0),
    "b from the cell corner": lambda L, pos, p, h: np.abs(O.l2p(np.abs(L), np.abs(pos), p, h)),
}


@pytest.mark.parametrize("name", sorted(L2P_ABS_MUTANTS))
def test_l2p_abs_pins_catch_planted_mistakes(name):
    assert not _l2p_abs_pins_hold(L2P_ABS_MUTANTS[name]), name


# ---------------------------------------------------------------------------
# the multi-level oracle's absolute variants
# ---------------------------------------------------------------------------

def _pin_level_single_entry(fn, p, k, src, n, h, sigma_check=True, v=4.0):
    """One moment entry on a level of n cells per axis: Labs_m(t) = |v| |T_{src-t}[k][m]|
    at that level's spacing for every t with src - t in IL(t), zero elsewhere."""
    ks = O.multi_indices(p)
    ik = ks.index(k)
    M = np.zeros((len(ks), n, n, n))
    M[ik, src[2], src[1], src[0]] = -v
    got = fn(M, p, h)
    want = np.zeros_like(got)
    bound = np.zeros_like(got)
    lists = {sig: set(T.interaction_list(sig)) for sig in product((0, 1), repeat=3)}
    for tz, ty, tx in product(range(n), repeat=3):
        d = (src[0] - tx, src[1] - ty, src[2] - tz)
        if d in lists[(tx & 1, ty & 1, tz & 1)]:
            Tt, omax = _tables_exact(d, p, h)
            want[:, tz, ty, tx] = v * np.abs(Tt[ik])
            bound[:, tz, ty, tx] = v * _order_scale(omax, p, k)
    return np.all(got[bound == 0] == 0) and np.all(np.abs(got - want) <= TOL * bound)


def _pin_upward_single_particle(fn, p=3, n=16, h=0.5):
    """One particle of mass -m at offset a from its finest cell's centre: level l's
    scale at its ancestor is |m| prod_i (|a_i| + sum of the |shifts|_i)^k_i / k_i!
    (the binomial theorem per axis), zero at every other cell."""
    pos = np.repeat(T._centres(n, h)[:, None, :], 1, axis=1).copy()
    mass = np.zeros((n ** 3, 1))
    j = (5, 10, 3)
    cell = j[0] + n * j[1] + n * n * j[2]
    a = np.array([0.3, -0.15, 0.05]) * h
    pos[cell, 0] += a
    mass[cell, 0] = -2.0
    got = fn(pos, mass, p, n, h)
    ks = O.multi_indices(p)
    u = np.abs(a)
    ok = True
    for lvl, Ml in enumerate(got):
        nl = n >> lvl
        J = tuple(x >> lvl for x in j)
        want = np.zeros_like(Ml)
        for ik, k in enumerate(ks):
            kf = factorial(k[0]) * factorial(k[1]) * factorial(k[2])
            want[ik, J[2], J[1], J[0]] = 2.0 * u[0] ** k[0] * u[1] ** k[1] * u[2] ** k[2] / kf
        ok = ok and np.all(np.abs(Ml - want) <= 1e-14 * np.max(want)) and Ml.shape[1] == nl
        # the next level's centre: the shift from the child's centre, added in absolute value
        hc = h * 2 ** lvl
        u = u + 0.5 * hc
    return ok


def _pin_downward_single_entry(fn, p=3, n=16, h=1.0):
    """One entry L_m = v on the coarsest level only: every finer level's scale at the
    descendants is |v| prod_i (sum of the |shifts|_i)^(m_i - q_i) / (m_i - q_i)! for
    q <= m (the binomial theorem per axis), zero elsewhere."""
    ks = O.multi_indices(p)
    levels = T.tree_levels(n)
    Ls = [np.zeros((len(ks), nl, nl, nl)) for nl in levels]
    m = (1, 2, 0)
    J = (2, 1, 3)
    Ls[-1][ks.index(m), J[2], J[1], J[0]] = -5.0
    got = fn(Ls, p, h)
    ok = True
    # walk down one child branch: the descendant (2J + o) with o = (1, 0, 1) per level
    s = np.zeros(3)
    cell = np.array(J)
    for lvl in range(len(levels) - 2, -1, -1):
        hc = h * 2 ** lvl
        cell = 2 * cell + np.array([1, 0, 1])
        s = s + 0.5 * hc
        want = np.zeros(len(ks))
        for iq, q in enumerate(ks):
            if all(q[a] <= m[a] for a in range(3)):
                r = [m[a] - q[a] for a in range(3)]
                want[iq] = 5.0 * np.prod([s[a] ** r[a] / factorial(r[a]) for a in range(3)])
        g = got[lvl][:, cell[2], cell[1], cell[0]]
        ok = ok and np.all(np.abs(g - want) <= 1e-14 * np.max(want))
        # the same level's cells outside the subtree of J are zero
        nl = levels[lvl]
        w = 2 ** (len(levels) - 1 - lvl)
        outside = np.ones((nl, nl, nl), bool)
        outside[J[2] * w:(J[2] + 1) * w, J[1] * w:(J[1] + 1) * w, J[0] * w:(J[0] + 1) * w] = False
        ok = ok and np.all(got[lvl][:, outside] == 0)
    return ok


def _pin_near_grid_positive(fn, n=8, h=0.5):
    pos, mass = synth.grid_particles(3, n, h, 2)
    a = fn(pos, mass, n, h)[0]
    b = T.near_grid(pos, mass, n, h)[0]
    return np.all(np.abs(a - b) <= 1e-14 * b)


def _pin_l2p_grid_components(fn, p=3, n=8, h=0.5):
    """As _pin_l2p_components, on the finest level of a domain."""
    ks = O.multi_indices(p)
    comps = {(1, 0, 2): 7.0, (0, 1, 0): -2.0, (2, 0, 0): -1.5}
    L = np.zeros((len(ks), n, n, n))
    for nn, v in comps.items():
        L[ks.index(nn)] = v
    pos, _ = synth.grid_particles(5, n, h, 2)
    got = fn(L, pos, p, n, h)
    want = _l2p_abs_by_hand(comps, pos - T._centres(n, h)[:, None, :])
    return np.all(np.abs(got - want) <= 1e-14 * np.maximum(want, 1e-300))


def _tree_pins_hold(level_fn, up_fn, down_fn, near_fn, l2p_fn):
    return (_pin_level_single_entry(level_fn, 3, (0, 0, 0), (7, 9, 4), 16, 0.5)
            and _pin_level_single_entry(level_fn, 2, (1, 0, 1), (2, 13, 8), 16, 2.0)
            and _pin_upward_single_particle(up_fn)
            and _pin_downward_single_entry(down_fn)
            and _pin_near_grid_positive(near_fn)
            and _pin_l2p_grid_components(l2p_fn))


TREE_FNS = dict(
    level_fn=lambda M, p, h: T.m2l_level(M, p, h, absolute=True),
    up_fn=lambda pos, mass, p, n, h: T.upward(pos, mass, p, n, h, absolute=True),
    down_fn=lambda Ls, p, h: T.downward(Ls, p, h, absolute=True),
    near_fn=lambda pos, mass, n, h: T.near_grid(pos, mass, n, h, absolute=True),
    l2p_fn=lambda L, pos, p, n, h: T.l2p_grid_abs(L, pos, p, n, h),
)


def test_tree_absolute_variants_pins():
    assert _tree_pins_hold(**TREE_FNS)


TREE_MUTANTS = {
    "level doubled": dict(level_fn=lambda M, p, h: 2.0 * T.m2l_level(M, p, h, absolute=True)),
    "level at the finest spacing": dict(level_fn=lambda M, p, h: T.m2l_level(M, p, 1.0, absolute=True)),
    "level over the union list": dict(
        level_fn=lambda M, p, h: T.m2l_level(M, p, h, top=True, absolute=True)),
    "M2M shift doubled": dict(up_fn=lambda pos, mass, p, n, h: [T.upward(pos, mass, p, n, h, True)[0]] + [
        T.m2m(Ml, p, 2.0 * h * 2 ** i, True) for i, Ml in enumerate(T.upward(pos, mass, p, n, h, True)[:-1])]),
    "L2L without its own level": dict(down_fn=lambda Ls, p, h: [
        2.0 * x for x in T.downward(Ls, p, h, absolute=True)]),
    "near grid doubled": dict(near_fn=lambda pos, mass, n, h: 2.0 * T.near_grid(pos, mass, n, h, absolute=True)),
    "L2P grid at the corner": dict(l2p_fn=lambda L, pos, p, n, h: np.abs(
        T.l2p_grid(np.abs(L), np.abs(pos), p, n, h))),
}


@pytest.mark.parametrize("name", sorted(TREE_MUTANTS))
def test_tree_pins_catch_planted_mistakes(name):
    fns = dict(TREE_FNS)
    fns.update(TREE_MUTANTS[name])
    assert not _tree_pins_hold(**fns), name
