"""Oracle of the multi-level gravity iteration on a uniform octree.

TEST INFRASTRUCTURE ONLY (see the package docstring): slow, plain, float64.

This is the paper's three-step gravity iteration (Sec. VII-C, "Usage of
multiple HPX tasks per Kokkos kernel invocation": a bottom-up traversal,
the cell-to-cell interactions on every level, a top-down traversal) on a
fully refined cubic domain (Sec. IV-C, "Octo-Tiger": the octree's cells
carry multipole moments, leaves act as point masses).

Domain and levels:
  * n^3 finest cells (n a power of two, n >= 8), spacing h; cell j = (x, y, z)
    spans [j h, (j + 1) h) per axis, centre (j + 1/2) h; arrays are [..][z][y][x]
    and particles are pos [n^3][ppc][3], mass [n^3][ppc] with cell index
    x + n y + n^2 z;
  * level l = 0 is the finest; level l has n / 2^l cells per axis of spacing
    2^l h, down to the coarsest level J with 4 cells per axis; the parent of
    cell j at level l is j // 2 at level l + 1.

Steps (the moments, tables and truncation |k|, |n| <= p of the single-level
oracle in fmm.py):
  P2M  on level 0;
  M2M  M_k(J) = sum over the 8 children j of J, sum_{q <= k} M_q(j) s^(k-q) / (k-q)!,
       s = c_j - c_J (moments re-expanded about the parent centre: exact);
  M2L  on every level, L_n(t) = sum_{s in IL(t)} sum_k M_k(s) T_{s-t}[k][n] at that
       level's spacing, with the interaction list
         IL(t) = {s : |s - t|^2 > 4 and |parent(s) - parent(t)|^2 <= 4}
       (cells not near each other whose parents are near), and on the coarsest
       level every cell that is not near; absent cells (outside the domain) add
       nothing. IL depends only on the parity sigma = t mod 2 of the target:
       IL(t) = t + IL_sigma, |IL_sigma| = 231 in the interior;
  L2L  L_n(j) += sum_{m >= n, |m| <= p} L_m(J) s^(m-n) / (m-n)!, s = c_j - c_J
       (the parent's local polynomial re-expanded about the child centre:
       exact), applied from the coarsest level down;
  and at the finest level L2P plus the near field over the cells with
  |d|^2 <= 4 (fmm.l2p, fmm.near_field).
Every pair of finest cells is then accounted for exactly once: directly if
the cells are near, else through M2L on the unique level where their
ancestors are not near but the ancestors' parents are (or on the coarsest
level) -- pinned by enumeration.
"""

from itertools import product
from math import factorial

import numpy as np

from .fmm import _monomials, multi_indices, ncomp, near_stencil, stencil_tensors

PAD = 6


def tree_levels(n):
    """Cells per axis of every level, finest first: n, n/2, ..., 4."""
    if n < 8 or n & (n - 1):
        raise ValueError("n must be a power of two >= 8")
    out = [n]
    while out[-1] > 4:
        out.append(out[-1] // 2)
    return out


def _near(d):
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= 4


def interaction_list(sigma):
    """IL_sigma = {d : |d|^2 > 4, |floor((sigma + d) / 2)|^2 <= 4}, for a target of
    parity sigma (its parent's offset to the source's parent is floor((sigma + d)/2));
    in the order dz, dy, dx ascending."""
    out = []
    for dz, dy, dx in product(range(-6, 7), repeat=3):
        d = (dx, dy, dz)
        if _near(d):
            continue
        D = tuple((s + v) // 2 for s, v in zip(sigma, d))
        if _near(D):
            out.append(d)
    return out


def top_list():
    """Coarsest level (4 cells per axis): every offset that is not near, |d_i| <= 3."""
    return [(dx, dy, dz) for dz, dy, dx in product(range(-3, 4), repeat=3) if not _near((dx, dy, dz))]


def _centres(n, h):
    g = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x, y, z], axis=-1).reshape(n ** 3, 3)


def p2m_grid(pos, mass, p, n, h):
    """M_k(j) = sum_i m_i (y_i - c_j)^k / k! on the finest level; [C, n, n, n]."""
    a = np.asarray(pos, np.float64) - _centres(n, h)[:, None, :]
    mono = _monomials(a, p)                                   # [C, n^3, ppc]
    return np.einsum("cjk,jk->cj", mono, np.asarray(mass, np.float64)).reshape(-1, n, n, n)


def _shift_terms(p):
    """(ik, iq, r) for k, q in I_p with q <= k componentwise, r = k - q."""
    ks = multi_indices(p)
    out = []
    for ik, k in enumerate(ks):
        for iq, q in enumerate(ks):
            if all(q[a] <= k[a] for a in range(3)):
                out.append((ik, iq, (k[0] - q[0], k[1] - q[1], k[2] - q[2])))
    return out


def _pow_fact(s, r):
    return (s[0] ** r[0] * s[1] ** r[1] * s[2] ** r[2]
            / (factorial(r[0]) * factorial(r[1]) * factorial(r[2])))


def m2m(Mc, p, hc, absolute=False):
    """Parent moments from the child level (spacing hc): [C, n/2, n/2, n/2].
    absolute: the same sums of |terms| (the rounding scale)."""
    C, nc = Mc.shape[0], Mc.shape[1]
    Mp = np.zeros((C, nc // 2, nc // 2, nc // 2))
    terms = _shift_terms(p)
    for oz, oy, ox in product((0, 1), repeat=3):
        # child centre (2J + o + 1/2) hc, parent centre (2J + 1) hc
        s = ((ox - 0.5) * hc, (oy - 0.5) * hc, (oz - 0.5) * hc)
        child = Mc[:, oz::2, oy::2, ox::2]
        if absolute:
            s, child = tuple(abs(v) for v in s), np.abs(child)
        for ik, iq, r in terms:
            Mp[ik] += child[iq] * _pow_fact(s, r)
    return Mp


def l2l(Lp, p, hc, absolute=False):
    """Children's share of the parent level's local expansions: [C, 2n, 2n, 2n]
    for child spacing hc (the parent's polynomial re-expanded at each child centre).
    absolute: the same sums of |terms|."""
    C, npar = Lp.shape[0], Lp.shape[1]
    Lc = np.zeros((C, 2 * npar, 2 * npar, 2 * npar))
    terms = _shift_terms(p)             # (m, n, m - n) with n <= m
    for oz, oy, ox in product((0, 1), repeat=3):
        s = ((ox - 0.5) * hc, (oy - 0.5) * hc, (oz - 0.5) * hc)
        src = Lp
        if absolute:
            s, src = tuple(abs(v) for v in s), np.abs(Lp)
        view = Lc[:, oz::2, oy::2, ox::2]
        for im, in_, r in terms:
            view[in_] += src[im] * _pow_fact(s, r)
    return Lc


def m2l_level(M, p, h, top=False, absolute=False):
    """L_n(t) = sum_{d in IL_sigma(t)} sum_k M_k(t + d) T_d[k][n] on one level of
    spacing h (top: the coarsest level's list); sources outside the domain are
    absent. One [C x C] . [C x (n/2)^3] product per (parity, offset).
    absolute: |T| against |M| (the rounding scale)."""
    C, n = M.shape[0], M.shape[1]
    if absolute:
        M = np.abs(M)
    Mp = np.zeros((C, n + 2 * PAD, n + 2 * PAD, n + 2 * PAD))
    Mp[:, PAD:PAD + n, PAD:PAD + n, PAD:PAD + n] = M
    L = np.zeros_like(M)
    for sig in product((0, 1), repeat=3):
        offs = top_list() if top else interaction_list(sig)
        T = stencil_tensors(p, h, offs)
        if absolute:
            T = np.abs(T)
        tgt = L[:, sig[2]::2, sig[1]::2, sig[0]::2]
        for d, Td in zip(offs, T):
            src = Mp[:, PAD + sig[2] + d[2]:PAD + n + d[2]:2,
                     PAD + sig[1] + d[1]:PAD + n + d[1]:2,
                     PAD + sig[0] + d[0]:PAD + n + d[0]:2]
            tgt += np.tensordot(Td.T, src, axes=1)
    return L


def upward(pos, mass, p, n, h, absolute=False):
    """Moments of every level, finest first (absolute: the rounding scales, from
    |y - c| and |m|)."""
    if absolute:
        c = _centres(n, h)[:, None, :]
        pos, mass = c + np.abs(np.asarray(pos, np.float64) - c), np.abs(mass)
    Ms = [p2m_grid(pos, mass, p, n, h)]
    for lvl in range(len(tree_levels(n)) - 1):
        Ms.append(m2m(Ms[-1], p, h * 2 ** lvl, absolute))
    return Ms


def m2l_levels(Ms, p, h, absolute=False):
    """Each level's own M2L (the coarsest with the top list), finest first."""
    J = len(Ms) - 1
    return [m2l_level(M, p, h * 2 ** lvl, top=(lvl == J), absolute=absolute) for lvl, M in enumerate(Ms)]


def downward(Ls, p, h, absolute=False):
    """Totals: L(level) = own M2L + L2L of the parent level's total, coarsest first."""
    out = [None] * len(Ls)
    out[-1] = np.abs(Ls[-1]) if absolute else Ls[-1]
    for lvl in range(len(Ls) - 2, -1, -1):
        own = np.abs(Ls[lvl]) if absolute else Ls[lvl]
        out[lvl] = own + l2l(out[lvl + 1], p, h * 2 ** lvl, absolute)
    return out


def l2p_grid_abs(L0, pos, p, n, h):
    """Rounding scale of l2p_grid: |L| at |b|."""
    c = _centres(n, h)[:, None, :]
    return np.abs(l2p_grid(np.abs(L0), c + np.abs(np.asarray(pos, np.float64) - c), p, n, h))


def l2p_grid(L0, pos, p, n, h):
    """Potential and gradient of the finest-level local expansions at the particles:
    [4, n^3, ppc] (phi, d/dx, d/dy, d/dz), as fmm.l2p for every cell of the domain."""
    ks = multi_indices(p)
    Lf = np.asarray(L0, np.float64).reshape(len(ks), -1)
    b = np.asarray(pos, np.float64) - _centres(n, h)[:, None, :]
    mono = _monomials(b, p)                                   # [C, n^3, ppc]
    out = np.zeros((4,) + b.shape[:2])
    out[0] = np.einsum("cj,cjk->jk", Lf, mono)
    for ax in range(3):
        for c_m, m in enumerate(ks):
            if sum(m) > p - 1:
                continue
            e = [0, 0, 0]
            e[ax] = 1
            out[1 + ax] += Lf[ks.index((m[0] + e[0], m[1] + e[1], m[2] + e[2]))][:, None] * mono[c_m]
    return out


def near_grid(pos, mass, n, h, absolute=False):
    """Direct sums over the near cells (|d|^2 <= 4) inside the domain, the particle
    itself excluded: [4, n^3, ppc]. absolute: the scales sum m/r and sum m/r^2."""
    pos = np.asarray(pos, np.float64).reshape(n, n, n, -1, 3)
    mass = np.asarray(mass, np.float64).reshape(n, n, n, -1)
    ppc = mass.shape[-1]
    P = np.full((n + 4, n + 4, n + 4, ppc, 3), np.nan)
    Mm = np.zeros((n + 4, n + 4, n + 4, ppc))
    P[2:-2, 2:-2, 2:-2] = pos
    Mm[2:-2, 2:-2, 2:-2] = mass
    out = np.zeros((4, n, n, n, ppc))
    for d in near_stencil():
        sl = (slice(2 + d[2], 2 + d[2] + n), slice(2 + d[1], 2 + d[1] + n), slice(2 + d[0], 2 + d[0] + n))
        ys, ms = P[sl], Mm[sl]                                # [n, n, n, ppc_s, 3]
        dy = pos[:, :, :, :, None, :] - ys[:, :, :, None, :, :]
        r = np.sqrt(np.sum(dy * dy, axis=-1))                 # [n, n, n, ppc, ppc_s]
        mj = np.broadcast_to(ms[:, :, :, None, :], r.shape).copy()
        outside = np.isnan(r)
        mj[outside] = 0.0
        r[outside] = 1.0
        dy[outside] = 0.0
        if d == (0, 0, 0):
            i = np.arange(ppc)
            mj[..., i, i] = 0.0
            r[..., i, i] = 1.0
        if absolute:
            out[0] += np.sum(mj / r, axis=-1)
            out[1:] += np.sum(mj / r ** 2, axis=-1)[None]
        else:
            out[0] += np.sum(mj / r, axis=-1)
            out[1:] -= np.moveaxis(np.einsum("...ij,...ijk->...ik", mj / r ** 3, dy), -1, 0)
    return out.reshape(4, n ** 3, ppc)


def solve(pos, mass, p, n, h):
    """The whole iteration: potential and gradient at every particle, [4, n^3, ppc]."""
    Ms = upward(pos, mass, p, n, h)
    Lt = downward(m2l_levels(Ms, p, h), p, h)
    return l2p_grid(Lt[0], pos, p, n, h) + near_grid(pos, mass, n, h)


def direct_all(pos, mass):
    """Brute force over every pair of particles: phi_i = sum_{j != i} m_j / r_ij and
    its gradient at y_i; [4, N] for N particles (any shape [..., 3] / [...])."""
    Y = np.asarray(pos, np.float64).reshape(-1, 3)
    m = np.asarray(mass, np.float64).reshape(-1)
    N = len(m)
    out = np.zeros((4, N))
    for i0 in range(0, N, 512):
        yi = Y[i0:i0 + 512]
        dy = yi[:, None, :] - Y[None, :, :]
        r = np.sqrt(np.sum(dy * dy, axis=-1))
        idx = np.arange(i0, min(i0 + 512, N))
        r[idx - i0, idx] = np.inf
        out[0, i0:i0 + 512] = np.sum(m[None, :] / r, axis=1)
        out[1:, i0:i0 + 512] = -np.einsum("ij,ijk->ki", m[None, :] / r ** 3, dy)
    return out


# ---------------------------------------------------------------------------
# one finest cell at a time (for sampled checks of large domains)
# ---------------------------------------------------------------------------

def shift_local(Lv, p, s, absolute=False):
    """A local polynomial (coefficients Lv [C]) re-expanded about a point moved by
    s: L'_n = sum_{m >= n} L_m s^(m-n) / (m-n)! (exact for degree p)."""
    out = np.zeros_like(np.asarray(Lv, np.float64))
    if absolute:
        Lv, s = np.abs(Lv), tuple(abs(v) for v in s)
    for im, in_, r in _shift_terms(p):
        out[in_] += Lv[im] * _pow_fact(s, r)
    return out


def local_at(pos, mass, p, n, h, t, absolute=False):
    """The finest-level total local expansion of cell t = (x, y, z), from the
    definitions directly: on every level l, the interaction-list sum of the
    ancestor A = t >> l, with each source cell's moments taken about its centre
    from all the particles it contains (what P2M and M2M give, exactly), then
    the polynomial moved from A's centre to t's (what the chain of L2L gives,
    exactly). absolute: the same sums over absolute values."""
    levels = tree_levels(n)
    J = len(levels) - 1
    ppc = np.asarray(mass).shape[-1]
    P = np.asarray(pos, np.float64).reshape(n, n, n, ppc, 3)
    W = np.asarray(mass, np.float64).reshape(n, n, n, ppc)
    t = np.asarray(t)
    C = ncomp(p)
    total = np.zeros(C)
    for lvl, nl in enumerate(levels):
        w = 2 ** lvl
        hl = h * w
        A = t >> lvl
        offs = top_list() if lvl == J else interaction_list(tuple(int(v) for v in A & 1))
        Ts = stencil_tensors(p, hl, offs)
        if absolute:
            Ts = np.abs(Ts)
        Lv = np.zeros(C)
        for d, Td in zip(offs, Ts):
            s = A + np.array(d)
            if np.any(s < 0) or np.any(s >= nl):
                continue
            blk = (slice(s[2] * w, (s[2] + 1) * w), slice(s[1] * w, (s[1] + 1) * w), slice(s[0] * w, (s[0] + 1) * w))
            a = P[blk].reshape(-1, 3) - (s + 0.5) * hl
            m = W[blk].reshape(-1)
            if absolute:
                a, m = np.abs(a), np.abs(m)
            Lv += Td.T @ (_monomials(a, p) @ m)
        total += shift_local(Lv, p, tuple((t + 0.5) * h - (A + 0.5) * hl), absolute)
    return total


def evaluate_at(pos, mass, p, n, h, t, absolute=False):
    """Potential and gradient at the particles of finest cell t: L2P of local_at
    plus the near field over the cells t + d, |d|^2 <= 4, inside the domain
    (particle itself excluded); [4, ppc]. absolute: the rounding scales."""
    ppc = np.asarray(mass).shape[-1]
    P = np.asarray(pos, np.float64).reshape(n, n, n, ppc, 3)
    W = np.asarray(mass, np.float64).reshape(n, n, n, ppc)
    t = np.asarray(t)
    ks = multi_indices(p)
    Lv = local_at(pos, mass, p, n, h, t, absolute)
    b = P[t[2], t[1], t[0]] - (t + 0.5) * h                  # [ppc, 3]
    if absolute:
        b = np.abs(b)
    mono = _monomials(b, p)
    out = np.zeros((4, ppc))
    out[0] = Lv @ mono
    for ax in range(3):
        for c_m, m in enumerate(ks):
            if sum(m) > p - 1:
                continue
            e = [0, 0, 0]
            e[ax] = 1
            out[1 + ax] += Lv[ks.index((m[0] + e[0], m[1] + e[1], m[2] + e[2]))] * mono[c_m]
    y = P[t[2], t[1], t[0]]
    for d in near_stencil():
        s = t + np.array(d)
        if np.any(s < 0) or np.any(s >= n):
            continue
        ys, ms = P[s[2], s[1], s[0]], W[s[2], s[1], s[0]]
        dy = y[:, None, :] - ys[None, :, :]
        r = np.sqrt(np.sum(dy * dy, axis=-1))
        mj = np.broadcast_to(ms[None, :], r.shape).copy()
        if d == (0, 0, 0):
            np.fill_diagonal(mj, 0.0)
            np.fill_diagonal(r, 1.0)
        if absolute:
            out[0] += np.sum(mj / r, axis=1)
            out[1:] += np.sum(mj / r ** 2, axis=1)[None]
        else:
            out[0] += np.sum(mj / r, axis=1)
            out[1:] -= np.einsum("ij,ijk->ki", mj / r ** 3, dy)
    return out
