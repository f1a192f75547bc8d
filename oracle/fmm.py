"""Oracle definitions: P2M, derivative tensors of 1/r, M2L, their adjoints.

TEST INFRASTRUCTURE ONLY (see the package docstring): slow, plain, float64.

Geometry (one sub-grid, the paper's N = 8 sub-grid of Sec. IV-C "Octo-Tiger"):
  * a frame of 24^3 cells j = (x, y, z), x fastest, linear index x + 24 y + 576 z:
    the 8^3 target sub-grid in the middle plus its 26 same-level neighbours;
  * cell j spans [j h, (j + 1) h) per axis, centre c_j = (j + 1/2) h;
  * neighbour block beta(j) = j // 8 in {0,1,2}^3, mask bit bx + 3 by + 9 bz,
    the centre block is bit 13 and is always present;
  * targets are the cells of the centre block, t = j - 8 in [0, 8)^3.

Multi-indices k = (kx, ky, kz), |k| = kx + ky + kz, k! = kx! ky! kz!.
I_p = {k : |k| <= p} in graded order (order 0, then x, y, z, then
xx, xy, xz, yy, yz, zz, ...), C(p) = |I_p|.

Definitions (Cartesian Taylor expansion of 1/|x - y| in both arguments):
  M_k(j)  = sum_i m_i a_i^k / k!,  a_i = y_i - c_j                        (P2M)
  D_m(R)  = d^m (1/|r|) at r = R                                          (Hobson)
  T_d[k][n] = (-1)^|k| D_{k+n}(R_d),  R_d = c_target - c_source = -d h
  L_n(t)  = sum_{d in S, beta(t+d) present} sum_k M_k(t + d) T_d[k][n]    (M2L)
so that Phi(c_t + b) ~ sum_n L_n b^n / n! with Phi(x) = sum m / |x - y|.
"""

from math import factorial

import numpy as np

FRAME = 24
BLOCK = 8
NCELL = FRAME ** 3
CENTRE_BIT = 13
FULL_MASK = (1 << 27) - 1


# ---------------------------------------------------------------------------
# index sets, stencil, frame
# ---------------------------------------------------------------------------

def multi_indices(p):
    """I_p in graded order: for n = 0..p, kx = n..0, ky = n-kx..0, kz = rest."""
    out = []
    for n in range(p + 1):
        for kx in range(n, -1, -1):
            for ky in range(n - kx, -1, -1):
                out.append((kx, ky, n - kx - ky))
    return out


def ncomp(p):
    """C(p) = (p+1)(p+2)(p+3)/6, the number of multi-indices with |k| <= p."""
    return (p + 1) * (p + 2) * (p + 3) // 6


def stencil(rmin2=5, rmax2=36):
    """Same-level interaction stencil S = {d in Z^3 : rmin2 <= |d|^2 <= rmax2}.

    The default is the spherical shell 2 < |d| <= 6 (|S| = 892), listed with
    dz slowest, then dy, then dx. d is the source cell minus the target cell.
    """
    r = int(np.floor(np.sqrt(rmax2)))
    out = []
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                q = dx * dx + dy * dy + dz * dz
                if rmin2 <= q <= rmax2:
                    out.append((dx, dy, dz))
    return out


def double_factorial(n):
    """n!! with (-1)!! = 0!! = 1."""
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


def cell_centres(h):
    """Centres (j + 1/2) h of the 24^3 frame cells, shape [13824, 3] (x, y, z)."""
    idx = np.arange(NCELL)
    j = np.stack([idx % FRAME, (idx // FRAME) % FRAME, idx // (FRAME * FRAME)], axis=1)
    return (j + 0.5) * h


def present_cells(mask):
    """Boolean [24, 24, 24] ([z][y][x]) of cells whose neighbour block is present."""
    b = np.arange(FRAME) // BLOCK
    bz, by, bx = np.meshgrid(b, b, b, indexing="ij")
    bit = bx + 3 * by + 9 * bz
    return ((int(mask) >> bit) & 1).astype(bool)


def _monomials(a, p, with_factorial=True):
    """a^k (/ k!) for all k in I_p; a has shape [..., 3]; returns [C, ...]."""
    ks = multi_indices(p)
    out = np.empty((len(ks),) + a.shape[:-1])
    for c, (kx, ky, kz) in enumerate(ks):
        v = a[..., 0] ** kx * a[..., 1] ** ky * a[..., 2] ** kz
        if with_factorial:
            v = v / (factorial(kx) * factorial(ky) * factorial(kz))
        out[c] = v
    return out


# ---------------------------------------------------------------------------
# derivatives of 1/r (Hobson's closed form)
# ---------------------------------------------------------------------------

def _hobson_term_coeff(a, i):
    """a! / (2^i i! (a - 2i)!)."""
    return factorial(a) // (2 ** i * factorial(i) * factorial(a - 2 * i))


def dtensor(m, R):
    """D_m(R) = d^m (1/|r|) at r = R, for one multi-index m; R has shape [..., 3].

    Hobson's formula: with n = |m| = a + b + c and s = i + j + l,
      D_m = sum_{i<=a/2, j<=b/2, l<=c/2} (-1)^(n-s) (2n-2s-1)!!
            [a!/(2^i i!(a-2i)!)] [b!/(2^j j!(b-2j)!)] [c!/(2^l l!(c-2l)!)]
            x^(a-2i) y^(b-2j) z^(c-2l) / r^(2n-2s+1).
    """
    a, b, c = m
    n = a + b + c
    R = np.asarray(R, dtype=np.float64)
    x, y, z = R[..., 0], R[..., 1], R[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    out = np.zeros(R.shape[:-1])
    for i in range(a // 2 + 1):
        for j in range(b // 2 + 1):
            for l in range(c // 2 + 1):
                s = i + j + l
                coeff = ((-1) ** (n - s)) * double_factorial(2 * n - 2 * s - 1) \
                    * _hobson_term_coeff(a, i) * _hobson_term_coeff(b, j) * _hobson_term_coeff(c, l)
                out = out + float(coeff) * (x ** (a - 2 * i)) * (y ** (b - 2 * j)) * (z ** (c - 2 * l)) \
                    / r ** (2 * n - 2 * s + 1)
    return out


def dtensor_all(order, R):
    """{m: D_m(R)} for every multi-index with |m| <= order."""
    return {m: dtensor(m, R) for m in multi_indices(order)}


def stencil_tensors(p, h, offsets=None):
    """T_d[k][n] = (-1)^|k| D_{k+n}(-d h) for d in offsets; shape [|S|, C, C].

    D is evaluated directly at R = -d h (no power-of-two rescaling here).
    """
    offsets = stencil() if offsets is None else offsets
    ks = multi_indices(p)
    R = -np.asarray(offsets, dtype=np.float64) * h
    D = dtensor_all(2 * p, R)
    C = len(ks)
    T = np.empty((len(offsets), C, C))
    for ik, k in enumerate(ks):
        sign = -1.0 if sum(k) % 2 else 1.0
        for jn, n in enumerate(ks):
            T[:, ik, jn] = sign * D[(k[0] + n[0], k[1] + n[1], k[2] + n[2])]
    return T


# ---------------------------------------------------------------------------
# P2M and its adjoint
# ---------------------------------------------------------------------------

def p2m(pos, mass, p, h, mask=FULL_MASK):
    """Cell moments M_k(j) = sum_i m_i a_i^k / k! about the cell centres.

    pos [13824, ppc, 3] absolute frame coordinates, mass [13824, ppc];
    returns M [C, 24, 24, 24] ([k][z][y][x]); cells of absent blocks are 0.
    The leaf case of the paper (a cell's mass as one monopole at its centre)
    is the special case a_i = 0.
    """
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    a = pos - cell_centres(h)[:, None, :]
    mono = _monomials(a, p)                       # [C, 13824, ppc]
    M = np.einsum("cji,ji->cj", mono, mass)        # sum over particles
    M = M.reshape(-1, FRAME, FRAME, FRAME)
    return np.where(present_cells(mask)[None], M, 0.0)


def p2m_adjoint(pos, G, p, h, mask=FULL_MASK):
    """dLoss/dm_i = sum_k G_k(j) a_i^k / k!; zero for particles in absent blocks.

    pos [13824, ppc, 3], G [C, 24, 24, 24]; returns [13824, ppc].
    """
    pos = np.asarray(pos, dtype=np.float64)
    a = pos - cell_centres(h)[:, None, :]
    mono = _monomials(a, p)                       # [C, 13824, ppc]
    Gc = np.asarray(G, dtype=np.float64).reshape(-1, NCELL)
    g = np.einsum("cji,cj->ji", mono, Gc)
    return np.where(present_cells(mask).reshape(NCELL)[:, None], g, 0.0)


# ---------------------------------------------------------------------------
# M2L, its absolute-value bound and its adjoint
# ---------------------------------------------------------------------------

def _source_window(src, d):
    dx, dy, dz = d
    lo = BLOCK
    return src[:, lo + dz:lo + BLOCK + dz, lo + dy:lo + BLOCK + dy, lo + dx:lo + BLOCK + dx]


def _masked(M, mask):
    # absent blocks are treated as zero moments and their storage is never used
    return np.where(present_cells(mask)[None], np.asarray(M, dtype=np.float64), 0.0)


def m2l(M, p, h, mask=FULL_MASK, offsets=None):
    """L_n(t) = sum_{d in S} sum_k M_k(t + d) T_d[k][n] for the 512 targets.

    One [512 x C] . [C x C] product per stencil offset. M [C, 24, 24, 24];
    returns L [C, 8, 8, 8].
    """
    offsets = stencil() if offsets is None else offsets
    C = ncomp(p)
    src = _masked(M, mask)
    T = stencil_tensors(p, h, offsets)
    L = np.zeros((C, BLOCK ** 3))
    for d, Td in zip(offsets, T):
        L += Td.T @ _source_window(src, d).reshape(C, -1)
    return L.reshape(C, BLOCK, BLOCK, BLOCK)


def m2l_abs(M, p, h, mask=FULL_MASK, offsets=None):
    """Labs_n(t) = sum_d sum_k |M_k(t + d)| |T_d[k][n]|: the scale of the rounding
    error of any summation order of L, used as the tolerance scale."""
    offsets = stencil() if offsets is None else offsets
    C = ncomp(p)
    src = np.abs(_masked(M, mask))
    T = np.abs(stencil_tensors(p, h, offsets))
    L = np.zeros((C, BLOCK ** 3))
    for d, Td in zip(offsets, T):
        L += Td.T @ _source_window(src, d).reshape(C, -1)
    return L.reshape(C, BLOCK, BLOCK, BLOCK)


def m2l_adjoint(W, p, h, mask=FULL_MASK, offsets=None):
    """G_k(s) = sum_{d : s - d in target block} sum_n W_n(s - d) T_d[k][n].

    The transpose of m2l with respect to M, written out directly (each
    offset scatters T_d W into the shifted window), so that T_{-d} = T_d^T
    is a property to test rather than an assumption. W [C, 8, 8, 8];
    returns G [C, 24, 24, 24], zero outside the reachable window and on
    absent blocks.
    """
    offsets = stencil() if offsets is None else offsets
    C = ncomp(p)
    Wf = np.asarray(W, dtype=np.float64).reshape(C, -1)
    T = stencil_tensors(p, h, offsets)
    G = np.zeros((C, FRAME, FRAME, FRAME))
    for d, Td in zip(offsets, T):
        _source_window(G, d)[...] += (Td @ Wf).reshape(C, BLOCK, BLOCK, BLOCK)
    return np.where(present_cells(mask)[None], G, 0.0)


def m2l_adjoint_abs(W, p, h, mask=FULL_MASK, offsets=None):
    """Gabs: m2l_adjoint on |W| and |T|, the tolerance scale of G."""
    offsets = stencil() if offsets is None else offsets
    C = ncomp(p)
    Wf = np.abs(np.asarray(W, dtype=np.float64)).reshape(C, -1)
    T = np.abs(stencil_tensors(p, h, offsets))
    G = np.zeros((C, FRAME, FRAME, FRAME))
    for d, Td in zip(offsets, T):
        _source_window(G, d)[...] += (Td @ Wf).reshape(C, BLOCK, BLOCK, BLOCK)
    return np.where(present_cells(mask)[None], G, 0.0)


def pair_count(mask, offsets=None):
    """Number of (target cell, offset) pairs whose source block is present."""
    offsets = stencil() if offsets is None else offsets
    pres = present_cells(mask)
    return int(sum(_source_window(pres[None], d).sum() for d in offsets))


# ---------------------------------------------------------------------------
# direct Newtonian sum (small inputs only)
# ---------------------------------------------------------------------------

def direct_sum(pos, mass, h, order, mask=FULL_MASK, offsets=None, targets=None):
    """Exact derivatives of Phi(x) = sum m_i / |x - y_i| at target centres.

    Sources: the particles of the cells t + d, d in offsets, in present
    blocks. L^exact_n(t) = sum m_i D_n(c_t - y_i) for |n| <= order.
    targets: list of (tx, ty, tz) in [0, 8)^3 (default: all 512).
    Returns [len(targets), C(order)].
    """
    offsets = stencil() if offsets is None else offsets
    if targets is None:
        targets = [(x, y, z) for z in range(BLOCK) for y in range(BLOCK) for x in range(BLOCK)]
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    pres = present_cells(mask)
    ns = multi_indices(order)
    out = np.zeros((len(targets), len(ns)))
    for it, t in enumerate(targets):
        jt = np.array(t) + BLOCK
        ct = (jt + 0.5) * h
        ys, ms = [], []
        for d in offsets:
            js = jt + np.array(d)
            if not pres[js[2], js[1], js[0]]:
                continue
            cell = js[0] + FRAME * js[1] + FRAME * FRAME * js[2]
            ys.append(pos[cell])
            ms.append(mass[cell])
        if not ys:
            continue
        Y = np.concatenate(ys)
        Mm = np.concatenate(ms)
        R = ct[None, :] - Y
        for c, n in enumerate(ns):
            out[it, c] = np.sum(Mm * dtensor(n, R))
    return out


# ---------------------------------------------------------------------------
# evaluation at the target particles: near field and L2P
# ---------------------------------------------------------------------------

def near_stencil():
    """N = {d in Z^3 : |d|^2 <= 4}, 33 offsets including d = 0: the cells whose
    particles are summed directly. With the M2L shell S (5 <= |d|^2 <= 36) it
    covers every same-level cell with |d| <= 6."""
    return stencil(0, 4)


def _target_cells():
    """Frame indices j of the 512 target cells, in target order (x fastest)."""
    return [(x + BLOCK, y + BLOCK, z + BLOCK)
            for z in range(BLOCK) for y in range(BLOCK) for x in range(BLOCK)]


def l2p(L, pos, p, h):
    """Far-field potential and gradient at the target block's particles.

    phi(y) = sum_n L_n(t) b^n / n! and d phi / d y_i = sum_{|m| <= p-1} L_{m + e_i}(t) b^m / m!,
    b = y - c_t (the Taylor polynomial of the local expansion and its gradient).
    L [C, 8, 8, 8]; pos [13824, ppc, 3]. Returns [4, 512, ppc]: phi, gx, gy, gz.
    """
    ks = multi_indices(p)
    pos = np.asarray(pos, dtype=np.float64)
    Lf = np.asarray(L, dtype=np.float64).reshape(len(ks), -1)
    ppc = pos.shape[1]
    out = np.zeros((4, BLOCK ** 3, ppc))
    for t, j in enumerate(_target_cells()):
        cell = j[0] + FRAME * j[1] + FRAME * FRAME * j[2]
        c = (np.array(j) + 0.5) * h
        b = pos[cell] - c[None, :]                      # [ppc, 3]
        mono = _monomials(b, p)                         # [C, ppc], b^n / n!
        out[0, t] = Lf[:, t] @ mono
        for ax in range(3):
            e = [0, 0, 0]
            e[ax] = 1
            for c_m, m in enumerate(ks):
                if sum(m) > p - 1:
                    continue
                n = (m[0] + e[0], m[1] + e[1], m[2] + e[2])
                out[1 + ax, t] += Lf[ks.index(n), t] * mono[c_m]
    return out


def _near_pairs(pos, mass, h, mask, fn):
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    pres = present_cells(mask)
    ppc = pos.shape[1]
    out = np.zeros((4, BLOCK ** 3, ppc))
    for t, j in enumerate(_target_cells()):
        ct = j[0] + FRAME * j[1] + FRAME * FRAME * j[2]
        yi = pos[ct]                                    # [ppc, 3]
        for d in near_stencil():
            js = (j[0] + d[0], j[1] + d[1], j[2] + d[2])
            if not pres[js[2], js[1], js[0]]:
                continue
            cs = js[0] + FRAME * js[1] + FRAME * FRAME * js[2]
            dy = yi[:, None, :] - pos[cs][None, :, :]    # [ppc, ppc_src, 3], y_i - y_j
            r = np.sqrt(np.sum(dy * dy, axis=-1))
            mj = np.broadcast_to(mass[cs][None, :], r.shape).copy()
            if d == (0, 0, 0):
                np.fill_diagonal(mj, 0.0)               # no self-interaction
                np.fill_diagonal(r, 1.0)
            fn(out, t, mj, r, dy)
    return out


def near_field(pos, mass, h, mask=FULL_MASK):
    """Direct sums over the near cells for the target block's particles:
    phi_i = sum_{j != i} m_j / |y_i - y_j| and grad_i = -sum_{j != i} m_j (y_i - y_j) / |y_i - y_j|^3,
    over the particles j of the cells cell(i) + d, d in N, in present blocks.
    Returns [4, 512, ppc]: phi, gx, gy, gz."""
    def acc(out, t, mj, r, dy):
        out[0, t] += np.sum(mj / r, axis=1)
        out[1:, t] -= np.einsum("ij,ijk->ki", mj / r ** 3, dy)
    return _near_pairs(pos, mass, h, mask, acc)


def near_field_abs(pos, mass, h, mask=FULL_MASK):
    """Scales of the rounding of near_field: sum m/r for phi and sum m/r^2 for
    every gradient component (masses are positive)."""
    def acc(out, t, mj, r, dy):
        out[0, t] += np.sum(mj / r, axis=1)
        out[1:, t] += np.sum(mj / r ** 2, axis=1)[None, :]
    return _near_pairs(pos, mass, h, mask, acc)


def l2p_abs(L, pos, p, h):
    """Scales of the rounding of l2p: l2p with |L| and |b|."""
    cs = cell_centres(h).reshape(FRAME ** 3, 1, 3)
    posa = cs + np.abs(np.asarray(pos, dtype=np.float64) - cs)
    return np.abs(l2p(np.abs(L), posa, p, h))


def evaluate(pos, mass, p, h, mask=FULL_MASK, L=None):
    """Same-level potential and gradient at the target block's particles: the
    far part from the local expansion L (computed with m2l when not given)
    plus the near field. Returns [4, 512, ppc]."""
    if L is None:
        L = m2l(p2m(pos, mass, p, h, mask), p, h, mask)
    return l2p(L, pos, p, h) + near_field(pos, mass, h, mask)


# ---------------------------------------------------------------------------
# harmonic (traceless) form of M2L
# ---------------------------------------------------------------------------

def harmonic_indices(p):
    """K'_p = {k in I_p : k_z <= 1}, in the graded order of I_p: the (p+1)^2
    multi-indices that carry the independent components of a tensor family
    that is harmonic in its index (sum_i T[k + 2 e_i] = 0)."""
    return [k for k in multi_indices(p) if k[2] <= 1]


def harmonic_fold(p):
    """F [C, C'] with T[k] = sum_{k'} F[k, k'] T[k'] for every k in I_p and every
    family T that is harmonic in k.

    For k_z >= 2, harmonicity at k - 2 e_z gives
    T[(a, b, c)] = -T[(a+2, b, c-2)] - T[(a, b+2, c-2)]; applying it until the
    z-index is 0 or 1 expresses every T[k] through K'_p with integer
    coefficients (rows of k in K'_p are unit rows).
    """
    ks = multi_indices(p)
    hs = harmonic_indices(p)
    col = {k: i for i, k in enumerate(hs)}
    F = np.zeros((len(ks), len(hs)))

    def expand(row, k, coef):
        a, b, c = k
        if c <= 1:
            F[row, col[k]] += coef
            return
        expand(row, (a + 2, b, c - 2), -coef)
        expand(row, (a, b + 2, c - 2), -coef)

    for row, k in enumerate(ks):
        expand(row, k, 1.0)
    return F


def m2l_harmonic(M, p, h, mask=FULL_MASK, offsets=None):
    """The M2L of m2l() computed in the harmonic form.

    T_d[k][n] = (-1)^|k| D_{k+n}(R_d) is harmonic in k and in n, because 1/r is
    harmonic away from the origin. So with F = harmonic_fold(p):
      * sum_k M_k T_d[k][n] = sum_{k'} Mh_{k'} T_d[k'][n], with Mh = F^T M
        (the folded moments, C' = (p+1)^2 per cell);
      * L is harmonic in n, so only the C' columns n' in K'_p are contracted
        and L_n = sum_{n'} F[n, n'] L_{n'}.
    Per offset this is one [512 x C'] . [C' x C'] product with the dense table
    restricted to K'_p x K'_p. The result equals m2l() up to rounding.
    """
    offsets = stencil() if offsets is None else offsets
    ks = multi_indices(p)
    hs = harmonic_indices(p)
    hidx = [ks.index(k) for k in hs]
    Cp = len(hs)
    F = harmonic_fold(p)
    src = _masked(M, mask)
    Mh = np.tensordot(F.T, src, axes=(1, 0))                 # [C', 24, 24, 24]
    T = stencil_tensors(p, h, offsets)[:, hidx][:, :, hidx]  # [S, C', C']
    Lh = np.zeros((Cp, BLOCK ** 3))
    for d, Td in zip(offsets, T):
        Lh += Td.T @ _source_window(Mh, d).reshape(Cp, -1)
    L = F @ Lh
    return L.reshape(len(ks), BLOCK, BLOCK, BLOCK)


# ---------------------------------------------------------------------------
# split-precision expectation model
# ---------------------------------------------------------------------------

def m2l_split32_emulated(M, p, h, mask=FULL_MASK, offsets=None, block=64):
    """Expectation model of the split-FP32 M2L (not a bitwise reference).

    Moments are scaled to unit spacing (M_k h^-|k|), tables taken at h = 1;
    both are split into float32 hi/lo parts; per block of `block` offsets the
    three products hi.hi + hi.lo + lo.hi are summed in float32, the block sum
    is added to a float64 total, and L is scaled by h^(-1-|n|) at the end.
    """
    offsets = stencil() if offsets is None else offsets
    ks = multi_indices(p)
    C = len(ks)
    order = np.array([sum(k) for k in ks], dtype=np.float64)
    src = _masked(M, mask) * (h ** -order)[:, None, None, None]
    T = stencil_tensors(p, 1.0, offsets)
    m_hi = src.astype(np.float32)
    m_lo = (src - m_hi.astype(np.float64)).astype(np.float32)
    t_hi = T.astype(np.float32)
    t_lo = (T - t_hi.astype(np.float64)).astype(np.float32)
    L = np.zeros((C, BLOCK ** 3))
    for b0 in range(0, len(offsets), block):
        acc = np.zeros((C, BLOCK ** 3), dtype=np.float32)
        for i in range(b0, min(b0 + block, len(offsets))):
            d = offsets[i]
            wh = _source_window(m_hi, d).reshape(C, -1)
            wl = _source_window(m_lo, d).reshape(C, -1)
            acc += t_hi[i].T @ wh
            acc += t_lo[i].T @ wh
            acc += t_hi[i].T @ wl
        L += acc.astype(np.float64)
    L *= (h ** (-1.0 - order))[:, None]
    return L.reshape(C, BLOCK, BLOCK, BLOCK)


# ---------------------------------------------------------------------------
# exact-slice (Ozaki-style) low-precision M2L: expectation model
# ---------------------------------------------------------------------------
#
# The error-free splitting of Ozaki, Ogita, Oishi and Rump (2012), with int8
# slices and exact integer accumulation as Ootomo, Ozaki and Yokota apply it
# to matrix products on integer units: each float64 operand is scaled by a
# power of two into (-1, 1) and cut into s signed 7-bit integer slices,
#   X = sum_{i < s} x_i 2^(-7 (i + 1)) + r,  |x_i| <= 127,  |r| < 2^(-7 s);
# slice products x_i y_j are summed exactly in integers, and only the pairs
# with i + j <= s are kept (the rest weigh less than the truncation r).
#
# Applied to the harmonic form of M2L (the contraction over (d, k') of the
# folded moments with the tables restricted to K'_p x K'_p):
#   * the reduction runs over offsets and folded components together, so one
#     power of two must scale a whole operand row or column: the moments of a
#     sub-grid share one exponent e_A (after a fixed per-component prescale
#     2^f_k' that evens out the components' ranges), and each table column n'
#     has its own exponent e_B(n') over (d, k');
#   * the prescale is compensated in the tables (2^-f_k' on row k'), so the
#     products are unchanged;
#   * f_k' comes from the geometric bound of a folded moment per unit of cell
#     mass: with |a_i| <= h/2 per axis and the h^-|k| scaling, |M_k h^-|k|| <=
#     m 2^-|k| / k!, so |Mh_k'| <= m b_k' with b_k' = sum_k |F[k, k']| 2^-|k| / k!
#     and f_k' = -floor(log2 b_k').

SLICE_BITS = 7


def slice_prescale(p):
    """f_k' for the folded components K'_p (see above); integers, 0 for order 0."""
    ks = multi_indices(p)
    F = harmonic_fold(p)
    out = []
    for c in range(F.shape[1]):
        b = sum(abs(F[r, c]) * 0.5 ** sum(k) / (factorial(k[0]) * factorial(k[1]) * factorial(k[2]))
                for r, k in enumerate(ks) if F[r, c] != 0)
        out.append(-int(np.floor(np.log2(b))))
    return np.array(out, dtype=np.int64)


def pow2_exponent(x):
    """e with x / 2^e in [1/2, 1) for x > 0 (frexp's exponent); 0 for x = 0."""
    return int(np.frexp(float(x))[1]) if x > 0 else 0


def slice_int8(X, s):
    """s integer slices of X (every |X| < 1): X = sum_i S_i 2^(-7 (i+1)) + r,
    S_i integers with |S_i| <= 127, |r| < 2^(-7 s). Truncation toward zero, so
    every slice keeps the sign of X. Exact in float64 (power-of-two scalings
    and integer parts)."""
    X = np.asarray(X, dtype=np.float64)
    assert np.all(np.abs(X) < 1.0)
    out, Y = [], X.copy()
    for _ in range(s):
        Y = Y * 2.0 ** SLICE_BITS
        q = np.trunc(Y)
        out.append(q)
        Y = Y - q
    return out


def slice_pairs(s):
    """The kept slice products (i, j), i, j < s, i + j <= s, in the order they
    are summed: by i, then j."""
    return [(i, j) for i in range(s) for j in range(s) if i + j <= s]


def slice_tables(p, offsets=None):
    """Table operand of the exact-slice M2L at unit spacing: B[d][k'][n'] =
    T_d[k'][n'] 2^-f_k' 2^-e_B(n') (harmonic rows and columns), and e_B."""
    offsets = stencil() if offsets is None else offsets
    ks = multi_indices(p)
    hidx = [ks.index(k) for k in harmonic_indices(p)]
    T = stencil_tensors(p, 1.0, offsets)[:, hidx][:, :, hidx]
    Tf = T * 2.0 ** (-slice_prescale(p).astype(np.float64))[None, :, None]
    eB = np.array([pow2_exponent(np.abs(Tf[:, :, n]).max()) for n in range(Tf.shape[2])])
    return Tf * 2.0 ** (-eB.astype(np.float64))[None, None, :], eB


def m2l_exact_slice(M, p, h, mask=FULL_MASK, slices=7, offsets=None, with_accumulators=False):
    """Expectation model of the exact-slice M2L (harmonic form, int8 slices).

    Steps: fold and h-scale the moments (Mh_k' = h^-|k'| sum_k F[k, k'] M_k);
    prescale by 2^f_k'; one exponent e_A for the sub-grid (from the largest
    |value| over the reachable window [2, 22)^3, the only cells M2L reads);
    A = that / 2^e_A and B from slice_tables, both cut into
    `slices` slices; for every kept pair (i, j) the integer sum
    acc_ij[t][n'] = sum_{d, k'} A_i[k'](t + d) B_j[d][k'][n'] (exact);
    Lh_n' = 2^(e_A + e_B(n')) sum_{(i, j)} 2^(-7 (i + j + 2)) acc_ij (float64, in
    slice_pairs order); L = F Lh, scaled by h^(-1-|n|). Returns L [C, 8, 8, 8]
    (and the accumulators {(i, j): int array [512, C']} if asked).
    """
    offsets = stencil() if offsets is None else offsets
    ks = multi_indices(p)
    hs = harmonic_indices(p)
    Cp = len(hs)
    F = harmonic_fold(p)
    ordh = np.array([sum(k) for k in hs], dtype=np.float64)
    Mh = np.tensordot(F.T, _masked(M, mask), axes=(1, 0)) * (h ** -ordh)[:, None, None, None]
    # M2L reads only the reachable window [2, 22)^3 of the frame: the exponent
    # comes from there, and the cells outside it are never sliced
    Ms = np.zeros_like(Mh)
    w = slice(2, 22)
    Ms[:, w, w, w] = Mh[:, w, w, w] * 2.0 ** slice_prescale(p).astype(np.float64)[:, None, None, None]
    eA = pow2_exponent(np.abs(Ms).max())
    A = Ms * 2.0 ** -eA
    B, eB = slice_tables(p, offsets)
    As = slice_int8(A, slices)
    Bs = slice_int8(B, slices)
    lo = BLOCK
    acc = {}
    Lh = np.zeros((Cp, BLOCK ** 3))
    for i, j in slice_pairs(slices):
        Ai = As[i].astype(np.int64)
        a = np.zeros((BLOCK ** 3, Cp), dtype=np.int64)
        for d, Bd in zip(offsets, Bs[j].astype(np.int64)):
            dx, dy, dz = d
            win = Ai[:, lo + dz:lo + BLOCK + dz, lo + dy:lo + BLOCK + dy, lo + dx:lo + BLOCK + dx]
            a += win.reshape(Cp, -1).T @ Bd
        acc[(i, j)] = a
        Lh += a.T.astype(np.float64) * 2.0 ** (-SLICE_BITS * (i + j + 2))
    Lh *= 2.0 ** (eA + eB.astype(np.float64))[:, None]
    L = (F @ Lh) * (h ** (-1.0 - np.array([sum(k) for k in ks], dtype=np.float64)))[:, None]
    L = L.reshape(len(ks), BLOCK, BLOCK, BLOCK)
    return (L, acc) if with_accumulators else L
