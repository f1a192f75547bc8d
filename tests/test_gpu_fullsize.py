"""GPU parity at the benchmark sizes, in the launch configuration bench.py
times: whole batches run on the device, sampled sub-grids are checked
against the oracle one by one, and whole-batch properties are checked on
everything (finite, deterministic). Also the differentiable path: central
finite differences on 64 mass entries and the oracle gradient.
"""
import numpy as np
import pytest

import oracle as O
import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import ensure_library

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


def device_batch(torch, w):
    with synth.SharedBatch(w) as sb:
        pos = torch.from_numpy(sb.pos).to("cuda")
        mass = torch.from_numpy(sb.mass).to("cuda")
        torch.cuda.synchronize()
    return pos, mass


def host_subgrid(w, b):
    return synth.subgrid_particles(w.seed, b, w.h(b), w.ppc)


def check_sampled(w, desc, L, sample, tol=TOL):
    worst = 0.0
    for b in sample:
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        C = fmm.ncomp(p)
        o = int(desc["l_off"][b])
        Lg = L[o:o + C * 512].cpu().numpy().reshape(C, 8, 8, 8)
        pos, mass = host_subgrid(w, b)
        M = O.p2m(pos, mass, p, h, mask)
        Lo, La = O.m2l(M, p, h, mask), O.m2l_abs(M, p, h, mask)
        r = np.max(np.abs(Lg - Lo) / La)
        assert r <= tol, (b, p, r)
        worst = max(worst, r)
    return worst


def test_uniform_4096_fp64_and_split(ctx, torch):
    w = synth.config(2)
    desc, m_el, l_el = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    pos, mass = device_batch(torch, w)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.empty(l_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, pos, mass, 8, M)
    ctx.autotune(desc, M, L, fmm.FMM_FP64)
    ctx.m2l(desc, M, L)
    L2 = torch.empty_like(L)
    ctx.m2l(desc, M, L2)
    torch.cuda.synchronize()
    assert torch.isfinite(L).all() and torch.equal(L, L2)
    worst = check_sampled(w, desc, L, [0, 1, 2047, 4095])
    print("4096 batch, dense FP64: max |dL|/Labs %.3g on sampled sub-grids" % worst)
    # split precision on the same moments: bounded error, everywhere finite
    Ls = torch.empty_like(L)
    ctx.m2l(desc, M, Ls, fmm.FMM_SPLIT_FP32)
    torch.cuda.synchronize()
    assert torch.isfinite(Ls).all()
    rel = []
    for b in (0, 4095):
        o = int(desc["l_off"][b])
        pos_b, mass_b = host_subgrid(w, b)
        Mo = O.p2m(pos_b, mass_b, 3, 1.0)
        Lo, La = O.m2l(Mo, 3, 1.0), O.m2l_abs(Mo, 3, 1.0)
        rel.append((np.abs(Ls[o:o + 20 * 512].cpu().numpy().reshape(20, 8, 8, 8) - Lo) / La).ravel())
    rel = np.concatenate(rel)
    print("4096 batch, split FP32: |dL|/Labs max %.3g, median %.3g" % (rel.max(), np.median(rel)))
    assert rel.max() < 1e-6 and np.median(rel) < 5e-8
    # the configuration the step is timed in: P2M over the rows holding the
    # reachable window, then the autotuned harmonic form, replayed from its graph
    Mw = torch.full_like(M, float("nan"))
    ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 1)
    try:
        ctx.p2m(desc, pos, mass, 8, Mw)
    finally:
        ctx.set_option(fmm.FMM_OPT_P2M_WINDOW, 0)
    Lh = torch.empty_like(L)
    ctx.autotune(desc, Mw, Lh, fmm.FMM_FP64_HARMONIC)
    ctx.m2l(desc, Mw, Lh, fmm.FMM_FP64_HARMONIC)
    Lh2 = torch.empty_like(L)
    ctx.m2l(desc, Mw, Lh2, fmm.FMM_FP64_HARMONIC)
    torch.cuda.synchronize()
    assert torch.isfinite(Lh).all() and torch.equal(Lh, Lh2)
    worst = check_sampled(w, desc, Lh, [0, 1, 2047, 4095])
    print("4096 batch, harmonic FP64 (the step's form): max |dL|/Labs %.3g on sampled sub-grids" % worst)
    # the step as the bench times it: one launch (fmm_p2m_m2l), replayed from its
    # graph: the same moments in the rows and the same L, bit for bit
    Mf = torch.full_like(M, float("nan"))
    Lf = torch.empty_like(L)
    for _ in range(2):
        ctx.p2m_m2l(desc, pos, mass, 8, Mf, Lf, fmm.FMM_FP64_HARMONIC)
    torch.cuda.synchronize()
    assert torch.equal(Lf, Lh)
    assert torch.equal(torch.nan_to_num(Mf, 0.0), torch.nan_to_num(Mw, 0.0))
    # the exact-slice M2L as the bench times it (the window-row moments), at 7 and 6
    # slices: 1e-12 and 1e-11 of Labs on sampled sub-grids, deterministic
    for slices, tol in ((7, 1e-12), (6, 1e-11)):
        ctx.set_option(fmm.FMM_OPT_SLICES, slices)
        try:
            Lx = torch.full_like(L, float("nan"))
            Lx2 = torch.full_like(L, float("nan"))
            ctx.m2l(desc, Mw, Lx, fmm.FMM_EXACT_SLICE)
            ctx.m2l(desc, Mw, Lx2, fmm.FMM_EXACT_SLICE)
            torch.cuda.synchronize()
        finally:
            ctx.set_option(fmm.FMM_OPT_SLICES, 7)
        assert torch.isfinite(Lx).all() and torch.equal(Lx, Lx2)
        worst = check_sampled(w, desc, Lx, [0, 1, 2047, 4095], tol)
        print("exact slices, %d slices: max |dL|/Labs %.3g on sampled sub-grids" % (slices, worst))


def test_uniform_4096_evaluate(ctx, torch):
    # P2M -> harmonic M2L -> evaluation at all 16.8M target particles, as timed;
    # sampled sub-grids against the oracle's own chain; the whole output is finite,
    # deterministic, and the potential is positive everywhere (positive masses)
    w = synth.config(2)
    desc, m_el, l_el = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    pos, mass = device_batch(torch, w)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.empty(l_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, pos, mass, 8, M)
    ctx.m2l(desc, M, L, fmm.FMM_FP64_HARMONIC)
    del M
    n = w.nsub * 4 * 512 * 8
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.evaluate(desc, pos, mass, 8, L, out)
    out2 = torch.empty_like(out)
    ctx.evaluate(desc, pos, mass, 8, L, out2)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all() and torch.equal(out, out2)
    got = out.view(w.nsub, 4, 512, 8)
    assert (got[:, 0] > 0).all()
    for b in (0, 2049, 4095):
        pos_b, mass_b = host_subgrid(w, b)
        Mo = O.p2m(pos_b, mass_b, 3, 1.0)
        Lo, La = O.m2l(Mo, 3, 1.0), O.m2l_abs(Mo, 3, 1.0)
        want = O.l2p(Lo, pos_b, 3, 1.0) + O.near_field(pos_b, mass_b, 1.0)
        scale = (O.l2p_abs(Lo, pos_b, 3, 1.0) + O.near_field_abs(pos_b, mass_b, 1.0)
                 + O.l2p_abs(La, pos_b, 3, 1.0))
        err = np.abs(got[b].cpu().numpy() - want)
        assert np.all(err <= TOL * scale), (b, float(np.max(err / scale)))


def test_tree_128_solve(ctx, torch):
    # the multi-level iteration on a 128^3 domain (16.8M particles, p = 3), as
    # timed: two solves bitwise equal, finite, positive potential; two cells (a
    # corner and an interior one) against the oracle's per-cell route
    import oracle.tree as T
    n, ppc, p = 128, 8, 3
    tree = fmm.Tree(p, n, ppc, 0, 1)         # the harmonic form of the level M2L, as timed
    _, elems = fmm.tree_size(tree)
    pos_h, mass_h = synth.grid_particles(40, n, 1.0, ppc)
    pos, mass = torch.from_numpy(pos_h).to("cuda"), torch.from_numpy(mass_h).to("cuda")
    M = torch.empty(elems, dtype=torch.float64, device="cuda")
    L = torch.empty(elems, dtype=torch.float64, device="cuda")
    out = torch.empty(4 * n ** 3 * ppc, dtype=torch.float64, device="cuda")
    out2 = torch.empty_like(out)
    ctx.tree_solve(tree, pos, mass, M, L, out)
    ctx.tree_solve(tree, pos, mass, M, L, out2)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all() and torch.equal(out, out2)
    E = out.view(4, n, n, n, ppc)
    assert (E[0] > 0).all()
    for t in [(0, 0, 0), (77, 31, 100)]:
        want = T.evaluate_at(pos_h, mass_h, p, n, 1.0, t)
        scale = T.evaluate_at(pos_h, mass_h, p, n, 1.0, t, absolute=True)
        got = E[:, t[2], t[1], t[0]].cpu().numpy()
        assert np.all(np.abs(got - want) <= TOL * scale), (t, float(np.max(np.abs(got - want) / scale)))


def test_uneven_6000(ctx, torch):
    w = synth.config(3)
    desc, m_el, l_el = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    pos, mass = device_batch(torch, w)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.empty(l_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, pos, mass, 8, M)
    ctx.m2l(desc, M, L)
    torch.cuda.synchronize()
    assert torch.isfinite(L).all()
    # one sample of each order and spacing, plus the fewest- and most-masked sub-grids
    sample = set()
    for p in (2, 3, 4):
        sample.add(int(np.nonzero(w.p == p)[0][0]))
    for lh in (0, 1, 2):
        sample.add(int(np.nonzero(w.log2_inv_h == lh)[0][0]))
    nbits = np.array([bin(int(m)).count("1") for m in w.mask])
    sample.add(int(np.argmin(nbits)))
    sample.add(int(np.argmax(nbits)))
    worst = check_sampled(w, desc, L, sorted(sample))
    print("uneven 6000: max |dL|/Labs %.3g on %d sampled sub-grids" % (worst, len(sample)))


def test_gradient_2048_fd_and_oracle(ctx, torch):
    from paper_2304_11002_amd.autograd import gravity_local_expansion
    w = synth.config(5)
    desc, m_el, l_el = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    pos, mass = device_batch(torch, w)
    wt = torch.from_numpy(synth.loss_weights(w.seed, w.nsub)).to("cuda").reshape(-1)
    m = mass.clone().requires_grad_(True)
    L = gravity_local_expansion(ctx, desc, pos, m)
    loss = torch.dot(wt, L)
    loss.backward()
    g = m.grad.detach()
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    gmax = float(g.abs().max())
    entries = synth.fd_entries(w.seed, w.nsub)
    eps = 1e-6
    wt_h = wt.cpu().numpy().reshape(w.nsub, 20, 512)
    by_sub = {}
    for b, cell, i in entries:
        by_sub.setdefault(int(b), []).append((int(cell), int(i)))
    with torch.no_grad():
        for b, cells in by_sub.items():
            o = int(desc["l_off"][b])
            for cell, i in cells:
                mp = mass.clone()
                mp[b, cell, i] += eps
                Lp = gravity_local_expansion(ctx, desc, pos, mp)[o:o + 10240].cpu().numpy()
                mp[b, cell, i] -= 2 * eps
                Lm = gravity_local_expansion(ctx, desc, pos, mp)[o:o + 10240].cpu().numpy()
                fd = float(np.sum(wt_h[b].ravel() * (Lp - Lm)) / (2 * eps))
                gi = float(g[b, cell, i])
                # the loss is linear in the masses: central differences are exact up to
                # the rounding of L(m +- eps) (|L_0| ~ 3e3), bounded here entry-wise by
                # the spacing of each L value, weighted by |w| and added in quadrature
                moved = Lp != Lm
                rnd = np.sqrt(np.sum((wt_h[b].ravel()[moved] * np.spacing(np.abs(Lp[moved]))) ** 2))
                tol = 1e-5 * max(abs(gi), 1e-3 * gmax) + 8 * rnd / (2 * eps)
                assert abs(fd - gi) <= tol, (b, cell, i, fd, gi, tol)
    # the oracle's gradient on the sub-grids those entries fall in
    for b in list(by_sub)[:6]:
        pos_b, mass_b = host_subgrid(w, b)
        W = wt_h[b].reshape(20, 8, 8, 8)
        Go = O.m2l_adjoint(W, 3, 1.0)
        go = O.p2m_adjoint(pos_b, Go, 3, 1.0)
        Ga = O.m2l_adjoint_abs(W, 3, 1.0)
        c = O.cell_centres(1.0)[:, None, :]
        scale = O.p2m_adjoint(c + np.abs(pos_b - c), Ga, 3, 1.0)
        gb = g[b].cpu().numpy()
        nz = scale > 0
        print("gradient 2048, sub-grid %d: max |dg|/scale %.3g against the oracle"
              % (b, float(np.max(np.abs(gb - go)[nz] / scale[nz]))))
        assert np.all(np.abs(gb - go) <= TOL * scale)


@pytest.mark.parametrize("harmonic", [False, True])
def test_gradcheck_fast_mode_one_subgrid(ctx, torch, harmonic):
    from paper_2304_11002_amd.autograd import gravity_local_expansion
    w = synth.config(3, nsub=2)
    desc, _, _ = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    P, Mm = [], []
    for b in range(2):
        pos, mass = host_subgrid(w, b)
        P.append(pos)
        Mm.append(mass)
    pos = torch.from_numpy(np.stack(P)).to("cuda")
    mass = torch.from_numpy(np.stack(Mm)).to("cuda").requires_grad_(True)
    # L is linear in the masses, so fast-mode gradcheck (random projections) is exact
    # up to rounding; with |L_0| ~ 3e3 the rounding of L(m +- eps u) limits the
    # numerical side to ~1e-5 relative, hence the tolerances (the exact gradient is
    # checked against the oracle above)
    assert torch.autograd.gradcheck(lambda m: gravity_local_expansion(ctx, desc, pos, m, harmonic=harmonic),
                                    (mass,),
                                    eps=1e-6, atol=1e-4, rtol=1e-4, fast_mode=True)
