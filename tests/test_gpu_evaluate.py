"""GPU parity of the evaluation at the particles (near field + L2P) through
the C ABI against the oracle.

Tolerance: per output entry |x_gpu - x_oracle| <= 1e-12 * x_abs, with x_abs
the same sums over absolute values (l2p_abs + near_field_abs). When L comes
from the device M2L, its own error (<= 1e-12 Labs per entry) passes into
the far part with weights |b^n| / n!, so the scale adds l2p_abs(Labs).
"""
import numpy as np
import pytest

import oracle as O
import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import descriptors, ensure_library, particles, split_views, to_dev

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


def random_L(desc, seed):
    """Seeded local expansions, order n scaled by 0.5^n like a far field."""
    rng = np.random.default_rng([seed, 77])
    out = []
    for d in desc:
        p = int(d["p"])
        scale = np.array([0.5 ** sum(k) for k in O.multi_indices(p)])
        out.append((rng.standard_normal((fmm.ncomp(p), 512)) * scale[:, None]).ravel())
    return np.concatenate(out)


def poisoned(pos, mass, desc):
    """Copies with the particles of absent blocks set to NaN (never to be read)."""
    pos, mass = pos.copy(), mass.copy()
    for b, d in enumerate(desc):
        absent = ~O.present_cells(int(d["mask"])).ravel()
        pos[b][absent] = np.nan
        mass[b][absent] = np.nan
    return pos, mass


def run_evaluate(ctx, torch, desc, pos, mass, ppc, L):
    out = torch.full((len(desc) * 4 * 512 * ppc,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.evaluate(desc, to_dev(pos), to_dev(mass), ppc, L if not isinstance(L, np.ndarray) else to_dev(L), out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(len(desc), 4, 512, ppc)


def check(got, want, scale, what):
    err = np.abs(got - want)
    bad = ~(err <= TOL * scale)
    assert not bad.any(), "%s: %d entries off, worst ratio %.3g" % (
        what, bad.sum(), np.nanmax(err / np.maximum(scale, 1e-300)))
    return float(np.max(err / scale))


def oracle_parts(pos, mass, p, h, mask, L):
    want = O.l2p(L, pos, p, h) + O.near_field(pos, mass, h, mask)
    scale = O.l2p_abs(L, pos, p, h) + O.near_field_abs(pos, mass, h, mask)
    return want, scale


@pytest.mark.parametrize("ppc", [8, 3, 13])
def test_evaluate_matches_oracle_mixed_batch(ctx, torch, ppc):
    # mixed p and h, random masks with the absent blocks' particles poisoned;
    # ppc 3 and 13 leave ragged particle chunks (and idle threads)
    w = synth.uneven_workload("ev_mixed", 31, 6)
    w.ppc = ppc
    idx = list(range(w.nsub))
    desc, _, l_el = descriptors(w, idx)
    pos, mass = particles(w, idx)
    L = random_L(desc, ppc)
    ppos, pmass = poisoned(pos, mass, desc)
    got = run_evaluate(ctx, torch, desc, ppos, pmass, ppc, L)
    Ls = split_views(L, desc, "L")
    assert sorted(set(w.p.tolist())) == [2, 3, 4]
    for b in idx:
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        want, scale = oracle_parts(pos[b], mass[b], p, h, mask, Ls[b])
        check(got[b], want, scale, "sub-grid %d (p=%d, h=%g, ppc=%d)" % (b, p, h, ppc))


def test_evaluate_edge_cases(ctx, torch):
    # empty batch; centre block only; one particle per cell (no same-cell pair);
    # 64 particles per cell (eight chunks) at the smallest spacing
    ctx.evaluate(np.zeros(0, fmm.DESC_DTYPE), None, None, 8, None, None)
    for ppc, p, lh, mask in [(1, 3, 0, synth.FULL_MASK), (8, 2, 1, 1 << 13), (64, 4, 2, synth.FULL_MASK)]:
        w = synth.Workload("ev_edge", 40 + ppc, np.array([p], np.int32), np.array([lh], np.int32),
                           np.array([mask], np.uint32), ppc=ppc)
        desc, _, _ = descriptors(w, [0])
        pos, mass = particles(w, [0])
        L = random_L(desc, 5)
        ppos, pmass = poisoned(pos, mass, desc)
        got = run_evaluate(ctx, torch, desc, ppos, pmass, ppc, L)
        want, scale = oracle_parts(pos[0], mass[0], p, w.h(0), mask, L.reshape(-1, 8, 8, 8))
        check(got[0], want, scale, "edge ppc=%d p=%d mask=%x" % (ppc, p, mask))


@pytest.mark.parametrize("prec", [fmm.FMM_FP64, fmm.FMM_FP64_HARMONIC])
def test_p2m_m2l_evaluate_chain_matches_oracle(ctx, torch, prec):
    # the whole same-level solve on the device against the oracle's own chain
    # (oracle L from oracle M); mixed p, h and masks
    w = synth.config(3, nsub=4)
    idx = list(range(w.nsub))
    desc, m_el, l_el = descriptors(w, idx)
    pos, mass = particles(w, idx)
    dpos, dmass = to_dev(pos), to_dev(mass)
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.empty(l_el, dtype=torch.float64, device="cuda")
    ctx.p2m(desc, dpos, dmass, w.ppc, M)
    ctx.m2l(desc, M, L, prec)
    out = torch.empty(len(desc) * 4 * 512 * w.ppc, dtype=torch.float64, device="cuda")
    ctx.evaluate(desc, dpos, dmass, w.ppc, L, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(len(desc), 4, 512, w.ppc)
    for b in idx:
        p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
        Mo = O.p2m(pos[b], mass[b], p, h, mask)
        Lo, La = O.m2l(Mo, p, h, mask), O.m2l_abs(Mo, p, h, mask)
        want, scale = oracle_parts(pos[b], mass[b], p, h, mask, Lo)
        scale = scale + O.l2p_abs(La, pos[b], p, h)
        check(got[b], want, scale, "chain sub-grid %d (p=%d, prec=%d)" % (b, p, prec))


def test_evaluate_is_deterministic_and_writes_only_its_output(ctx, torch):
    w = synth.config(3, nsub=5)
    idx = list(range(w.nsub))
    desc, _, _ = descriptors(w, idx)
    pos, mass = particles(w, idx)
    L = to_dev(random_L(desc, 9))
    dpos, dmass = to_dev(pos), to_dev(mass)
    n = len(desc) * 4 * 512 * w.ppc
    buf = torch.full((n + 1024,), -7.0, dtype=torch.float64, device="cuda")
    ctx.evaluate(desc, dpos, dmass, w.ppc, L, buf[512:512 + n])
    out2 = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.evaluate(desc, dpos, dmass, w.ppc, L, out2)
    torch.cuda.synchronize()
    assert torch.equal(buf[512:512 + n], out2) and torch.isfinite(out2).all()
    assert (buf[:512] == -7.0).all() and (buf[512 + n:] == -7.0).all()
