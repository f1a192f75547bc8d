"""GPU parity of the exact-slice M2L (FMM_EXACT_SLICE: int8 slices, exact int32
sums on the matrix cores) against the float64 oracle and against the
oracle's expectation model of the same splitting (oracle.m2l_exact_slice).

Bars, per entry and relative to the oracle's absolute-value sum Labs:
* against the float64 M2L: 1e-11 at 6 slices, 1e-12 at 7, 1e-13 at 8 (the
  model's own error is 1.4e-12 to 2.5e-12, 1.3e-14 to 1.7e-14 and 2e-15 to
  3e-15 on workload sub-grids);
* against the model: 2e-13 at every slice count. Both sides cut the same
  values into the same slices and sum the kept slice products exactly; they
  differ only where float64 rounding of the fold or of the device tables (a
  derivative recurrence, against the oracle's closed form) moves a value
  across a slice boundary, and in the float64 sum of the slice products.
"""
import numpy as np
import pytest

import oracle as O
import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import ensure_library, split_views, to_dev

pytestmark = pytest.mark.gpu
BAR = {6: 1e-11, 7: 1e-12, 8: 1e-13}
MODEL_TOL = 2e-13


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


def _batch(seed, n, orders=(2, 3)):
    """n sub-grids of orders 2 and 3 with random masks (first one full) and
    spacings, particles drawn like the uneven workload."""
    rng = np.random.default_rng(seed)
    p = rng.choice(orders, n)
    l2 = rng.integers(0, 3, n)
    masks = [O.FULL_MASK] + [synth.random_mask(rng) for _ in range(n - 1)]
    desc, m_el, l_el = fmm.make_descriptors(p, l2, masks)
    pos, mass = [], []
    for b in range(n):
        ps, ms = synth.subgrid_particles(seed, b, 2.0 ** -int(l2[b]))
        pos.append(ps)
        mass.append(ms)
    return desc, m_el, l_el, np.stack(pos), np.stack(mass)


def _run(ctx, torch, desc, m_el, l_el, pos, mass, slices):
    M = torch.empty(m_el, dtype=torch.float64, device="cuda")
    L = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.p2m(desc, to_dev(pos), to_dev(mass), 8, M)
    ctx.set_option(fmm.FMM_OPT_SLICES, slices)
    try:
        ctx.m2l(desc, M, L, fmm.FMM_EXACT_SLICE)
    finally:
        ctx.set_option(fmm.FMM_OPT_SLICES, 7)
    torch.cuda.synchronize()
    return M.cpu().numpy(), L.cpu().numpy()


def _check(desc, Mh, Lh, slices, model_at=()):
    worst, worst_model = 0.0, 0.0
    for b, (d, Mv, Lv) in enumerate(zip(desc, split_views(Mh, desc, "M"), split_views(Lh, desc, "L"))):
        p, h, mask = int(d["p"]), 2.0 ** -int(d["log2_inv_h"]), int(d["mask"])
        L = O.m2l(Mv, p, h, mask)
        La = O.m2l_abs(Mv, p, h, mask)
        r = np.max(np.abs(Lv - L) / La)
        assert r <= BAR[slices], "sub-grid %d (p=%d, h=%g): %.3g of Labs" % (b, p, h, r)
        worst = max(worst, r)
        if b in model_at:
            Lm = O.m2l_exact_slice(Mv, p, h, mask, slices)
            rm = np.max(np.abs(Lv - Lm) / La)
            assert rm <= MODEL_TOL, "sub-grid %d against the model: %.3g of Labs" % (b, rm)
            worst_model = max(worst_model, rm)
    return worst, worst_model


@pytest.mark.parametrize("slices", [6, 7, 8])
def test_single_subgrid_against_oracle_and_model(ctx, torch, slices):
    w = synth.config(1)
    desc, m_el, l_el = fmm.make_descriptors(w.p, w.log2_inv_h, w.mask)
    pos, mass = synth.subgrid_particles(0)
    Mh, Lh = _run(ctx, torch, desc, m_el, l_el, pos[None], mass[None], slices)
    worst, wm = _check(desc, Mh, Lh, slices, model_at=(0,))
    print("slices %d: max |dL|/Labs %.3g against the oracle, %.3g against the model" % (slices, worst, wm))


def test_mixed_batch_orders_masks_spacings(ctx, torch):
    desc, m_el, l_el, pos, mass = _batch(31, 40)
    Mh, Lh = _run(ctx, torch, desc, m_el, l_el, pos, mass, 7)
    # the model at a masked p = 2 and a masked p = 3 sub-grid
    p2 = [b for b in range(1, 40) if desc[b]["p"] == 2][0]
    p3 = [b for b in range(1, 40) if desc[b]["p"] == 3][0]
    worst, wm = _check(desc, Mh, Lh, 7, model_at=(p2, p3))
    print("mixed batch: max |dL|/Labs %.3g, against the model %.3g" % (worst, wm))


def test_ragged_batch_larger_than_the_gpu(ctx, torch):
    # more sub-grids than compute units (workgroups take several each), in a
    # ragged layout; every present block and an all-absent neighbourhood included
    n = 300
    desc, m_el, l_el, pos, mass = _batch(32, n)
    desc["mask"][5] = 1 << synth.CENTRE_BIT
    Mh, Lh = _run(ctx, torch, desc, m_el, l_el, pos, mass, 7)
    for b in list(range(0, n, 37)) + [5, n - 1]:
        _check(desc[b:b + 1], Mh, Lh, 7)


def test_deterministic_and_equal_to_a_sub_batch(ctx, torch):
    desc, m_el, l_el, pos, mass = _batch(33, 12)
    _, L1 = _run(ctx, torch, desc, m_el, l_el, pos, mass, 7)
    _, L2 = _run(ctx, torch, desc, m_el, l_el, pos, mass, 7)
    assert np.array_equal(L1, L2)
    # a sub-grid's result does not depend on the rest of the batch
    d1, m1, l1 = fmm.make_descriptors(desc["p"][4:5], desc["log2_inv_h"][4:5], desc["mask"][4:5])
    _, L3 = _run(ctx, torch, d1, m1, l1, pos[4:5], mass[4:5], 7)
    assert np.array_equal(split_views(L1, desc, "L")[4], split_views(L3, d1, "L")[0])


def test_order_4_is_unsupported(ctx, torch):
    desc, m_el, l_el = fmm.make_descriptors([3, 4], [0, 0], [O.FULL_MASK] * 2)
    M = torch.zeros(m_el, dtype=torch.float64, device="cuda")
    L = torch.zeros(l_el, dtype=torch.float64, device="cuda")
    with pytest.raises(fmm.FMMError) as ex:
        ctx.m2l(desc, M, L, fmm.FMM_EXACT_SLICE)
    assert ex.value.status == fmm.FMM_EUNSUPPORTED
