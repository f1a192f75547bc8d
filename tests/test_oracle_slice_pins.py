"""Pins of the exact-slice M2L expectation model (oracle.m2l_exact_slice), the
oracle of the int8 matrix-core path.

The model follows the error-free splitting of Ozaki et al. with int8 slices:
operands scaled by powers of two into (-1, 1), cut into 7-bit integer
slices, slice products summed exactly as integers. Its pins:
* the slicing itself reconstructs every value with at most 7 s significant
  bits exactly, with integer slices in [-127, 127] that keep the value's sign;
* the prescale f_k' equals the geometric bound of the folded moments worked
  out by hand, and bounds the prescaled moments of any cell;
* the result converges to the float64 M2L of the oracle as slices are added
  (error falling by ~2^-7 per slice) and stays within the rigorous truncation
  bound of the splitting;
* every integer sum fits int32 (the hardware accumulator).
Planted mistakes (the i + j = s diagonal dropped, table exponents taken per
row, the prescale left uncompensated) each fail a pin.
"""
from math import factorial

import numpy as np
import pytest

import oracle as O
import oracle.fmm as OF
import synth


def test_slicing_is_exact_and_signed():
    rng = np.random.default_rng(3)
    for s in (1, 4, 7, 8):
        X = rng.uniform(-1, 1, 4096)
        X[:4] = [0.0, -0.0, 1 - 2.0 ** -53, -(1 - 2.0 ** -53)]
        Xs = np.trunc(X * 2.0 ** (7 * s)) * 2.0 ** (-7 * s)      # at most 7 s significant bits
        parts = O.slice_int8(Xs, s)
        rec = sum(q * 2.0 ** (-7 * (i + 1)) for i, q in enumerate(parts))
        assert np.array_equal(rec, Xs)
        for q in parts:
            assert np.array_equal(q, np.trunc(q)) and np.abs(q).max() <= 127
            assert np.all(q * Xs >= 0)                             # sign of the value
        # any float64: the remainder is below the last slice's weight
        parts = O.slice_int8(X, s)
        rec = sum(q * 2.0 ** (-7 * (i + 1)) for i, q in enumerate(parts))
        assert np.all(np.abs(X - rec) < 2.0 ** (-7 * s))


def test_kept_slice_pairs():
    assert O.slice_pairs(7) == [(i, j) for i in range(7) for j in range(7) if i + j <= 7]
    assert [len(O.slice_pairs(s)) for s in (5, 6, 7, 8)] == [19, 26, 34, 43]


def test_prescale_is_the_geometric_bound():
    # by hand: order 0 -> b = 1, f = 0; x, y, z -> b = 1/2, f = 1; (2,0,0) collects
    # (2,0,0) and (0,0,2) with coefficients 1 and -1: b = 2 * 2^-2 / 2! = 1/4, f = 2;
    # (1,1,0) collects itself only: b = 2^-2, f = 2; (0,1,1) likewise
    f = O.slice_prescale(3)
    hs = O.harmonic_indices(3)
    assert f[hs.index((0, 0, 0))] == 0 and f[hs.index((1, 0, 0))] == 1 and f[hs.index((0, 0, 1))] == 1
    assert f[hs.index((2, 0, 0))] == 2 and f[hs.index((1, 1, 0))] == 2 and f[hs.index((0, 1, 1))] == 2
    F = O.harmonic_fold(3)
    ks = O.multi_indices(3)
    for c, k in enumerate(hs):
        b = sum(abs(F[r, c]) * 0.5 ** sum(kk) / (factorial(kk[0]) * factorial(kk[1]) * factorial(kk[2]))
                for r, kk in enumerate(ks))
        assert 1.0 <= b * 2.0 ** f[c] < 2.0
    assert np.array_equal(O.slice_prescale(2), f[:9])
    # cells of unit mass with particles anywhere inside: the prescaled folded
    # moments stay below 2 (the bound is reached within a factor of 4 at some cell)
    rng = np.random.default_rng(5)
    a = rng.uniform(-0.5, 0.5, (4000, 8, 3))
    a[:8] = np.sign(rng.uniform(-1, 1, (8, 8, 3))) * 0.5                # corners
    m = rng.dirichlet(np.ones(8), 4000)
    mono = np.stack([np.prod(a ** np.array(k), axis=-1) / (factorial(k[0]) * factorial(k[1]) * factorial(k[2]))
                     for k in ks])                                   # [C, cells, 8]
    Mk = np.einsum("cij,ij->ci", mono, m)
    Mh = F.T @ Mk * 2.0 ** f[:, None]
    assert np.abs(Mh).max() < 2.0 and np.all(np.abs(Mh).max(axis=1) > 0.25)


@pytest.fixture(scope="module")
def subgrids():
    out = []
    for p, h, sub, mseed in [(3, 1.0, 0, None), (2, 0.25, 7, 4)]:
        mask = O.FULL_MASK if mseed is None else synth.random_mask(np.random.default_rng(mseed))
        pos, mass = synth.subgrid_particles(2, sub, h)
        M = O.p2m(pos, mass, p, h, mask)
        out.append((M, p, h, mask, O.m2l(M, p, h, mask), O.m2l_abs(M, p, h, mask)))
    return out


# largest |L_model - L| / Labs allowed per slice count: the model's measured
# error (5: 1.7e-10 - 2.7e-10, 6: 1.4e-12 - 2.5e-12, 7: 1.3e-14 - 1.7e-14,
# 8: 2e-15 - 3e-15 on these and other workload sub-grids) with margin
SLICE_BOUND = {5: 1e-9, 6: 1e-11, 7: 5e-14, 8: 1e-14}


def _converges(model, subgrids):
    for M, p, h, mask, L, La in subgrids:
        prev = np.inf
        for s in (5, 6, 7, 8):
            e = np.max(np.abs(model(M, p, h, mask, s) - L) / La)
            if not e <= SLICE_BOUND[s] or not e < prev:
                return False
            prev = e
    return True


def test_model_converges_to_the_float64_m2l(subgrids):
    assert _converges(lambda M, p, h, mask, s: O.m2l_exact_slice(M, p, h, mask, s), subgrids)


def test_truncation_bound_of_the_splitting(subgrids):
    # per product |AB - sum_kept a_i b_j 2^-7(i+j+2)| <= 2 * 2^-7s + sum over the
    # dropped pairs of 127^2 2^-7(i+j+2); per target column n' at most 892 C' products,
    # scaled back by 2^(e_A + e_B(n'))
    for M, p, h, mask, L, La in subgrids:
        hs = O.harmonic_indices(p)
        hidx = [O.multi_indices(p).index(k) for k in hs]
        Lh = O.m2l_harmonic(M, p, h, mask)[hidx].reshape(len(hs), -1)
        F = O.harmonic_fold(p)
        ordh = np.array([sum(k) for k in hs], dtype=np.float64)
        Ms = (np.tensordot(F.T, np.where(O.present_cells(mask)[None], M, 0.0), axes=(1, 0))
              * (h ** -ordh)[:, None, None, None] * 2.0 ** O.slice_prescale(p)[:, None, None, None])
        eA = O.pow2_exponent(np.abs(Ms[:, 2:22, 2:22, 2:22]).max())
        _, eB = O.slice_tables(p)
        for s in (5, 7):
            dropped = sum(127.0 ** 2 * 2.0 ** (-7 * (i + j + 2)) for i in range(s) for j in range(s) if i + j > s)
            per = 2 * 2.0 ** (-7 * s) + dropped
            bound = 892 * len(hs) * per * 2.0 ** (eA + eB)[:, None] * (h ** (-1.0 - ordh))[:, None]
            got = O.m2l_exact_slice(M, p, h, mask, s)[hidx].reshape(len(hs), -1)
            assert np.all(np.abs(got - Lh) <= bound + 1e-14 * La[hidx].reshape(len(hs), -1))


def test_integer_sums_fit_int32(subgrids):
    # worst case per kept pair: 892 offsets x 16 components x 127^2, and per slice
    # group g = i + j at most 8 pairs: within int32 either way
    assert 892 * 16 * 127 ** 2 * 8 < 2 ** 31
    for M, p, h, mask, L, La in subgrids:
        _, acc = O.m2l_exact_slice(M, p, h, mask, 7, with_accumulators=True)
        assert max(np.abs(a).max() for a in acc.values()) < 2 ** 31
        groups = {}
        for (i, j), a in acc.items():
            groups[i + j] = groups.get(i + j, 0) + a
        assert max(np.abs(g).max() for g in groups.values()) < 2 ** 31


def _slice_tables_rows(p, offsets=None):
    # planted: exponents per table row k' instead of per column n'
    Bt, eB = OF.__dict__["_orig_slice_tables"](p, offsets)
    Tf = Bt * 2.0 ** eB[None, None, :]
    er = np.array([O.pow2_exponent(np.abs(Tf[:, k, :]).max()) for k in range(Tf.shape[1])])
    return Tf * 2.0 ** (-er)[None, :, None], eB


def _slice_tables_no_prescale(p, offsets=None):
    # planted: the moments' prescale left uncompensated in the tables
    Bt, eB = OF.__dict__["_orig_slice_tables"](p, offsets)
    Tf = Bt * 2.0 ** eB[None, None, :] * 2.0 ** O.slice_prescale(p)[None, :, None]
    eB2 = np.array([O.pow2_exponent(np.abs(Tf[:, :, n]).max()) for n in range(Tf.shape[2])])
    return Tf * 2.0 ** (-eB2)[None, None, :], eB2


MUTANTS = {
    "diagonal i + j = s dropped": ("slice_pairs", lambda s: [(i, j) for i in range(s) for j in range(s) if i + j < s]),
    "table exponents per row": ("slice_tables", _slice_tables_rows),
    "prescale uncompensated": ("slice_tables", _slice_tables_no_prescale),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name, subgrids, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setitem(OF.__dict__, "_orig_slice_tables", OF.slice_tables)
    monkeypatch.setattr(OF, attr, fn)
    assert not _converges(lambda M, p, h, mask, s: OF.m2l_exact_slice(M, p, h, mask, s), subgrids[:1]), name
