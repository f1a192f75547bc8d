"""CPU emulation of exact-slice low precision for M2L (int8 slices of the
moments and of T_d with shared power-of-two exponents, Ozaki-style). It
measures how many slices per operand one p = 3 sub-grid needs to stay within
the 1e-12 absolute-sum bound of the float64 parity tests: seven. The library has no
such kernel; this pins the figure its design weighs.

The contraction of Sec. VII-C is written as one product
A [512 targets x (offset, k)] . B [(offset, k) x n]. Exponents:
* one per moment component k over the whole window, compensated in the
  table rows, so each window value is sliced once;
* one per output column n of the tables.
Each operand is cut into s slices of 7 magnitude bits (int8). Only the
products of slices i + j <= s are summed (the truncated triangle). Each slice
product is exact: an int32 accumulator holds its sums, and float64 evaluates
them exactly here.
"""
import numpy as np
import pytest

import oracle as O
import synth

BITS = 7
P = 3


@pytest.fixture(scope="module")
def operands():
    w = synth.config(2, nsub=1)
    seed, b = synth.subgrid_seed_args(w, 0)
    h = w.h(0)
    pos, mass = synth.subgrid_particles(seed, b, h, w.ppc)
    M = O.p2m(pos, mass, P, h, int(w.mask[0]))
    S = O.stencil()
    C = O.ncomp(P)
    lo = O.BLOCK
    A = np.concatenate([M[:, lo + dz:lo + 8 + dz, lo + dy:lo + 8 + dy, lo + dx:lo + 8 + dx].reshape(C, -1).T
                        for dx, dy, dz in S], axis=1)
    B = O.stencil_tensors(P, h).reshape(len(S) * C, C)
    L = (A @ B).T.reshape(C, 8, 8, 8)
    Labs = (np.abs(A) @ np.abs(B)).T.reshape(C, 8, 8, 8)
    # the product form is the oracle's M2L
    assert np.all(np.abs(L - O.m2l(M, P, h)) <= 1e-13 * O.m2l_abs(M, P, h))
    return A, B, L, Labs


def split(X, s):
    """s integer slices (|slice| <= 127) of X, |X| < 1: X ~ sum_q S_q 2^(-7(q+1))."""
    assert np.abs(X).max() < 1
    out, Y = [], X.copy()
    for _ in range(s):
        Y = Y * 2 ** BITS
        q = np.trunc(Y)
        out.append(q)
        Y = Y - q
    return out


def exponent(m):
    """e with m / 2^e in [0.5, 1)"""
    return np.frexp(m)[1].astype(np.float64)


def sliced_m2l(A, B, s):
    C = B.shape[1]
    k = np.arange(A.shape[1]) % C
    ek = np.array([exponent(np.abs(A[:, k == c]).max()) for c in range(C)])
    A2 = A / 2.0 ** ek[k][None, :]
    B2 = B * 2.0 ** ek[k][:, None]
    eb = exponent(np.abs(B2).max(axis=0))
    As, Bs = split(A2, s), split(B2 / 2.0 ** eb[None, :], s)
    for q in As + Bs:
        assert np.abs(q).max() <= 127 and np.array_equal(q, np.trunc(q))
    out, nprod = np.zeros((A.shape[0], C)), 0
    for i in range(s):
        for j in range(min(s, s - i + 1)):
            out += (As[i] @ Bs[j]) * 2.0 ** (-BITS * (i + j + 2))
            nprod += 1
    return out * 2.0 ** eb[None, :], nprod


def test_slice_products_fit_int32(operands):
    A, B, _, _ = operands
    assert A.shape[1] * 127 ** 2 < 2 ** 31


@pytest.mark.parametrize("s,nprod,lo,hi", [(5, 19, 1e-12, 1e-9), (6, 26, 1e-13, 1e-11), (7, 34, 0.0, 1e-13)])
def test_slices_needed_for_the_parity_bound(operands, s, nprod, lo, hi):
    # 5 slices miss the 1e-12 bound, 6 sit at it (the potential column, a sum
    # of positive terms, carries the truncation of both operands), 7 clear it
    A, B, L, Labs = operands
    Ls, n = sliced_m2l(A, B, s)
    assert n == nprod
    err = np.abs(Ls.T.reshape(L.shape) - L) / Labs
    assert lo < err.max() <= hi, "s=%d: max %.3g" % (s, err.max())
