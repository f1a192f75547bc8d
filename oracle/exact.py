"""Exact derivatives of 1/r at integer points, by symbolic differentiation.

TEST INFRASTRUCTURE ONLY. This is an independent derivation used to pin the
oracle's closed form (Hobson's formula in ``fmm.dtensor``): it never uses
that formula. Writing D_m = P_m(x, y, z) / r^(2|m|+1) with P_m a homogeneous
integer polynomial of degree |m|, the quotient rule gives

    P_{m + e_x} = r^2 dP_m/dx - (2|m| + 1) x P_m,     P_0 = 1,

and likewise for y and z. At an integer point d the value is the integer
P_m(d) divided by (|d|^2)^|m| sqrt(|d|^2), which is rounded once to float64
from a 60-digit decimal evaluation.
"""

from decimal import Decimal, getcontext

_poly_cache = {(0, 0, 0): {(0, 0, 0): 1}}


def _mul_r2(poly):
    out = {}
    for (a, b, c), v in poly.items():
        for e in ((2, 0, 0), (0, 2, 0), (0, 0, 2)):
            key = (a + e[0], b + e[1], c + e[2])
            out[key] = out.get(key, 0) + v
    return out


def _diff(poly, axis):
    out = {}
    for mono, v in poly.items():
        if mono[axis] == 0:
            continue
        key = list(mono)
        key[axis] -= 1
        key = tuple(key)
        out[key] = out.get(key, 0) + v * mono[axis]
    return out


def _mul_var(poly, axis, factor):
    out = {}
    for mono, v in poly.items():
        key = list(mono)
        key[axis] += 1
        key = tuple(key)
        out[key] = out.get(key, 0) + v * factor
    return out


def _add(p, q):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, 0) + v
    return {k: v for k, v in out.items() if v != 0}


def numerator_poly(m):
    """Integer polynomial P_m with d^m (1/r) = P_m / r^(2|m|+1), as {exponents: coeff}."""
    m = tuple(m)
    if m in _poly_cache:
        return _poly_cache[m]
    # differentiate the lexicographically preceding multi-index along one axis
    axis = 0 if m[0] > 0 else (1 if m[1] > 0 else 2)
    prev = list(m)
    prev[axis] -= 1
    prev = tuple(prev)
    P = numerator_poly(prev)
    n = sum(prev)
    res = _add(_mul_r2(_diff(P, axis)), _mul_var(P, axis, -(2 * n + 1)))
    _poly_cache[m] = res
    return res


def numerator_at(m, d):
    """P_m(d) for an integer point d (exact integer)."""
    x, y, z = (int(v) for v in d)
    return sum(v * x ** a * y ** b * z ** c for (a, b, c), v in numerator_poly(m).items())


def dtensor_exact(m, d):
    """d^m (1/r) at the integer point d, correctly rounded to float64."""
    getcontext().prec = 60
    r2 = sum(int(v) ** 2 for v in d)
    n = sum(m)
    num = Decimal(numerator_at(m, d))
    val = num / (Decimal(r2) ** n * Decimal(r2).sqrt())
    return float(val)
