"""Independent reference values for the oracle pins: derivatives of the
Newtonian Green's function -1/|r| by symbolic differentiation (sympy),
evaluated in 30-digit arithmetic (mpmath). Shares nothing with the oracle's
closed forms."""
import functools

import mpmath
import sympy as sp

from synthetic import moment_exponents

EXP4 = moment_exponents(4)
EXP3 = EXP4[:20]


@functools.lru_cache(maxsize=None)
def _derivative_functions(maxorder=4):
    x, y, z = sp.symbols("x y z", real=True)
    G = -1 / sp.sqrt(x ** 2 + y ** 2 + z ** 2)
    fns = []
    for a, b, c in moment_exponents(maxorder):
        d = G
        if a:
            d = sp.diff(d, x, a)
        if b:
            d = sp.diff(d, y, b)
        if c:
            d = sp.diff(d, z, c)
        fns.append(sp.lambdify((x, y, z), d, "mpmath"))
    return fns


def green_mp(r, order=4, dps=30):
    """d^gamma(-1/|r|) for |gamma| <= order at r (3 numbers), as mpf."""
    n = (order + 1) * (order + 2) * (order + 3) // 6
    with mpmath.workdps(dps):
        rx, ry, rz = (mpmath.mpf(float(v)) for v in r)
        return [f(rx, ry, rz) for f in _derivative_functions(max(4, order))[:n]]
