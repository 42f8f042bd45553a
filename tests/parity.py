"""Parity criterion shared by the GPU tests.

For every sub-grid and every group of components (the 20 outputs grouped by
order 0..3; the 3 position-gradient components as one group):
    max |got - ref| <= tol * D,    D = max |ref|  over that sub-grid's cells.
Componentwise relative error is not used: components that cancel (e.g. a
dipole-like output on a symmetry plane) have no meaningful relative error.

Where the oracle also supplies A, the sum of the magnitudes of the terms of
each output, the denominator is D = max(max|ref|, 1e-2 * max A): in sub-grids
whose outputs cancel by more than a factor of 100 (near-uniform density
regions, measured up to ~600 for second-order outputs), 1e-12 of max|ref|
would be below the FP64 rounding noise of any reordered sum of the same
terms; there the bound is 1e-14 of the term magnitudes instead.
"""
import numpy as np

ORDER_GROUPS_20 = [[0], [1, 2, 3], list(range(4, 10)), list(range(10, 20))]
GROUPS_3 = [[0, 1, 2]]


def parity_report(got, ref, tol=1e-12, groups=None, A=None):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    ncomp, n = ref.shape
    assert n % 512 == 0
    if groups is None:
        groups = ORDER_GROUPS_20 if ncomp == 20 else GROUPS_3
    nsub = n // 512
    worst = 0.0
    worst_plain = 0.0
    bad = []
    for g in groups:
        r = ref[g].reshape(len(g), nsub, 512)
        d = np.abs(got[g].reshape(len(g), nsub, 512) - r)
        scale = np.abs(r).max(axis=(0, 2))
        err = d.max(axis=(0, 2))
        plain = np.where(scale > 0, err / np.where(scale > 0, scale, 1.0),
                         np.where(err > 0, np.inf, 0.0))
        worst_plain = max(worst_plain, float(plain.max()))
        if A is not None:
            a = np.asarray(A, np.float64)[g].reshape(len(g), nsub, 512).max(axis=(0, 2))
            scale = np.maximum(scale, 1e-2 * a)
        ratio = np.where(scale > 0, err / np.where(scale > 0, scale, 1.0),
                         np.where(err > 0, np.inf, 0.0))
        worst = max(worst, float(ratio.max()))
        for s in np.nonzero(ratio > tol)[0][:5]:
            bad.append((g[0], int(s), float(ratio[s])))
    return worst, worst_plain, bad


def assert_parity(got, ref, tol=1e-12, groups=None, what="", A=None):
    worst, worst_plain, bad = parity_report(got, ref, tol, groups, A)
    assert not bad, "%s: parity %.3e > %.1e at (first comp, sub-grid, ratio) %s" % (
        what, worst, tol, bad)
    if A is not None:
        print("%s: worst %.2e (plain max|ref| denominator: %.2e)" % (what, worst, worst_plain))
    return worst
