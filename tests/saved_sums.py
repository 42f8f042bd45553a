"""The saved target-side sums of the two-launch step against the oracle
(shared by the GPU tests): the saved component g = a + e_k of a target cell
is the oracle's target-side derivative dL_a(i)/dX_i,k (of the total-order
or, full=True, of the full truncation's L)."""
import numpy as np

import oracle
from parity import assert_parity

TOL = 1e-12


def saved_index():
    """(a, k) of each of the 24 saved components g = a + e_k (orders 1..4,
    z exponent below 2, graded lexicographic), and their order groups."""
    exps20 = [tuple(oracle.multi_index(g)) for g in range(20)]
    idx20 = {e: g for g, e in enumerate(exps20)}
    kept = []
    for n in range(1, 5):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                c = n - a - b
                if c < 2:
                    kept.append((a, b, c))
    assert len(kept) == 24
    pairs = []
    for e in kept:
        k = 0 if e[0] > 0 else (1 if e[1] > 0 else 2)
        al = list(e)
        al[k] -= 1
        pairs.append((idx20[tuple(al)], k))
    groups = [[i for i, e in enumerate(kept) if sum(e) == n] for n in range(1, 5)]
    return pairs, groups


def saved_reference(batch, M, X, tsel=None, full=False):
    """The oracle's values of the saved sums for targets tsel, (24, n*512),
    and the magnitudes of their terms."""
    D, A = oracle.batched_forward_tgrad(batch, M, X, tsel=tsel, want_abs=True, full=full)
    pairs, _ = saved_index()
    return (np.stack([D[a, k] for a, k in pairs]), np.stack([A[a, k] for a, k in pairs]))


def check_saved(got, batch, M, X, what, tsel=None, full=False):
    ref, A = saved_reference(batch, M, X, tsel, full)
    _, groups = saved_index()
    return assert_parity(got, ref, TOL, groups=groups, what=what, A=A)
