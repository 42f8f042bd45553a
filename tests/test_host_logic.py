"""Host-side logic of the library, on the CPU (no device call): the stencil
tables the kernels walk and the descriptor validation, pair counting and
launch order of a batched plan, against brute force with numpy."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import synthetic  # noqa: E402

ot = pytest.importorskip("paper_2303_08058_amd")


def brute_slot_pairs():
    """Pairs between the 8^3 targets (halo cells 8..15) and each neighbour
    block, from the criterion |d|^2 > 16 and |floor(j/2) - floor(i/2)|^2 <= 16."""
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], axis=1)
    ti = loc + 8
    out = []
    for slot in range(27):
        tj = loc + 8 * np.array([slot % 3, (slot // 3) % 3, slot // 9])
        d = tj[None] - ti[:, None]
        p = tj[None] // 2 - ti[:, None] // 2
        out.append(int(np.count_nonzero(((d * d).sum(-1) > 16) & ((p * p).sum(-1) <= 16))))
    return np.array(out)


def test_stencil_tables_match_brute_force():
    sp, off, rows = ot.ot_fmm_stencil_info()
    assert np.array_equal(sp, brute_slot_pairs())
    assert sp.sum() == 512 * 1799
    assert list(off) == [1799, 1799]
    # every (dz, dy) line of the stencil holds at most 2 x-intervals
    assert 0 < rows[0] <= 2 * 19 * 19 and 0 < rows[1] <= 2 * 19 * 19


def expected_pairs(batch):
    sp = brute_slot_pairs()
    present = np.asarray(batch["nbr"]) >= 0
    work = (present * sp[None, :]).sum(axis=1)
    return int(work.sum()), work


@pytest.mark.parametrize("n,frac,periodic", [(3, 0.5, False), (4, 0.3, True), (8, 0.2, True)])
def test_pair_counts_and_work_order(n, frac, periodic):
    batch = synthetic.lattice_batch(n, periodic=periodic)
    batch = synthetic.apply_missing(batch, frac, synthetic._rng(100 + n))
    pairs, work, order = ot.ot_fmm_count_pairs(batch)
    exp_pairs, exp_work = expected_pairs(batch)
    assert pairs == exp_pairs
    assert np.array_equal(work, exp_work)
    # launch order: a permutation, longest work first, ties in target order
    assert np.array_equal(np.sort(order), np.arange(batch["T"]))
    w = work[order]
    assert np.all(np.diff(w) <= 0)
    ties = np.diff(w) == 0
    assert np.all(np.diff(order)[ties] > 0)


def test_subset_targets_and_isolated_target():
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 0], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[1, :] = -1
    nbr[1, 13] = 0                       # only itself
    batch = {"S": 27, "T": 2, "tgt": tg, "nbr": nbr}
    pairs, work, order = ot.ot_fmm_count_pairs(batch)
    sp = brute_slot_pairs()
    assert work[1] == sp[13] and work[0] == sp.sum()
    assert pairs == sp.sum() + sp[13] and list(order) == [0, 1]


def _bad(batch, **kw):
    b = dict(batch)
    b.update(kw)
    with pytest.raises(ot.OtFmmError) as e:
        ot.ot_fmm_count_pairs(b)
    assert e.value.code == ot.OT_FMM_EINVAL


def test_descriptor_validation():
    batch = synthetic.lattice_batch(2, periodic=True)
    nbr = batch["nbr"].copy()
    nbr[0, 13] = 1
    _bad(batch, nbr=nbr)                                     # slot 13 is not the target
    nbr = batch["nbr"].copy()
    nbr[3, 4] = 8
    _bad(batch, nbr=nbr)                                     # out of range
    tgt = batch["tgt"].copy()
    tgt[1] = tgt[0]
    _bad(batch, tgt=tgt)                                     # repeated target
    _bad(batch, period=None)                                 # shift without period
    sh = batch["shift"].copy()
    sh[0, 0, 0] = -128
    _bad(batch, shift=sh)                                    # cannot be negated
    # two targets claiming the same (source, slot) relation: target 1 names
    # target 0's slot-0 neighbour in its own slot 0
    nbr = batch["nbr"].copy()
    nbr[1, 0] = nbr[0, 0]
    _bad(batch, nbr=nbr)
    # and a valid descriptor passes
    assert ot.ot_fmm_count_pairs(batch)[0] == 8 * 512 * 1799


def _piece_locality(order, batch, nxcd):
    """Fraction of the (item, neighbour item) relations whose two ends run on
    the same XCD (work-group b on XCD b % nxcd)."""
    xcd = np.empty(len(order), np.int64)
    xcd[order] = np.arange(len(order)) % nxcd
    tindex = -np.ones(batch["S"], np.int64)
    tindex[batch["tgt"]] = np.arange(batch["T"])
    same = total = 0
    for t in range(batch["T"]):
        for q in range(27):
            b = batch["nbr"][t, q]
            if q == 13 or b < 0 or tindex[b] < 0:
                continue
            total += 1
            same += xcd[t] == xcd[tindex[b]]
    return same / total


@pytest.mark.parametrize("periodic", [False, True])
def test_xcd_local_orders(periodic):
    batch = synthetic.apply_missing(synthetic.lattice_batch(8, periodic=periodic), 0.2, synthetic._rng(5))
    fl, rl, rloc = ot.ot_fmm_work_orders(batch, nxcd=8)
    for o, n in ((fl, batch["T"]), (rl, batch["S"]), (rloc, batch["S"])):
        assert np.array_equal(np.sort(o), np.arange(n))
    # the longest-first store order of the source-role pass: non-increasing work
    # (a store block's work = the pairs of the targets that see it)
    sp = brute_slot_pairs()
    rw = np.zeros(batch["S"], np.int64)
    for t in range(batch["T"]):
        for q in range(27):
            b = batch["nbr"][t, q]
            if b >= 0:
                rw[b] += sp[q]
    assert np.all(np.diff(rw[rl]) <= 0)
    # pieces are spatially compact: many neighbour relations stay on one XCD,
    # against ~1/8 for the longest-first order dealt round robin
    _, _, lpt = ot.ot_fmm_count_pairs(batch)
    loc, ref = _piece_locality(fl, batch, 8), _piece_locality(lpt, batch, 8)
    assert loc > 0.45 and ref < 0.3, (loc, ref)  # a 4^3 piece keeps at most 56% of its 26-neighbour relations
    # each XCD's piece carries about 1/8 of the work
    _, work, _ = ot.ot_fmm_count_pairs(batch)
    per = np.bincount(np.argsort(fl) % 8, weights=work, minlength=8)
    assert per.max() / per.min() < 1.05


def test_parent_lattice_keeps_the_fine_domain_length():
    """The parent level's periodic shift is the fine domain's length (centres
    stay in fine-cell units), and its node numbering is the octree's."""
    import synthetic
    for n in (4, 8):
        fine = synthetic.lattice_batch(n, periodic=True)
        par = synthetic.parent_lattice(n, periodic=True)
        assert np.array_equal(par["period"], fine["period"])
        ch = synthetic.octree_children(n)
        assert par["S"] == ch.shape[0] == (n // 2) ** 3
        # parent node P covers fine sub-grids 2p + {0,1} per axis
        m = n // 2
        for P in (0, m * m * m - 1, 1 + m):
            px, py, pz = P % m, (P // m) % m, P // (m * m)
            kids = sorted(int(c) for c in ch[P])
            want = sorted((2 * px + a) + n * (2 * py + b) + n * n * (2 * pz + c)
                          for c in (0, 1) for b in (0, 1) for a in (0, 1))
            assert kids == want
    assert synthetic.parent_lattice(4, periodic=False)["period"] is None
