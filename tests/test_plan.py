"""The stage (b) contraction plan (host logic, no GPU).

Upsilon_{mu,(n2,n3)}(b1, b2, b3) = sum_i x_i A(b1) B(b2) C(b3) (Sect. 3.1).
The library forms each distinct product of three blocks once, as a row block
times a pair of column blocks over all bin triples, and reads every
(mu, n2, n3) with the same blocks at permuted bins (the radial symmetry of
Table 2).  These tests check the plan the library reports against the
oracle's own factor table: every (mu, n2, n3) gets exactly its x and its
three blocks, each at the bin the factor table puts it, and no distinct
product is formed twice.
"""
import numpy as np
import pytest

from helpers import ensure_built

import oracle.estimator as est

X_KIND = {"g": 0, "gc": 1, "w": 2}
FAMILY = {"G": 0, "W": 1}


def factor_blocks(mu, n2, n3):
    """x kind and the (family, conjugated, order) of the blocks at Theta_1, 2, 3."""
    x, *fac = est.FACTORS[mu]
    blocks = [(FAMILY[f], int(cj), a * n2 + b * n3 + c) for f, cj, (a, b, c) in fac]
    return X_KIND[x], blocks


@pytest.fixture(scope="module")
def lib():
    return ensure_built()


@pytest.mark.parametrize("nmax", [0, 1, 3, 8, 10, 15, 16])
def test_plan_reads_every_correlator_at_its_blocks(lib, nmax):
    import paper_2509_07974_amd as fp
    plan, nitems = fp.debug_pair_plan(nmax)
    nn = 2 * nmax + 1
    assert plan.shape == (9, nn, nn, 16)
    item_cols = {}
    row_of = {}
    multisets = set()
    for mu in range(9):
        for i2, n2 in enumerate(range(-nmax, nmax + 1)):
            for i3, n3 in enumerate(range(-nmax, nmax + 1)):
                v = [int(t) for t in plan[mu, i2, i3]]
                x, blocks = factor_blocks(mu, n2, n3)
                assert v[0] == x
                roles = [tuple(v[1:4]), tuple(v[4:7]), tuple(v[7:10])]
                src = v[10:13]
                # the three roles take the three bins once each ...
                assert sorted(src) == [0, 1, 2]
                # ... and the block at each role is the factor table's block at that bin
                for role, s in zip(roles, src):
                    assert role == blocks[s], (mu, n2, n3, roles, src, blocks)
                item, blk, nblk = v[13:16]
                assert 0 <= item < nitems and 0 <= blk < nblk
                # one column pair per work item, one row block per (item, block)
                assert item_cols.setdefault(item, (roles[1], roles[2])) == (roles[1], roles[2])
                assert row_of.setdefault((item, blk), (x, roles[0])) == (x, roles[0])
                multisets.add((x, tuple(sorted(blocks))))
    # every distinct product of three blocks is formed exactly once
    assert len(row_of) == len(multisets)
    # the symmetry pays: fewer row blocks than (mu, n2, n3) from nmax 1 on
    if nmax >= 1:
        assert len(row_of) < 9 * nn * nn


def test_plan_rejects_bad_arguments(lib):
    import ctypes as C
    out = np.zeros(16 * 9, dtype=np.int32)
    assert lib.fpcf4_debug_pair_plan(-1, out.ctypes.data, None) != 0
    assert lib.fpcf4_debug_pair_plan(17, out.ctypes.data, None) != 0
    assert lib.fpcf4_debug_pair_plan(0, None, None) != 0
    n = C.c_int64(0)
    assert lib.fpcf4_debug_pair_plan(0, out.ctypes.data, C.byref(n)) == 0 and n.value > 0


# ---------------------------------------------------------------------------
# degenerate-term sums (App. A.1, Table 1)
# ---------------------------------------------------------------------------
E_FAMILY = {"Q": 2, "A": 3, "V": 4, "T": 5, "M": 6, "U": 7}


def corr_terms(mu, nmax):
    """Per slot of the correction buffer (orders n3 of Theta_1 = Theta_2,
    orders n2 of Theta_1 = Theta_3, orders n2 + n3 of Theta_2 = Theta_3, the
    triple term): x, the Table 1 block (family, order) and the remaining
    factor (family, conjugated, order), from the oracle's tables."""
    x, A, B, C = est.FACTORS[mu]
    c12, c13, c23, t = est.TABLE1[mu]
    out = []
    for kind, (eb, fb, orders) in enumerate(((c12, C, range(-nmax, nmax + 1)),
                                            (c13, B, range(-nmax, nmax + 1)),
                                            (c23, A, range(-2 * nmax, 2 * nmax + 1)))):
        for o in orders:
            # the sum's order index: n3 (kind 0), n2 (kind 1), s = n2 + n3 (kind 2)
            n2, n3 = {0: (0, o), 1: (o, 0), 2: (o, 0)}[kind]
            ea, ebb, ec = eb[1]
            fa, fbb, fc = fb[2]
            if kind == 2:   # both orders depend on s = n2 + n3 only (a = b)
                assert ea == ebb and fa == fbb
            e = (E_FAMILY[eb[0]], ea * n2 + ebb * n3 + ec)
            f = (FAMILY[fb[0]], int(fb[1]), fa * n2 + fbb * n3 + fc)
            out.append((X_KIND[x], e, f))
    out.append((X_KIND[x], (E_FAMILY[t[0]], t[1][2]), None))
    return out


@pytest.mark.parametrize("nmax", [0, 1, 3, 8, 10, 15, 16])
def test_corr_plan_forms_each_table1_sum_once(lib, nmax):
    import paper_2509_07974_amd as fp
    plan, nsums = fp.debug_corr_plan(nmax)
    assert plan.shape == (9, 8 * nmax + 4, 8)
    key_of_sum = {}
    keys = set()
    for mu in range(9):
        terms = corr_terms(mu, nmax)
        assert len(terms) == plan.shape[1]
        for slot, (x, e, f) in enumerate(terms):
            v = [int(t) for t in plan[mu, slot]]
            assert v[0] == x, (mu, slot)
            assert (v[1], v[2]) == e, (mu, slot, v, e)
            if f is None:
                assert v[3] == -1
            else:
                assert (v[3], v[4], v[5]) == f, (mu, slot, v, f)
            key = (x, e, f)
            keys.add(key)
            # one distinct sum per (x, E, F), and no two keys share a sum
            assert key_of_sum.setdefault(v[6], key) == key
            assert 0 <= v[6] < nsums
    assert len(key_of_sum) == len(keys) == nsums
    # the three pair kinds share sums: fewer than the 9 (8 nmax + 3) pair slots
    if nmax >= 1:
        assert nsums < 9 * (8 * nmax + 4)
