"""GPU parity at the largest workload: 2400'x2400' lognormal catalogue,
N = 1e7, 16 log bins over 0.5-200', nmax 15, mixed fp16 path with the
centre tiling of the full run.  The oracle computes a seeded sample of
centres one by one (all 1e7 galaxies stay neighbours); the GPU path runs the
same centres.  Tiling is checked as a property: the same centre set split
into ragged tiles gives the same result as one tile."""
import functools
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_parity, rel_per_mu

pytestmark = pytest.mark.gpu
PROCS = max(1, min(16, os.cpu_count() or 1))   # the host share of one GPU


@functools.lru_cache(None)
def c4():
    return synth.workload("lognormal-10m")


@pytest.fixture(scope="module")
def fp():
    import paper_2509_07974_amd as m
    m.lib()
    return m


@functools.lru_cache(None)
def c4_sample():
    """64 seeded centres (two 32-centre chunks), every galaxy a neighbour:
    the oracle and its term scale in a process pool (about half a minute)."""
    cat, edges, nmax, _ = c4()
    idx = np.sort(np.random.default_rng(44).choice(cat.n, 64, replace=False))
    ref = oracle.upsilon_parallel(*cat.arrays(), edges, nmax, centers=idx, processes=PROCS, parts=PROCS)
    S = oracle.abs_bound_parallel(*cat.arrays(), edges, idx, processes=PROCS)
    return idx, ref, S


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp64"])
def test_lognormal10m_sampled_centres(fp, prec):
    cat, edges, nmax, _ = c4()
    idx, ref, S = c4_sample()
    got = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision=prec, centers=idx)
    assert_parity(got, ref, prec, S, label="lognormal-10m 64 centres")
    counts, _, _ = fp.debug_multipoles(*cat.arrays(), edges, nmax, centers=idx)
    assert np.array_equal(counts, oracle.bin_counts(cat.x, cat.y, edges, idx))


def test_lognormal10m_tiles_match_single_tile(fp):
    cat, edges, nmax, _ = c4()
    idx = np.random.default_rng(45).choice(cat.n, 3000, replace=False)
    one = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp64", centers=idx)
    many = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp64", centers=idx,
                                       tile_centers=777)
    assert np.all(rel_per_mu(many, one) < 1e-13)


C4_TREE = (0.5, 3, 40.0)   # grids of 0.5', 1', 2', r_min 40


@functools.lru_cache(None)
def c4_tree_sample():
    cat, edges, nmax, _ = c4()
    idx = np.sort(np.random.default_rng(17).choice(cat.n, 4, replace=False))
    return idx, oracle.upsilon_tree(*cat.arrays(), edges, nmax, *C4_TREE, centers=idx)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_lognormal10m_tree_sampled_centres(fp, prec):
    """The tree approximation at the largest workload (reduced catalogues on
    0.5', 1', 2' grids, r_min 40: the six outer bins from reduced
    catalogues, two of them on each grid; nmax 15): four seeded centres
    against the tree oracle."""
    cat, edges, nmax, _ = c4()
    assert oracle.tree_levels(edges, *C4_TREE) == [0] * 10 + [1, 1, 2, 2, 3, 3]
    idx, ref = c4_tree_sample()
    print(f"tree lognormal-10m centres {idx.tolist()} {prec}", flush=True)
    got = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision=prec, tree=C4_TREE, centers=idx)
    assert_parity(got, ref, prec, label="tree lognormal-10m")


@functools.lru_cache(None)
def c4_sample3(m=30):
    cat, edges, _, _ = c4()
    idx = np.sort(np.random.default_rng(19).choice(cat.n, 8, replace=False))
    return idx, oracle.upsilon3(*cat.arrays(), edges, m, centers=idx), \
        oracle.abs_bound(*cat.arrays(), edges, idx, order=3)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_lognormal10m_3pcf_sampled_centres(fp, prec):
    """The shear 3PCF at the largest workload, multipoles |n| <= 30 (records
    of order 15), eight seeded centres with every galaxy as neighbour (both
    mixed precisions take the same binary32 records here)."""
    cat, edges, _, _ = c4()
    idx, ref, S = c4_sample3()
    print(f"3pcf lognormal-10m m=30 centres {idx.tolist()} {prec}", flush=True)
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, 30, precision=prec, centers=idx)
    assert_parity(got, ref, prec, S, nbin=2, label="3pcf lognormal-10m")
