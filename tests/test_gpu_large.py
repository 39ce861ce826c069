"""GPU parity at the largest workload: 2400'x2400' lognormal catalogue,
N = 1e7, 16 log bins over 0.5-200', nmax 15, mixed fp16 path with the
centre tiling of the full run.  The oracle computes a seeded sample of
centres one by one (all 1e7 galaxies stay neighbours); the GPU path runs the
same centres.  Tiling is checked as a property: the same centre set split
into ragged tiles gives the same result as one tile."""
import functools

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_per_mu

pytestmark = pytest.mark.gpu


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
    cat, edges, nmax, _ = c4()
    idx = np.random.default_rng(44).choice(cat.n, 6, replace=False)
    return idx, oracle.upsilon(*cat.arrays(), edges, nmax, centers=idx)


@pytest.mark.parametrize("prec,tol", [("fp16", 1e-5), ("fp64", 1e-10)])
def test_lognormal10m_sampled_centres(fp, prec, tol):
    cat, edges, nmax, _ = c4()
    idx, ref = c4_sample()
    got = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision=prec, centers=idx)
    err = rel_per_mu(got, ref)
    assert np.all(err < tol), err
    counts, _, _ = fp.debug_multipoles(*cat.arrays(), edges, nmax, centers=idx)
    assert np.array_equal(counts, oracle.bin_counts(cat.x, cat.y, edges, idx))


def test_lognormal10m_tiles_match_single_tile(fp):
    cat, edges, nmax, _ = c4()
    idx = np.random.default_rng(45).choice(cat.n, 3000, replace=False)
    one = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp64", centers=idx)
    many = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp64", centers=idx,
                                       tile_centers=777)
    assert np.all(rel_per_mu(many, one) < 1e-13)
