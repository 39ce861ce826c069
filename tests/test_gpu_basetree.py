"""GPU parity of the BaseTree, Tree and DoubleTree approximations of the
shear 3PCF (App. F.3, algorithmic implementation) against their FP64
oracle, through the C ABI (mixed paths; the bars of helpers.assert_parity
without the term-scale bar: the discrete catalogue's absolute sums do not
bound the pseudo-galaxy terms), and the limit in which they equal the
discrete 3PCF."""
import functools

import numpy as np
import pytest

import oracle
from oracle import basetree as bt
import synth
from helpers import assert_parity, rel_per_mu

pytestmark = pytest.mark.gpu
M3 = 6
BASE = (0.5, 2, 4.0)      # grids 0.5' and 1': the four 1-30' bins -> [0, 1, 2, 2]
TREE = (0.4, 2, 5.0)      # neighbour grids 0.4' and 0.8': -> [0, 1, 2, 2]


@pytest.fixture(scope="module")
def fp():
    import paper_2509_07974_amd as m
    m.lib()
    return m


@functools.lru_cache(None)
def c0(nb=4):
    cat, _, _, _ = synth.workload("uniform-2k")
    return cat, synth.log_edges(1.0, 30.0, nb)


@functools.lru_cache(None)
def c0_ref(nb=4, distinct=True, mode="base"):
    cat, edges = c0(nb)
    kw = {"base": {"base": BASE}, "tree": {"tree": TREE}, "double": {"base": BASE, "tree": TREE}}[mode]
    return bt.upsilon3_doubletree(*cat.arrays(), edges, M3, distinct=distinct, **kw)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_basetree_c0_matches_oracle(fp, prec):
    cat, edges = c0()
    assert oracle.tree_levels(edges, *BASE) == [0, 1, 2, 2]
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision=prec, base=BASE)
    assert_parity(got, c0_ref(), prec, nbin=2, label="basetree c0")
    # an approximation: not the discrete result
    exact = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision=prec)
    assert np.max(rel_per_mu(got, exact)) > 1e-4


def test_basetree_raw_sums(fp):
    cat, edges = c0()
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", base=BASE,
                                      subtract_degenerate=False)
    assert_parity(got, c0_ref(4, False), "fp16", nbin=2, label="basetree c0 raw")


def test_basetree_many_bins(fp):
    """17 bins (two bin tiles, ragged) spread over three grids."""
    cat, edges = c0(17)
    lv = oracle.tree_levels(edges, *BASE)
    assert lv[0] == 0 and lv[-1] == 2 and 1 in lv
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", base=BASE)
    assert_parity(got, c0_ref(17), "fp16", nbin=2, label="basetree 17 bins")


def test_basetree_without_grids_is_discrete(fp):
    cat, edges = c0()
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", base=(0.5, 2, 1e3))
    exact = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16")
    assert np.all(rel_per_mu(got, exact) < 1e-14)


def test_basetree_device_inputs_match_host(fp):
    import torch
    cat, edges = c0()
    host = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", base=BASE)
    dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
    got = fp.estimate_3pcf_multipoles(*dev, edges, M3, precision="fp16", base=BASE)
    assert np.all(rel_per_mu(got.cpu().numpy(), host) < 1e-14)


@pytest.mark.parametrize("mode", ["tree", "double"])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_tree_and_doubletree_c0_match_oracle(fp, mode, prec):
    cat, edges = c0()
    assert oracle.tree_levels(edges, *TREE) == [0, 1, 2, 2]
    kw = {"tree": {"tree": TREE}, "double": {"base": BASE, "tree": TREE}}[mode]
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision=prec, **kw)
    assert_parity(got, c0_ref(4, True, mode), prec, nbin=2, label=f"{mode} c0")
    raw = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision=prec, subtract_degenerate=False, **kw)
    assert_parity(raw, c0_ref(4, False, mode), prec, nbin=2, label=f"{mode} c0 raw")


def test_tree_3pcf_tiles_and_subsets(fp):
    """The tree alone keeps the tiled path: tiles add up, and a centre subset
    is the sum over those centres (additivity against the complement)."""
    cat, edges = c0()
    one = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", tree=TREE)
    many = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", tree=TREE,
                                       tile_centers=333)
    assert np.all(rel_per_mu(many, one) < 1e-6)
    idx = np.arange(0, cat.n, 3)
    rest = np.setdiff1d(np.arange(cat.n), idx)
    a = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", tree=TREE, centers=idx)
    b = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", tree=TREE, centers=rest)
    assert np.all(rel_per_mu(a + b, one) < 1e-6)
