"""GPU parity of the shear 3PCF multipoles (the order-N construction at
N = 3, read from the stage (a) records) against the FP64 oracle.

Bars as for the 4PCF (helpers.assert_parity over all bin pairs and the
diagonal b1 = b2 alone, where the same-neighbour terms are removed): <= 1e-10
normwise per component in the FP64 path, <= 1e-5 in the mixed paths
(binary32 stage (a); the 3PCF contraction is binary64 in both), with the
largest-element, element-wise and term-scale bars.  At the full 1e6-galaxy size the oracle takes sampled
centres; the all-centre result is checked by the Theta_1 <-> Theta_2
relabelling relations, which hold at any size.
"""
import functools

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_parity, rel_per_mu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp16": 1e-5, "bf16": 1e-5}
M3 = 6   # 3PCF multipoles |n| <= 6 on the 2000-galaxy case


@pytest.fixture(scope="module")
def fp():
    import paper_2509_07974_amd as m
    m.lib()
    return m


@functools.lru_cache(None)
def c0():
    cat, edges, _, _ = synth.workload("uniform-2k")
    return cat, edges


@functools.lru_cache(None)
def c0_ref(distinct=True):
    cat, edges = c0()
    return oracle.upsilon3(*cat.arrays(), edges, M3, distinct=distinct)


@functools.lru_cache(None)
def c0_bound():
    cat, edges = c0()
    return oracle.abs_bound(*cat.arrays(), edges, order=3)


@functools.lru_cache(None)
def small(n=400, seed=21):
    cat, _ = c0()
    idx = np.random.default_rng(seed).choice(cat.n, n, replace=False)
    return synth.subset(cat, idx)


@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_3pcf_c0_distinct(fp, prec):
    cat, edges = c0()
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision=prec)
    assert got.shape == (5, 4, 4, 2 * M3 + 1)
    assert_parity(got, c0_ref(True), prec, c0_bound(), nbin=2, label="3pcf c0")


def test_3pcf_c0_raw_fp64(fp):
    cat, edges = c0()
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp64",
                                      subtract_degenerate=False)
    assert_parity(got, c0_ref(False), "fp64", c0_bound(), nbin=2, label="3pcf c0 raw")
    # the same-neighbour terms sit on the diagonal b1 == b2 only
    dist = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp64")
    off = ~np.eye(4, dtype=bool)
    assert np.array_equal(got[:, off], dist[:, off])


@pytest.mark.parametrize("m", [0, 1, 5, 32])
def test_3pcf_multipole_orders(fp, m):
    """Even and odd m (records of order ceil(m/2)), down to 0 and up to the
    largest supported."""
    c = small()
    _, edges = c0()
    got = fp.estimate_3pcf_multipoles(*c.arrays(), edges, m, precision="fp64")
    ref = oracle.upsilon3(*c.arrays(), edges, m)
    S = oracle.abs_bound(*c.arrays(), edges, order=3)
    assert_parity(got, ref, "fp64", S, nbin=2, label=f"3pcf m {m}")


@pytest.mark.parametrize("nb", [1, 9, 16])
def test_3pcf_bin_counts(fp, nb):
    c = small()
    edges = synth.log_edges(1.0, 30.0, nb)
    ref = oracle.upsilon3(*c.arrays(), edges, 3)
    S = oracle.abs_bound(*c.arrays(), edges, order=3)
    for prec in ("fp64", "fp16", "bf16"):
        got = fp.estimate_3pcf_multipoles(*c.arrays(), edges, 3, precision=prec)
        assert_parity(got, ref, prec, S, nbin=2, label=f"3pcf nb {nb}")


def test_3pcf_tiles_match_single_tile(fp):
    cat, edges = c0()
    one = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16")
    many = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16", tile_centers=333)
    assert np.all(rel_per_mu(many, one) < 1e-13)


def test_3pcf_centre_subset(fp):
    cat, edges = c0()
    idx = np.random.default_rng(3).choice(cat.n, 150, replace=False)
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp64", centers=idx)
    ref = oracle.upsilon3(*cat.arrays(), edges, M3, centers=idx)
    assert_parity(got, ref, "fp64", oracle.abs_bound(*cat.arrays(), edges, idx, order=3), nbin=2,
                  label="3pcf subset")


def test_3pcf_empty_and_out_of_range(fp):
    _, edges = c0()
    z = np.zeros(0)
    got = fp.estimate_3pcf_multipoles(z, z, z, z, z, edges, 3)
    assert got.shape == (5, 4, 4, 7) and not np.any(got)
    # two galaxies farther apart than the outer edge: no pair, all zeros
    x = np.array([0.0, 100.0])
    got = fp.estimate_3pcf_multipoles(x, x, x * 0 + .1, x * 0, x * 0 + 1, edges, 3)
    assert not np.any(got)


def test_3pcf_hand_example_on_gpu(fp):
    """The three-galaxy example worked by hand from the projected shears of
    Sect. 2.1 (tests/test_oracle3.py): centre (0, 0) w 2 gamma_c 0.1i,
    neighbours (1.5, 0) w 1 gamma_c 0.2i and (0, 3) w 1 gamma_c 0.3i, bins
    [1, 2), [2, 4): Gamma_0..3 = -0.012, -0.012, +0.012, +0.012 and N = 2
    times (-i)^n at (bin 0, bin 1), i^n at (bin 1, bin 0)."""
    x = np.array([0.0, 1.5, 0.0]); y = np.array([0.0, 0.0, 3.0])
    g1 = np.zeros(3); g2 = np.array([0.1, 0.2, 0.3]); w = np.array([2.0, 1.0, 1.0])
    edges = np.array([1.0, 2.0, 4.0])
    P = [-0.012, -0.012, 0.012, 0.012, 2.0]
    # binary32 stage (a): the records' 1e-6 bar (4e-7 measured)
    for prec, tol in (("fp64", 1e-15), ("fp16", 1e-6)):
        u = fp.estimate_3pcf_multipoles(x, y, g1, g2, w, edges, 3, precision=prec, centers=[0])
        for mu in range(5):
            for n in range(-3, 4):
                assert abs(u[mu, 0, 1, n + 3] - P[mu] * (-1j) ** n) < tol * max(1, abs(P[mu])), (prec, mu, n)
                assert abs(u[mu, 1, 0, n + 3] - P[mu] * (1j) ** n) < tol * max(1, abs(P[mu])), (prec, mu, n)


def test_3pcf_device_inputs_match_host(fp):
    import torch
    cat, edges = c0()
    dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
    got = fp.estimate_3pcf_multipoles(*dev, edges, M3, precision="fp16")
    host = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, M3, precision="fp16")
    assert np.array_equal(got.cpu().numpy(), host)


@functools.lru_cache(None)
def grf1m():
    cat, edges, _, _ = synth.workload("grf-1m")
    return cat, edges


@functools.lru_cache(None)
def grf1m_sample():
    cat, edges = grf1m()
    idx = np.random.default_rng(12).choice(cat.n, 8, replace=False)
    return idx, oracle.upsilon3(*cat.arrays(), edges, 10, centers=idx), \
        oracle.abs_bound(*cat.arrays(), edges, idx, order=3)


@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_3pcf_grf1m_sampled_centres(fp, prec):
    """Full-size 1e6-galaxy GRF catalogue, 12 bins, 3PCF multipoles |n| <= 10:
    seeded centres with every galaxy as neighbour."""
    cat, edges = grf1m()
    idx, ref, S = grf1m_sample()
    got = fp.estimate_3pcf_multipoles(*cat.arrays(), edges, 10, precision=prec, centers=idx)
    assert_parity(got, ref, prec, S, nbin=2, label="3pcf grf-1m")


def test_3pcf_grf1m_all_centres_relabelling(fp):
    """All 1e6 centres, mixed path: Upsilon_0, Upsilon_1 and N equal
    themselves and Upsilon_2 equals Upsilon_3 under (b1, b2, n) ->
    (b2, b1, -n); the two sides are formed from different record entries."""
    import torch
    cat, edges = grf1m()
    dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
    u = fp.estimate_3pcf_multipoles(*dev, edges, 10, precision="fp16").cpu().numpy()
    sw = np.transpose(u, (0, 2, 1, 3))[..., ::-1]
    for a, b in ((0, 0), (1, 1), (2, 3), (4, 4)):
        err = np.linalg.norm(u[a] - sw[b]) / np.linalg.norm(u[a])
        assert err < 1e-12, (a, b, err)
    assert np.linalg.norm(u[4][..., ::-1] - np.conj(u[4])) / np.linalg.norm(u[4]) < 1e-12
