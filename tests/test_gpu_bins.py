"""GPU parity beyond 16 radial bins, where the contraction kernels cut the
bins into tiles of at most 16 per bin dimension.

* The uniform 2000-galaxy catalogue at 17 and 33 log bins over 1-30' (tiles
  of 9 + 8 bins, ragged, and of 11 bins), nmax 3, every centre: the whole
  tensor against the oracle in all three precisions, bin counts bit-exact;
  the shear 3PCF at both, the tree approximation at 17 bins.
* grf-65bin, the binning of the paper's mock and survey measurements (65 log
  bins over 0.25-166.29', nmax 15), on 32 seeded centres: the 38 GB result
  stays on the device; 300 sampled bin triplets (random, coincident, on the
  tile edges) are compared with the oracle's sums at those triplets, and the
  natural components are streamed block by block with natural_blocks over
  all 65^3 triplets and compared where the blocks hold sampled triplets.
"""
import functools
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_parity, rel_per_mu

pytestmark = pytest.mark.gpu
PROCS = max(1, min(16, os.cpu_count() or 1))   # the host share of one GPU


@pytest.fixture(scope="module")
def fp():
    import paper_2509_07974_amd as m
    m.lib()
    return m


@functools.lru_cache(None)
def c0(nb):
    cat, _, nmax, _ = synth.workload("uniform-2k")
    return cat, synth.log_edges(1.0, 30.0, nb), nmax


@functools.lru_cache(None)
def c0_ref(nb):
    cat, edges, nmax = c0(nb)
    ref = oracle.upsilon_parallel(*cat.arrays(), edges, nmax, processes=PROCS)
    return ref, oracle.abs_bound_parallel(*cat.arrays(), edges, np.arange(cat.n), processes=PROCS)


@pytest.mark.parametrize("nb", [17, 33])
@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_many_bins_full_tensor(fp, nb, prec):
    cat, edges, nmax = c0(nb)
    ref, S = c0_ref(nb)
    got = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision=prec)
    assert_parity(got, ref, prec, S, label=f"c0 {nb} bins")


@pytest.mark.parametrize("nb", [17, 33])
def test_many_bins_counts_and_tiles(fp, nb):
    cat, edges, nmax = c0(nb)
    counts, _, _ = fp.debug_multipoles(*cat.arrays(), edges, nmax, precision="fp16")
    assert np.array_equal(counts, oracle.bin_counts(cat.x, cat.y, edges, range(cat.n)))
    one = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp16")
    many = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp16", tile_centers=613)
    assert np.all(rel_per_mu(many, one) < 1e-6)


@pytest.mark.parametrize("nb", [17, 33])
def test_many_bins_3pcf(fp, nb):
    cat, edges, _ = c0(nb)
    c = synth.subset(cat, np.random.default_rng(21).choice(cat.n, 400, replace=False))
    ref = oracle.upsilon3(*c.arrays(), edges, 6)
    S = oracle.abs_bound(*c.arrays(), edges, order=3)
    for prec in ("fp64", "fp16", "bf16"):
        got = fp.estimate_3pcf_multipoles(*c.arrays(), edges, 6, precision=prec)
        assert_parity(got, ref, prec, S, nbin=2, label=f"3pcf {nb} bins")


def test_device_inputs_and_centres_match_host(fp):
    import torch
    cat, edges, nmax = c0(17)
    idx = np.random.default_rng(12).choice(cat.n, 300, replace=False)
    host = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp64", centers=idx)
    dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
    got = fp.estimate_4pcf_multipoles(*dev, edges, nmax, precision="fp64", centers=idx)
    assert got.is_cuda
    assert np.all(rel_per_mu(got.cpu().numpy(), host) < 1e-14)
    got = fp.estimate_4pcf_multipoles(*dev, edges, nmax, precision="fp64",
                                      centers=torch.as_tensor(idx).cuda())
    assert np.all(rel_per_mu(got.cpu().numpy(), host) < 1e-14)


def test_many_bins_tree(fp):
    cat, edges, nmax = c0(17)
    tree = (0.5, 2, 10.0)
    levels = oracle.tree_levels(edges, *tree)
    assert levels[0] == 0 and levels[-1] == 2 and 1 in levels
    ref = oracle.upsilon_tree(*cat.arrays(), edges, nmax, *tree)
    got = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp16", tree=tree)
    assert_parity(got, ref, "fp16", label="tree 17 bins")


# --------------------------------------------------------------------------
# 65 bins, nmax 15
# --------------------------------------------------------------------------
NB65 = 65


@functools.lru_cache(None)
def g65():
    cat, edges, nmax, _ = synth.workload("grf-65bin")
    assert len(edges) - 1 == NB65 and nmax == 15
    return cat, edges, nmax


def triplets65():
    """240 random triplets (200 among the bins from 1.8' out: at 0.3
    galaxies per arcmin^2 most inner bins are empty), every kind of
    coincident bins, and triplets on both sides of each 13-bin tile edge."""
    rng = np.random.default_rng(47)
    t = [tuple(r) for r in rng.integers(20, NB65, size=(200, 3))]
    t += [tuple(r) for r in rng.integers(0, NB65, size=(40, 3))]
    for a, b in ((5, 40), (12, 13), (25, 26), (51, 64)):
        t += [(a, a, b), (a, b, a), (b, a, a), (a, a, a), (b, b, b)]
    edges = [0, 12, 13, 25, 26, 38, 39, 51, 52, 64]
    t += [tuple(rng.choice(edges, 3)) for _ in range(40)]
    return np.array(t, dtype=np.int64)


@functools.lru_cache(None)
def g65_ref():
    cat, edges, nmax = g65()
    idx = np.sort(np.random.default_rng(46).choice(cat.n, 32, replace=False))
    t = triplets65()
    ref = oracle.upsilon_triplets_parallel(*cat.arrays(), edges, nmax, t, idx, processes=PROCS)
    S = oracle.abs_bound_parallel(*cat.arrays(), edges, idx, processes=PROCS)
    return idx, t, ref, S[:, t[:, 0], t[:, 1], t[:, 2]]


def g65_device(fp, prec):
    import torch
    cat, edges, nmax = g65()
    idx = g65_ref()[0]
    dev = [torch.as_tensor(a, device="cuda") for a in cat.arrays()]
    got = fp.estimate_4pcf_multipoles(*dev, edges, nmax, precision=prec, centers=idx)
    assert tuple(got.shape) == (9, NB65, NB65, NB65, 31, 31) and got.is_cuda
    return got


def pick(ups, t):
    """The sampled triplets of a device result, selected on the host (the
    whole tensor is copied: 38 GB)."""
    return ups.cpu().numpy()[:, t[:, 0], t[:, 1], t[:, 2]]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_65_bins_nmax15_sampled(fp, prec):
    import torch
    idx, t, ref, S = g65_ref()
    eq = (t[:, 0] == t[:, 1]) | (t[:, 0] == t[:, 2]) | (t[:, 1] == t[:, 2])
    print(f"65 bins nmax 15 {prec}: estimate", flush=True)
    got = g65_device(fp, prec)
    sel = pick(got, t)
    # per-triplet summary first, so that a failure names its triplets
    err = np.abs(sel - ref).reshape(9, len(t), -1).max(axis=(0, 2))
    scale = np.maximum(S.max(axis=0), 1e-300)
    bad = np.nonzero(err > 1e-3 * scale)[0]
    print(f"65 bins {prec}: {bad.size} of {len(t)} triplets off; first:",
          [tuple(int(v) for v in t[k]) for k in bad[:12]], flush=True)
    assert_parity(sel, ref, prec, S, label="65 bins sampled triplets", eq=eq)
    if prec == "fp64":
        # the natural components of all 65^3 triplets, streamed in blocks,
        # checked at every 8th sampled triplet (the oracle's conversion costs
        # about half a second per triplet at 129 angular bins)
        nphi = 129
        t = t[::8]
        gref, nref = oracle.natural_components_selected(ref[:, ::8], nphi)
        lin = (t[:, 0] * NB65 + t[:, 1]) * NB65 + t[:, 2]
        seen = 0
        checked = np.zeros(len(t), dtype=bool)
        for tb, gam, nrm in fp.natural_blocks(got, nphi, block=8192):
            s0 = (tb[0, 0] * NB65 + tb[0, 1]) * NB65 + tb[0, 2]
            assert s0 == seen
            seen += tb.shape[0]
            inb = np.nonzero((lin >= s0) & (lin < seen))[0]
            if inb.size:
                pos = torch.as_tensor(lin[inb] - s0, device=gam.device)
                g = gam[:, pos].cpu().numpy()
                n = nrm[pos].cpu().numpy()
                # against the scale of all checked triplets: some hold only
                # the rounding residue of an empty angular bin
                assert np.linalg.norm(n - nref[inb]) <= 1e-10 * np.linalg.norm(nref)
                # Gamma = Ubar / Nbar where Nbar is well above its rounding
                # error (1e-16 of the largest): relative error below 1e-12
                ok = np.abs(nref[inb]) > 1e-4 * np.abs(nref).max()
                d = (g - gref[:, inb])[:, ok]
                assert np.linalg.norm(d) <= 1e-10 * max(np.linalg.norm(gref[:, inb][:, ok]), 1e-300)
                checked[inb] = True
            del gam, nrm
        assert seen == NB65 ** 3 and checked.all()
    del got
    torch.cuda.empty_cache()


def test_65_bins_counts(fp):
    cat, edges, nmax = g65()
    idx = g65_ref()[0]
    counts, _, _ = fp.debug_multipoles(*cat.arrays(), edges, nmax, precision="fp16", centers=idx)
    assert np.array_equal(counts, oracle.bin_counts(cat.x, cat.y, edges, idx))
    assert (counts[:, 30:] > 0).all()


# --------------------------------------------------------------------------
# the largest bin count
# --------------------------------------------------------------------------
NBMAX = 128


@functools.lru_cache(None)
def cmax():
    """uniform-2k with 128 log bins over 5-30' (8 tiles of 16 bins), nmax 2,
    200 seeded centres, 160 sampled triplets (random, coincident, tile edges)."""
    cat, _, _, _ = synth.workload("uniform-2k")
    edges = synth.log_edges(5.0, 30.0, NBMAX)
    rng = np.random.default_rng(49)
    idx = np.sort(rng.choice(cat.n, 200, replace=False))
    t = [tuple(r) for r in rng.integers(0, NBMAX, size=(120, 3))]
    for a, b in ((15, 16), (63, 64), (0, 127)):
        t += [(a, a, b), (a, b, a), (b, a, a), (a, a, a), (b, b, b)]
    t += [tuple(rng.choice([0, 15, 16, 31, 32, 111, 112, 127], 3)) for _ in range(25)]
    t = np.array(t, dtype=np.int64)
    ref = oracle.upsilon_triplets_parallel(*cat.arrays(), edges, 2, t, idx, processes=PROCS)
    S = oracle.abs_bound(*cat.arrays(), edges, idx)
    return cat, edges, idx, t, ref, S[:, t[:, 0], t[:, 1], t[:, 2]]


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_max_bins_sampled(fp, prec):
    import torch
    cat, edges, idx, t, ref, S = cmax()
    assert np.abs(ref).max() > 0
    dev = [torch.as_tensor(a, device="cuda") for a in cat.arrays()]
    got = fp.estimate_4pcf_multipoles(*dev, edges, 2, precision=prec, centers=idx)
    assert tuple(got.shape) == (9, NBMAX, NBMAX, NBMAX, 5, 5)
    sel = pick(got, t)
    del got
    torch.cuda.empty_cache()
    eq = (t[:, 0] == t[:, 1]) | (t[:, 0] == t[:, 2]) | (t[:, 1] == t[:, 2])
    assert_parity(sel, ref, prec, S, label="128 bins sampled triplets", eq=eq)


def test_max_bins_3pcf(fp):
    cat, edges, idx, _, _, _ = cmax()
    c = synth.subset(cat, np.random.default_rng(50).choice(cat.n, 300, replace=False))
    ref = oracle.upsilon3(*c.arrays(), edges, 4)
    S = oracle.abs_bound(*c.arrays(), edges, order=3)
    for prec in ("fp64", "fp16"):
        got = fp.estimate_3pcf_multipoles(*c.arrays(), edges, 4, precision=prec)
        assert_parity(got, ref, prec, S, nbin=2, label="3pcf 128 bins")
    with pytest.raises(fp.Fpcf4Error):
        fp.estimate_3pcf_multipoles(*c.arrays(), synth.log_edges(5.0, 30.0, NBMAX + 1), 4, precision="fp16")
