"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force
quadruplet enumeration of the definitions, a hand-computed example, the
paper's Table 2, exact invariances, integer closed forms and a library
pair counter.  ``test_planted_mistakes_are_caught`` plants plausible errors
in the oracle's tables and shows the brute-force pin catches each of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import estimator as est
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    """Normwise relative error per correlator (Frobenius)."""
    return np.array([np.linalg.norm(a[m] - b[m]) / max(np.linalg.norm(b[m]), 1e-300)
                     for m in range(a.shape[0])])


def tiny(seed, n=10, side=10.0):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, side, n), rng.uniform(0, side, n), rng.normal(0, .3, n),
            rng.normal(0, .3, n), rng.uniform(.5, 1.5, n))


TINY_EDGES = np.array([0.5, 3.0, 6.0, 15.0])


# --------------------------------------------------------------------------
# Multipole route == quadruplet definition (Sect. 3, 3.1, App. A.1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("distinct", [False, True])
def test_oracle_equals_brute_force_tiny(seed, distinct):
    cat = tiny(seed, n=9 + seed)
    a = oracle.upsilon(*cat, TINY_EDGES, 2, distinct=distinct)
    b = oracle.brute_upsilon(*cat, TINY_EDGES, 2, distinct=distinct)
    assert np.all(rel(a, b) < 1e-12)


def test_oracle_equals_brute_force_uniform2k_subset():
    """The seeded N=60 subset of the 60'x60' uniform catalogue, 4 bins, nmax 3."""
    cat, edges, nmax, _ = synth.workload("uniform-2k")
    sub = np.random.default_rng(1).choice(2000, 60, replace=False)
    c = synth.subset(cat, sub)
    a = oracle.upsilon(*c.arrays(), edges, nmax, distinct=True)
    b = oracle.brute_upsilon(*c.arrays(), edges, nmax, distinct=True)
    assert np.abs(b).max() > 0
    assert np.all(rel(a, b) < 1e-12)


def test_centre_subset_is_additive():
    cat = tiny(7, n=12)
    full = oracle.upsilon(*cat, TINY_EDGES, 2)
    part = oracle.upsilon(*cat, TINY_EDGES, 2, centers=[0, 3, 5]) + \
        oracle.upsilon(*cat, TINY_EDGES, 2, centers=[1, 2, 4, 6, 7, 8, 9, 10, 11])
    assert np.all(rel(part, full) < 1e-13)


# --------------------------------------------------------------------------
# Hand-computed example (phase and spin conventions, Sect. 2 and 3)
# --------------------------------------------------------------------------
def hand_catalogue():
    # centre X0 at the origin (w=2) and one neighbour per bin, edges 1,2,4,8:
    #   X1 (1.5, 0): phi=0    -> bin 0;  X2 (0, 3): phi=pi/2 -> bin 1;
    #   X3 (-7, 0): phi=pi    -> bin 2.
    # Shears chosen so that in the x-projection (zeta0 = (0+pi)/2 = pi/2,
    # zeta1 = 0, zeta2 = pi/2, zeta3 = pi) the projected shears
    # -gamma_c e^{-2i zeta} are s0 = 0.1i, s1 = -0.2i, s2 = 0.3i, s3 = 0.1:
    #   gamma_c0 = 0.1i, gamma_c1 = 0.2i, gamma_c2 = 0.3i, gamma_c3 = -0.1.
    x = np.array([0.0, 1.5, 0.0, -7.0])
    y = np.array([0.0, 0.0, 3.0, 0.0])
    g1 = np.array([0.0, 0.0, 0.0, -0.1])
    g2 = np.array([0.1, 0.2, 0.3, 0.0])
    w = np.array([2.0, 1.0, 1.0, 1.0])
    return (x, y, g1, g2, w), np.array([1.0, 2.0, 4.0, 8.0])


# Products w0 * s0 s1 s2 s3 with the conjugations of Gamma_0..7 (by hand):
#   G0: 2 (0.1i)(-0.2i)(0.3i)(0.1)   =  0.0012i     G1: 2 (-0.1i)(-0.2i)(0.3i)(0.1) = -0.0012i
#   G2: 2 (0.1i)(0.2i)(0.3i)(0.1)    = -0.0012i     G3: 2 (0.1i)(-0.2i)(-0.3i)(0.1) = -0.0012i
#   G4: = G0 (s3 real)               =  0.0012i     G5: 2 (-0.1i)(0.2i)(0.3i)(0.1)  =  0.0012i
#   G6: 2 (-0.1i)(-0.2i)(-0.3i)(0.1) =  0.0012i     G7: = G1 (s3 real)              = -0.0012i
#   N : 2
# Multipole phase e^{-i n2 phi12 - i n3 phi13}, phi12 = pi/2, phi13 = pi:
#   (0,0) -> 1, (1,0) -> -i, (0,1) -> -1, (1,1) -> i, (-1,2) -> i.
HAND_P = [0.0012j, -0.0012j, -0.0012j, -0.0012j, 0.0012j, 0.0012j, 0.0012j, -0.0012j, 2.0]
HAND_PHASE = {(0, 0): 1, (1, 0): -1j, (0, 1): -1, (1, 1): 1j, (-1, 2): 1j}


@pytest.mark.parametrize("distinct", [False, True])
def test_hand_example(distinct):
    cat, edges = hand_catalogue()
    nmax = 2
    u = oracle.upsilon(*cat, edges, nmax, centers=[0], distinct=distinct)
    for mu in range(9):
        for (n2, n3), ph in HAND_PHASE.items():
            got = u[mu, 0, 1, 2, n2 + nmax, n3 + nmax]
            assert abs(got - HAND_P[mu] * ph) < 1e-15, (mu, n2, n3, got)
    # (0,0,0): the raw sum holds the single j=k=l=X1 term, the distinct sum 0.
    # For Gamma_0 with all three at X1: zeta0 = 0, s0 = -0.1i, s1=s2=s3=-0.2i,
    # 2 (-0.1i)(-0.2i)^3 = 0.0016, phase 1 for every (n2, n3).
    got = u[0, 0, 0, 0]
    if distinct:
        assert np.abs(u[:, 0, 0, 0]).max() < 1e-16
    else:
        assert np.abs(got - 0.0016).max() < 1e-16
    # bins 0,1 repeated: only raw terms survive
    assert (np.abs(u[:, 0, 0, 1]).max() < 1e-16) == distinct


# --------------------------------------------------------------------------
# Table 2 of the paper (golden fixture)
# --------------------------------------------------------------------------
def load_table2():
    rows = []
    with open(os.path.join(HERE, "golden", "table2_symmetries.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            v = line.split()
            rows.append((int(v[0]), v[1], int(v[2]), tuple(map(int, v[3:6])), tuple(map(int, v[6:9]))))
    return rows


def test_table2_fixture_shape():
    rows = load_table2()
    assert len(rows) == 45
    assert {r[0] for r in rows} == set(range(9))


@pytest.mark.parametrize("distinct", [False, True])
def test_table2_relations(distinct):
    cat = tiny(11, n=14, side=8.0)
    nmax = 3
    u = oracle.upsilon(*cat, TINY_EDGES, nmax, distinct=distinct)
    nb = 3
    scale = np.abs(u).max(axis=(1, 2, 3, 4, 5))
    checked = 0
    for mu, perm, mu2, (a, b, c), (d, e, f) in load_table2():
        p = [int(ch) - 1 for ch in perm]
        for b1 in range(nb):
            for b2 in range(nb):
                for b3 in range(nb):
                    bb = (b1, b2, b3)
                    for n2 in range(-nmax, nmax + 1):
                        for n3 in range(-nmax, nmax + 1):
                            m2, m3 = a * n2 + b * n3 + c, d * n2 + e * n3 + f
                            if abs(m2) > nmax or abs(m3) > nmax:
                                continue
                            lhs = u[mu, b1, b2, b3, n2 + nmax, n3 + nmax]
                            rhs = u[mu2, bb[p[0]], bb[p[1]], bb[p[2]], m2 + nmax, m3 + nmax]
                            assert abs(lhs - rhs) <= 1e-12 * scale[mu], (mu, perm, bb, n2, n3)
                            checked += 1
    assert checked > 10000


# --------------------------------------------------------------------------
# Invariances (Sect. 2.2: natural components are rotation invariant)
# --------------------------------------------------------------------------
def small_uniform(seed=5, n=250, side=30.0):
    c = synth.uniform_catalogue(seed, n, side)
    return c.arrays(), np.array([1.0, 3.0, 7.0, 15.0])


@pytest.mark.parametrize("alpha", [0.7, 2.1])
def test_rotation_invariance(alpha):
    (x, y, g1, g2, w), edges = small_uniform()
    ca, sa = math.cos(alpha), math.sin(alpha)
    xr, yr = x * ca - y * sa, x * sa + y * ca
    gr = (g1 + 1j * g2) * np.exp(2j * alpha)
    cnt = oracle.bin_counts(x, y, edges, range(x.size))
    cntr = oracle.bin_counts(xr, yr, edges, range(x.size))
    assert np.array_equal(cnt, cntr)
    u0 = oracle.upsilon(x, y, g1, g2, w, edges, 3)
    u1 = oracle.upsilon(xr, yr, gr.real, gr.imag, w, edges, 3)
    assert np.all(rel(u1, u0) < 1e-12)


def test_rotation_90_exact_bins():
    (x, y, g1, g2, w), edges = small_uniform(seed=6)
    u0 = oracle.upsilon(x, y, g1, g2, w, edges, 3)
    u1 = oracle.upsilon(-y, x, -g1, -g2, w, edges, 3)
    assert np.all(rel(u1, u0) < 1e-13)


def test_mirror_conjugates():
    (x, y, g1, g2, w), edges = small_uniform(seed=7)
    u0 = oracle.upsilon(x, y, g1, g2, w, edges, 3)
    u1 = oracle.upsilon(x, -y, g1, -g2, w, edges, 3)
    assert np.all(rel(u1, np.conj(u0)) < 1e-13)


# --------------------------------------------------------------------------
# Integer closed forms (App. A.1) and real-weight symmetries (Eq. for N_n)
# --------------------------------------------------------------------------
def test_unit_weight_counts_closed_form():
    (x, y, g1, g2, _), edges = small_uniform(seed=8, n=300)
    w = np.ones_like(x)
    nmax = 2
    ud = oracle.upsilon(x, y, g1, g2, w, edges, nmax, distinct=True)
    ur = oracle.upsilon(x, y, g1, g2, w, edges, nmax, distinct=False)
    m = oracle.bin_counts(x, y, edges, range(x.size)).astype(np.float64)
    nb = 3
    d = np.eye(nb)
    exp_d = np.einsum("ia,ib,ic->abc", m, m, m) \
        - np.einsum("ia,ic,ab->abc", m, m, d) \
        - np.einsum("ia,ib,ac->abc", m, m, d) \
        - np.einsum("ia,ib,bc->abc", m, m, d) \
        + 2 * np.einsum("ia,ab,ac->abc", m, d, d)
    # = sum_i m_a (m_b - d_ab)(m_c - d_ac - d_bc)
    exp_alt = np.zeros((nb, nb, nb))
    for a in range(nb):
        for b in range(nb):
            for c in range(nb):
                exp_alt[a, b, c] = np.sum(m[:, a] * (m[:, b] - d[a, b]) * (m[:, c] - d[a, c] - d[b, c]))
    assert np.array_equal(exp_d, exp_alt)
    assert np.array_equal(ud[8, :, :, :, nmax, nmax].real, exp_alt)
    assert np.array_equal(ur[8, :, :, :, nmax, nmax].real, np.einsum("ia,ib,ic->abc", m, m, m))
    assert np.all(ud[8, :, :, :, nmax, nmax].imag == 0)


def test_real_weight_conjugate_symmetry():
    (x, y, g1, g2, w), edges = small_uniform(seed=9)
    nmax = 3
    u = oracle.upsilon(x, y, g1, g2, w, edges, nmax)
    n = u[8]
    assert np.abs(n[..., ::-1, ::-1] - np.conj(n)).max() < 1e-12 * np.abs(n).max()
    mp = oracle.multipoles(x, y, g1, g2, w, edges, nmax, range(20))
    lo, hi = mp["ranges"]["W"]
    assert lo == -hi
    W = mp["W"]
    assert np.abs(W[..., ::-1] - np.conj(W)).max() < 1e-12 * np.abs(W).max()


# --------------------------------------------------------------------------
# Binning: W_0 = weighted pair counts (double loop and a library counter)
# --------------------------------------------------------------------------
def test_pair_counts_double_loop_and_kdtree():
    (x, y, g1, g2, w), edges = small_uniform(seed=10, n=160, side=25.0)
    nb = edges.size - 1
    mp = oracle.multipoles(x, y, g1, g2, w, edges, 1, range(x.size))
    lo, _ = mp["ranges"]["W"]
    ww = np.einsum("i,ib->b", w, mp["W"][:, :, -lo].real)
    ref = np.zeros(nb)
    for i in range(x.size):
        for j in range(x.size):
            d = math.hypot(x[j] - x[i], y[j] - y[i])
            for b in range(nb):
                if edges[b] <= d < edges[b + 1]:
                    ref[b] += w[i] * w[j]
    assert np.allclose(ww, ref, rtol=1e-13, atol=0)
    scipy_spatial = pytest.importorskip("scipy.spatial")
    t = scipy_spatial.cKDTree(np.c_[x, y])
    cum = t.count_neighbors(t, edges, weights=(w, w), cumulative=True)
    assert np.allclose(ww, np.diff(cum), rtol=1e-12, atol=0)
    cnt = oracle.bin_counts(x, y, edges, range(x.size))
    cum_u = t.count_neighbors(t, edges, cumulative=True)
    assert np.array_equal(cnt.sum(0), np.diff(cum_u).astype(np.int64))


def test_family_ranges_and_entry_count():
    for n in range(0, 17):
        r = oracle.family_orders(n)
        assert r["G"] == (-2 * n - 3, 2 * n - 1)
        assert r["W"] == (-2 * n, 2 * n)
        assert r["V"] == (-2 * n, 2 * n)
        assert r["A"] == (-max(2 * n + 1, n + 2), max(2 * n + 1, n + 2))
        assert r["Q"] == (min(-2 * n - 5, -n - 6), max(2 * n - 3, n - 2))
        assert r["T"] == (-8, -4) and r["M"] == (-4, 0) and r["U"] == (0, 0)


# --------------------------------------------------------------------------
# Planted mistakes in the oracle are caught by the brute-force pin
# --------------------------------------------------------------------------
MUTATIONS = [
    ("TABLE1", 0, 0, ("Q", (0, 1, -4))),        # wrong order in a pair term
    ("TABLE1", 3, 2, ("Q", (-1, -1, -1))),      # wrong family
    ("TABLE1", 8, 3, ("V", (0, 0, 0))),         # triple term family
    ("FACTORS", 3, 2, ("G", False, (1, 0, -2))),  # dropped conjugate
    ("FACTORS", 0, 3, ("G", False, (0, -1, -2))),  # off-by-one order
    ("FACTORS", 1, 0, "g"),                     # wrong centre factor
    ("FACTORS", 5, 1, ("G", True, (-1, -1, -1))),  # wrong order in A
]


@pytest.mark.parametrize("table,mu,slot,value", MUTATIONS)
def test_planted_mistakes_are_caught(monkeypatch, table, mu, slot, value):
    cat = tiny(3, n=11)
    good = oracle.brute_upsilon(*cat, TINY_EDGES, 2, distinct=True)
    tab = [list(r) for r in getattr(est, table)]
    tab[mu][slot] = value
    monkeypatch.setattr(est, table, [tuple(r) for r in tab])
    bad = est.upsilon(*cat, TINY_EDGES, 2, distinct=True)
    assert rel(bad, good).max() > 1e-3


# --------------------------------------------------------------------------
# Natural components (multipoles -> angular bins); partly unpinned, see docs
# --------------------------------------------------------------------------
def test_angular_integrals_closed_form():
    from scipy.integrate import quad
    nphi = 7
    I = oracle.angular_integrals(4, nphi)
    ed = np.linspace(0, 2 * np.pi, nphi + 1)
    for mi, m in enumerate(range(-4, 5)):
        for a in range(nphi):
            re = quad(lambda p: math.cos(m * p), ed[a], ed[a + 1])[0]
            im = quad(lambda p: math.sin(m * p), ed[a], ed[a + 1])[0]
            assert abs(I[mi, a] - (re + 1j * im)) < 1e-12


def test_binned_sum_rule_and_monopole():
    rng = np.random.default_rng(3)
    nmax, nphi = 3, 8
    ups = rng.normal(size=(9, 2, 2, 2, 7, 7)) + 1j * rng.normal(size=(9, 2, 2, 2, 7, 7))
    b = oracle.binned_from_multipoles(ups, nphi)
    assert np.allclose(b.sum(axis=(-1, -2)), ups[..., nmax, nmax], rtol=1e-12, atol=1e-12)
    mono = np.zeros_like(ups)
    mono[..., nmax, nmax] = ups[..., nmax, nmax]
    bm = oracle.binned_from_multipoles(mono, nphi)
    assert np.allclose(bm, (ups[..., nmax, nmax] / nphi ** 2)[..., None, None], rtol=1e-12)


def test_binned_band_limited_quadrature():
    from scipy.integrate import dblquad
    rng = np.random.default_rng(4)
    nmax, nphi = 2, 5
    c = rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5))
    ups = np.zeros((9, 1, 1, 1, 5, 5), complex)
    ups[0, 0, 0, 0] = c
    b = oracle.binned_from_multipoles(ups, nphi)
    ed = np.linspace(0, 2 * np.pi, nphi + 1)
    ns = np.arange(-nmax, nmax + 1)

    def f(p13, p12, part):
        v = np.sum(c * np.exp(1j * (ns[:, None] * p12 + ns[None, :] * p13))) / (2 * np.pi) ** 2
        return v.real if part == 0 else v.imag

    for a, bb in [(0, 0), (1, 3), (4, 2)]:
        re = dblquad(f, ed[a], ed[a + 1], ed[bb], ed[bb + 1], args=(0,))[0]
        im = dblquad(f, ed[a], ed[a + 1], ed[bb], ed[bb + 1], args=(1,))[0]
        assert abs(b[0, 0, 0, 0, a, bb] - (re + 1j * im)) < 1e-10


def test_natural_components_converge_to_brute_angular_bins():
    """Truncated multipole conversion approaches the brute-force angular
    binning as nmax grows (slow, not bitwise: the expansion is truncated)."""
    cat = tiny(21, n=12, side=9.0)
    nphi = 4
    ref = oracle.brute_angular_bins(*cat, TINY_EDGES, nphi)
    errs = []
    for nmax in (2, 6, 14):
        u = oracle.upsilon(*cat, TINY_EDGES, nmax)
        b = oracle.binned_from_multipoles(u, nphi)
        errs.append(np.linalg.norm(b[8] - ref[8]) / np.linalg.norm(ref[8]))
    assert errs[2] < errs[0]


def test_natural_triplets_equal_slices_of_full_conversion():
    """The per-triplet form of the FP64 tail (used to stream large tensors)
    is the full conversion restricted to the listed triplets."""
    rng = np.random.default_rng(17)
    nb, nmax, nphi = 3, 2, 8
    nn = 2 * nmax + 1
    ups = rng.normal(size=(9, nb, nb, nb, nn, nn)) + 1j * rng.normal(size=(9, nb, nb, nb, nn, nn))
    ups[8] = np.abs(ups[8]) + 5.0          # a positive normalisation
    trip = np.array([[0, 1, 2], [2, 2, 2], [1, 0, 0], [0, 1, 2]])
    g, n = oracle.natural_components_triplets(ups, nphi, trip)
    G, N = oracle.natural_components(ups, nphi)
    for k, (a, b, c) in enumerate(trip):
        assert np.array_equal(n[k], N[a, b, c])
        assert np.array_equal(g[:, k], G[:, a, b, c])


def test_abs_bound_bounds_every_element_and_is_exact_for_n_at_zero_multipole():
    """The per-element scale S of the oracle (sum of absolute term values)
    bounds |Upsilon| for raw and distinct sums alike (triangle inequality);
    with positive weights the raw N at (n2, n3) = (0, 0) equals S[1] exactly,
    since W_0 is then the plain weight sum of the bin."""
    cat = synth.uniform_catalogue(9, 240, 25.0)
    edges = synth.log_edges(1.0, 12.0, 3)
    x, y, g1, g2, w = cat.arrays()
    S = oracle.abs_bound(x, y, g1, g2, w, edges)
    for distinct in (False, True):
        u = oracle.upsilon(x, y, g1, g2, w, edges, 2, distinct=distinct)
        assert np.all(np.abs(u[:8]) <= S[0][None, ..., None, None] * (1 + 1e-12))
        assert np.all(np.abs(u[8]) <= S[1][..., None, None] * (1 + 1e-12))
    raw = oracle.upsilon(x, y, g1, g2, w, edges, 2, distinct=False)
    assert np.allclose(raw[8, :, :, :, 2, 2].real, S[1], rtol=1e-13, atol=0)
    # the 3PCF variant bounds the order-3 sums the same way
    S3 = oracle.abs_bound(x, y, g1, g2, w, edges, order=3)
    u3 = oracle.upsilon3(x, y, g1, g2, w, edges, 2, distinct=False)
    assert np.all(np.abs(u3[:4]) <= S3[0][None, ..., None] * (1 + 1e-12))
    assert np.allclose(u3[4, :, :, 2].real, S3[1], rtol=1e-13, atol=0)


def test_parallel_oracle_equals_serial():
    """The process-pool variants (used to time the CPU baseline and for the
    large sampled parity cases) add chunk results in chunk order: equal to the
    serial oracle up to the order of the additions."""
    cat = synth.uniform_catalogue(10, 300, 30.0)
    edges = synth.log_edges(1.0, 15.0, 3)
    idx = np.arange(0, 300, 3)
    ser = oracle.upsilon(*cat.arrays(), edges, 2, centers=idx)
    par = oracle.upsilon_parallel(*cat.arrays(), edges, 2, centers=idx, processes=3, parts=5)
    assert np.allclose(par, ser, rtol=1e-13, atol=1e-13 * np.abs(ser).max())
    sb = oracle.abs_bound(*cat.arrays(), edges, idx)
    pb = oracle.abs_bound_parallel(*cat.arrays(), edges, idx, processes=3)
    assert np.allclose(pb, sb, rtol=1e-13, atol=0)


# --------------------------------------------------------------------------
# Sums at listed bin triplets (bin counts whose full tensor is too large)
# --------------------------------------------------------------------------
def triplet_sample(nb, seed, k):
    """k random bin triplets plus each kind of coincident bins (b1 = b2,
    b1 = b3, b2 = b3, all three) and the first and last bins."""
    rng = np.random.default_rng(seed)
    a, b = (int(v) for v in rng.choice(nb, 2, replace=False))
    special = [(a, a, b), (a, b, a), (b, a, a), (a, a, a), (0, 0, 0), (nb - 1, nb - 1, nb - 1),
               (0, nb - 1, nb - 1), (nb - 1, 0, nb - 1)]
    return np.concatenate([rng.integers(0, nb, size=(k, 3)), np.array(special)])


@pytest.mark.parametrize("distinct", [False, True])
def test_triplet_sums_equal_brute_force(distinct):
    """20 radial bins, nmax 2: the sums at listed triplets against the
    quadruplet enumeration of the definition, at random and coincident bins
    (every coincidence kind present with non-zero values)."""
    cat = tiny(11, n=40, side=12.0)
    nb = 20
    edges = synth.log_edges(0.4, 9.0, nb)
    t = triplet_sample(nb, 5, 60)
    # the bins holding most pairs, so that the coincident triplets are not empty
    cnt = oracle.bin_counts(cat[0], cat[1], edges, np.arange(40)).sum(axis=0)
    p, q = (int(v) for v in np.argsort(cnt)[-2:])
    t = np.concatenate([t, [(p, p, q), (p, q, p), (q, p, p), (p, p, p), (p, q, q)]])
    a = oracle.upsilon_triplets(*cat, edges, 2, t, distinct=distinct)
    full = oracle.brute_upsilon(*cat, edges, 2, distinct=distinct).reshape(9, nb, nb, nb, 5, 5)
    b = full[:, t[:, 0], t[:, 1], t[:, 2]]
    for k in range(len(t) - 5, len(t)):
        assert np.abs(b[:, k]).max() > 0
    assert np.all(rel(a, b) < 1e-12)


def test_triplet_sums_equal_full_tensor():
    """33 bins, nmax 3, 40 centres of the uniform 2000-galaxy catalogue: the
    triplet sums equal the corresponding elements of the full tensor."""
    cat, _, _, _ = synth.workload("uniform-2k")
    nb = 33
    edges = synth.log_edges(1.0, 30.0, nb)
    idx = np.random.default_rng(8).choice(cat.n, 40, replace=False)
    full = oracle.upsilon(*cat.arrays(), edges, 3, centers=idx)
    t = triplet_sample(nb, 9, 200)
    a = oracle.upsilon_triplets(*cat.arrays(), edges, 3, t, centers=idx)
    b = full[:, t[:, 0], t[:, 1], t[:, 2]]
    assert np.abs(b).max() > 0
    assert np.all(rel(a, b) < 1e-13)
    g1, n1 = oracle.natural_components_triplets(full, 17, t)
    g2, n2 = oracle.natural_components_selected(a, 17)
    assert np.linalg.norm(n1 - n2) <= 1e-12 * np.linalg.norm(n1)
    # Gamma = Ubar / Nbar: compared where Nbar is not a rounding residue of an
    # empty angular bin
    ok = np.abs(n1) > 1e-8 * np.abs(n1).max()
    assert np.linalg.norm((g1 - g2)[:, ok]) <= 1e-12 * np.linalg.norm(g1[:, ok])
    par = oracle.upsilon_triplets_parallel(*cat.arrays(), edges, 3, t, idx, processes=2)
    assert np.all(rel(par, a) < 1e-14)
