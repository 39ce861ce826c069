"""Pins of the order-N oracle (shear 3PCF multipoles) against what the paper
and the mathematics fix: the natural-component list of Sect. 2.2 (which the
beta-matrix enumeration must reproduce for N = 4), the explicit 4PCF factor
table of Sect. 3.1 (an independent derivation the general exponent rule must
agree with), triplet-by-triplet brute force, an integer closed form,
relabelling and rotation invariances, and planted mistakes."""
import numpy as np
import pytest

import oracle
from oracle import nthorder as nth
import synth


def rel(a, b):
    return np.array([np.linalg.norm(a[m] - b[m]) / max(np.linalg.norm(b[m]), 1e-300)
                     for m in range(a.shape[0])])


def tiny(seed, n=12, side=10.0):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, side, n), rng.uniform(0, side, n), rng.normal(0, .3, n),
            rng.normal(0, .3, n), rng.uniform(.5, 1.5, n))


EDGES = np.array([0.5, 3.0, 6.0, 15.0])


def test_beta_matrix_reproduces_sect22_list():
    """Sect. 2.2 conjugates, for Gamma_0..Gamma_7: none, X0, X1, X2, X3,
    X0X1, X0X2, X0X3."""
    paper = [(), (0,), (1,), (2,), (3,), (0, 1), (0, 2), (0, 3)]
    B = oracle.beta_matrix(4)
    assert B.shape == (8, 4)
    for mu, cc in enumerate(paper):
        want = np.ones(4, dtype=np.int64)
        want[list(cc)] = -1
        assert np.array_equal(B[mu], want), mu


def test_beta_matrix_counts_and_3pcf_components():
    for N in range(3, 8):
        B = oracle.beta_matrix(N)
        assert B.shape == (2 ** (N - 1), N)
        # no two rows equal, and no row the full conjugate of another
        rows = {tuple(r) for r in B}
        assert len(rows) == B.shape[0]
        assert not any(tuple(-np.array(r)) in rows for r in rows if N % 2 == 1)
    assert [tuple(r) for r in oracle.beta_matrix(3)] == [
        (1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)]


@pytest.mark.parametrize("seed", [0, 1])
def test_general_rule_equals_explicit_4pcf_table(seed):
    """N = 4 through the general exponent rule == the explicit factor table
    of Sect. 3.1 (raw sums: no distinctness in either)."""
    cat = tiny(seed, n=11)
    a = oracle.upsilon_n(*cat, EDGES, 4, 2)
    b = oracle.upsilon(*cat, EDGES, 2, distinct=False)
    assert np.abs(b).max() > 0
    assert np.all(rel(a, b) < 1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("distinct", [False, True])
def test_upsilon3_equals_brute_force(seed, distinct):
    cat = tiny(seed, n=10 + seed)
    a = oracle.upsilon3(*cat, EDGES, 4, distinct=distinct)
    b = oracle.brute_upsilon3(*cat, EDGES, 4, distinct=distinct)
    assert np.abs(b).max() > 0
    assert np.all(rel(a, b) < 1e-12)


def test_upsilon3_equals_brute_force_uniform2k_subset():
    cat, edges, _, _ = synth.workload("uniform-2k")
    sub = np.random.default_rng(1).choice(2000, 60, replace=False)
    c = synth.subset(cat, sub)
    a = oracle.upsilon3(*c.arrays(), edges, 6)
    b = oracle.brute_upsilon3(*c.arrays(), edges, 6)
    assert np.all(rel(a, b) < 1e-12)


def test_unit_weight_pair_count_closed_form():
    """w = 1: N_{n=0}(b1, b2) = sum_i m_{b1} (m_{b2} - delta_{b1 b2}) over
    distinct neighbour pairs, in exact integers."""
    x, y, g1, g2, _ = tiny(5, n=25)
    w = np.ones_like(x)
    ups = oracle.upsilon3(x, y, g1, g2, w, EDGES, 2)
    m = oracle.bin_counts(x, y, EDGES, range(x.size))
    nb = EDGES.size - 1
    want = np.zeros((nb, nb))
    for mi in m:
        want += np.outer(mi, mi) - np.diag(mi)
    got = ups[4, :, :, 2]
    assert np.array_equal(np.rint(got.real), want)
    assert np.abs(got.real - want).max() < 1e-9 and np.abs(got.imag).max() < 1e-9


def test_relabelling_theta1_theta2():
    """Swapping the two neighbour slots: Upsilon_0, Upsilon_1 and N map to
    themselves at -n with (b1, b2) swapped, Upsilon_2 and Upsilon_3 into
    each other; N_{-n} = conj N_n for real weights."""
    cat = tiny(7, n=20)
    u = oracle.upsilon3(*cat, EDGES, 3)
    sw = np.transpose(u, (0, 2, 1, 3))[..., ::-1]
    for a, b in ((0, 0), (1, 1), (2, 3), (3, 2), (4, 4)):
        assert np.allclose(u[a], sw[b], rtol=0, atol=1e-12 * np.abs(u[a]).max()), (a, b)


def test_norm_conjugate_symmetry():
    cat = tiny(8, n=20)
    u = oracle.upsilon3(*cat, EDGES, 3)
    assert np.allclose(u[4][..., ::-1], np.conj(u[4]), atol=1e-12 * np.abs(u[4]).max())


def test_rotation_invariance():
    """Rotating positions by alpha and shears by e^{2 i alpha} leaves every
    natural component unchanged."""
    x, y, g1, g2, w = tiny(9, n=18)
    a = 0.7
    xr = np.cos(a) * x - np.sin(a) * y
    yr = np.sin(a) * x + np.cos(a) * y
    gr = (g1 + 1j * g2) * np.exp(2j * a)
    u0 = oracle.upsilon3(x, y, g1, g2, w, EDGES, 3)
    u1 = oracle.upsilon3(xr, yr, gr.real, gr.imag, w, EDGES, 3)
    # the rotation moves pairs close to a bin edge only through rounding:
    # compare where the bin contents are unchanged (checked by the counts)
    assert np.array_equal(oracle.bin_counts(x, y, EDGES, range(x.size)),
                          oracle.bin_counts(xr, yr, EDGES, range(x.size)))
    assert np.all(rel(u1, u0) < 1e-12)


def test_planted_mistakes_are_caught():
    """A wrong sign of the centre term, a dropped factor 2 and a swapped
    slot conjugation each break agreement with brute force."""
    cat = tiny(3, n=12)
    ref = oracle.brute_upsilon3(*cat, EDGES, 3)

    def sign_flip(beta, ns):
        c = nth.arg_coefficients(beta, ns)
        return [c[0] + 2 * beta[0], c[1]]

    def no_factor_two(beta, ns):
        return [ns[0] - beta[0] - beta[1], -ns[0] - beta[0] - beta[2]]

    def swapped(beta, ns):
        c = nth.arg_coefficients(beta, ns)
        return [c[1], c[0]]

    for bad in (sign_flip, no_factor_two, swapped):
        got = oracle.upsilon3(*cat, EDGES, 3, coeff=bad)
        assert np.any(rel(got[:4], ref[:4]) > 1e-3), bad.__name__


def test_hand_example_three_galaxies():
    """Worked by hand from the definitions, not by the oracle: centre i at the
    origin (w 2, gamma_c = 0.1i), neighbour j at (1.5, 0) (w 1, gamma_c =
    0.2i, phi = 0, bin [1, 2)), neighbour k at (0, 3) (w 1, gamma_c = 0.3i,
    phi = pi/2, bin [2, 4)).  For (Theta_1, Theta_2) = (bin 0, bin 1):
    zeta_0 = pi/4, zeta_1 = 0, zeta_2 = pi/2, and the projected shears
    -gamma_c e^{-2i zeta} (Sect. 2.1) are -0.1, -0.2i and +0.3i, so
      Gamma_0 = (-0.1)(-0.2i)(0.3i) = -0.006,  Gamma_1 (centre conjugated)
      = -0.006,  Gamma_2 (slot 1) = (-0.1)(0.2i)(0.3i) = +0.006,
      Gamma_3 (slot 2) = (-0.1)(-0.2i)(-0.3i) = +0.006,
    times w_i w_j w_k = 2 and e^{-i n phi_12}, phi_12 = pi/2: (-i)^n.  For
    (bin 1, bin 0) the slots swap: phi_12 = -pi/2, the same products, i^n.
    A sign convention without the minus of the projection flips every shear
    component here."""
    x = np.array([0.0, 1.5, 0.0]); y = np.array([0.0, 0.0, 3.0])
    g1 = np.zeros(3); g2 = np.array([0.1, 0.2, 0.3]); w = np.array([2.0, 1.0, 1.0])
    edges = np.array([1.0, 2.0, 4.0])
    P = [-0.012, -0.012, 0.012, 0.012, 2.0]
    for fn in (lambda: nth.upsilon3(x, y, g1, g2, w, edges, 3, centers=[0]),
               lambda: nth.brute_upsilon3(x, y, g1, g2, w, edges, 3, centers=[0])):
        u = fn()
        for mu in range(5):
            for n in range(-3, 4):
                assert abs(u[mu, 0, 1, n + 3] - P[mu] * (-1j) ** n) < 1e-15
                assert abs(u[mu, 1, 0, n + 3] - P[mu] * (1j) ** n) < 1e-15
                assert abs(u[mu, 0, 0, n + 3]) < 1e-15 and abs(u[mu, 1, 1, n + 3]) < 1e-15
