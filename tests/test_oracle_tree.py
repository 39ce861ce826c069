"""Pins of the tree (reduced-catalogue) oracle: the per-bin resolution rule
worked by hand, the reduced catalogue against a library binned statistic,
the multipole route against a quadruplet-by-quadruplet definition, and the
two limits in which the approximation must vanish."""
import numpy as np
import pytest

import oracle


def tiny(seed, n=14, side=12.0):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, side, n), rng.uniform(0, side, n), rng.normal(0, .3, n),
            rng.normal(0, .3, n), rng.uniform(.5, 1.5, n))


def rel(a, b):
    return np.array([np.linalg.norm(a[m] - b[m]) / max(np.linalg.norm(b[m]), 1e-300)
                     for m in range(a.shape[0])])


def test_levels_follow_the_coarsest_resolution_rule():
    """Grids 0.5', 1', 2' and r_min = 40 (the paper's DES setting): a bin
    uses 2' from Theta_low = 80', 1' from 40', 0.5' from 20', else the
    discrete estimator."""
    edges = [10.0, 19.99, 20.0, 39.99, 40.0, 79.99, 80.0, 150.0, 166.0]
    assert oracle.tree_levels(edges, 0.5, 3, 40.0) == [0, 0, 1, 1, 2, 2, 3, 3]
    assert oracle.tree_levels(edges, 0.5, 1, 40.0) == [0, 0, 1, 1, 1, 1, 1, 1]
    assert oracle.tree_levels(edges, 0.5, 3, 1e9) == [0] * 8


def test_reduced_catalogue_matches_binned_statistic():
    stats = pytest.importorskip("scipy.stats")
    x, y, g1, g2, w = tiny(1, n=200, side=20.0)
    delta = 1.7
    R = oracle.reduced_catalogue(x, y, g1, g2, w, delta, x.min(), y.min())
    nx = int(np.floor((x.max() - x.min()) / delta)) + 1
    ny = int(np.floor((y.max() - y.min()) / delta)) + 1
    ix = np.floor((x - x.min()) / delta).astype(int)
    iy = np.floor((y - y.min()) / delta).astype(int)
    # library sums per cell; compare pseudo-galaxy by pseudo-galaxy via a member galaxy
    sw = stats.binned_statistic_2d(ix, iy, w, "sum", bins=[np.arange(nx + 1) - .5, np.arange(ny + 1) - .5])
    swx = stats.binned_statistic_2d(ix, iy, w * x, "sum", bins=[np.arange(nx + 1) - .5, np.arange(ny + 1) - .5])
    swg = stats.binned_statistic_2d(ix, iy, w * g1, "sum", bins=[np.arange(nx + 1) - .5, np.arange(ny + 1) - .5])
    sq = stats.binned_statistic_2d(ix, iy, (w * g1) ** 2 - (w * g2) ** 2, "sum",
                                   bins=[np.arange(nx + 1) - .5, np.arange(ny + 1) - .5])
    for j in range(x.size):
        c = R["cell"][j]
        W = sw.statistic[ix[j], iy[j]]
        assert np.isclose(R["sums"]["W"][c].real, W, rtol=1e-13)
        assert np.isclose(R["x"][c], swx.statistic[ix[j], iy[j]] / W, rtol=1e-13)
        assert np.isclose(R["sums"]["G"][c].real, swg.statistic[ix[j], iy[j]], rtol=1e-12, atol=1e-14)
        assert np.isclose(R["sums"]["Q"][c].real, sq.statistic[ix[j], iy[j]], rtol=1e-12, atol=1e-14)
    assert R["n"] == len({(a, b) for a, b in zip(ix, iy)})


@pytest.mark.parametrize("seed", [3, 4])
@pytest.mark.parametrize("distinct", [True, False])
def test_tree_multipoles_equal_quadruplet_definition(seed, distinct):
    cat = tiny(seed)
    edges = np.array([0.5, 2.0, 4.0, 9.0])
    assert oracle.tree_levels(edges, 0.5, 2, 4.0) == [0, 1, 2]
    a = oracle.upsilon_tree(*cat, edges, 1, 0.5, 2, 4.0, distinct=distinct)
    b = oracle.brute_tree_upsilon(*cat, edges, 1, 0.5, 2, 4.0, distinct=distinct)
    assert np.abs(b).max() > 0
    assert np.all(rel(a, b) < 1e-12)


def test_fine_grid_limit_is_the_discrete_estimator():
    """Cells far smaller than the galaxy spacing hold one galaxy each, so the
    pseudo-galaxies are the galaxies and every bin reproduces the discrete
    estimator."""
    x, y, g1, g2, w = tiny(5, n=40, side=30.0)
    edges = np.array([1.0, 3.0, 7.0, 15.0])
    assert oracle.tree_levels(edges, 1e-4, 1, 2.0) == [1, 1, 1]
    a = oracle.upsilon_tree(x, y, g1, g2, w, edges, 2, 1e-4, 1, 2.0)
    b = oracle.upsilon(x, y, g1, g2, w, edges, 2)
    assert np.all(rel(a, b) < 1e-10)


def test_no_qualifying_level_is_the_discrete_estimator():
    x, y, g1, g2, w = tiny(6, n=40, side=30.0)
    edges = np.array([1.0, 3.0, 7.0, 15.0])
    a = oracle.upsilon_tree(x, y, g1, g2, w, edges, 2, 0.5, 3, 1e6)
    b = oracle.upsilon(x, y, g1, g2, w, edges, 2)
    assert np.array_equal(a, b)


def test_rmin_below_two_rejected():
    x, y, g1, g2, w = tiny(7)
    with pytest.raises(ValueError):
        oracle.upsilon_tree(x, y, g1, g2, w, [1.0, 2.0], 1, 0.5, 1, 1.5)
