"""Pins of the BaseTree / DoubleTree oracle of the shear 3PCF (App. F.3,
algorithmic implementation) against things other than itself: the discrete
3PCF oracle (itself pinned by triplet enumeration) where no bin reaches a
grid, and an enumeration of the approximation's own definition (every
galaxy as base point, neighbours taken around the position of its cell on
each bin's grid, projected shears of Sect. 2.1) on tiny catalogues, for the
BaseTree, the Tree and their combination.  A planted mistake in the parent
map is caught."""
import numpy as np
import pytest

import oracle
from oracle import basetree as bt


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def tiny(seed, n=30, side=12.0):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, side, n), rng.uniform(0, side, n), rng.normal(0, .3, n),
            rng.normal(0, .3, n), rng.uniform(.5, 1.5, n))


EDGES = np.array([0.5, 1.5, 3.0, 6.0, 11.0])
BASE = (0.5, 2, 3.0)      # grids 0.5' and 1': bins -> [0, 1, 2, 2]
TREE = (0.4, 2, 3.0)      # neighbour grids 0.4' and 0.8': bins -> [0, 1, 2, 2]


def test_levels_of_the_pins():
    assert oracle.tree_levels(EDGES, *BASE) == [0, 1, 2, 2]
    assert oracle.tree_levels(EDGES, *TREE) == [0, 1, 2, 2]


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("distinct", [True, False])
def test_no_grid_is_the_discrete_3pcf(seed, distinct):
    cat = tiny(seed)
    ref = oracle.upsilon3(*cat, EDGES, 2, distinct=distinct)
    assert rel(bt.upsilon3_doubletree(*cat, EDGES, 2, distinct=distinct), ref) < 1e-13
    # grids no bin reaches
    assert rel(bt.upsilon3_doubletree(*cat, EDGES, 2, base=(0.5, 2, 1e3), tree=(0.5, 2, 1e3),
                                      distinct=distinct), ref) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("distinct", [True, False])
@pytest.mark.parametrize("mode", ["base", "tree", "double"])
def test_equals_enumeration_of_the_definition(seed, distinct, mode):
    cat = tiny(seed, n=26 + 2 * seed, side=5.0)   # dense: cells of 0.5' hold several galaxies
    kw = {"base": {"base": BASE}, "tree": {"tree": TREE}, "double": {"base": BASE, "tree": TREE}}[mode]
    a = bt.upsilon3_doubletree(*cat, EDGES, 2, distinct=distinct, **kw)
    b = bt.brute_upsilon3_doubletree(*cat, EDGES, 2, distinct=distinct, **kw)
    assert np.abs(b).max() > 0
    assert rel(a, b) < 1e-12
    # and it is an approximation
    assert rel(a, oracle.upsilon3(*cat, EDGES, 2, distinct=distinct)) > 1e-4


def test_fine_grid_limit_is_discrete():
    """Grids so fine that every cell holds one galaxy: the pseudo-galaxies are
    the galaxies and the recursion collapses to the discrete sum."""
    cat = tiny(4)
    assert set(oracle.tree_levels(EDGES, 1e-6, 3, 2.0)) == {3}
    a = bt.upsilon3_doubletree(*cat, EDGES, 3, base=(1e-6, 3, 2.0))
    assert rel(a, oracle.upsilon3(*cat, EDGES, 3)) < 1e-13


def test_planted_parent_swap_is_caught(monkeypatch):
    cat = tiny(5)
    good = bt.brute_upsilon3_doubletree(*cat, EDGES, 2, base=BASE)

    def swapped(cats, df, dc):
        if df == dc:
            return np.arange(cats[df]["n"])
        par = np.zeros(cats[df]["n"], dtype=np.int64)
        par[cats[df]["cell"][::-1]] = cats[dc]["cell"]      # members paired with the wrong cells
        return np.minimum(par, cats[dc]["n"] - 1)
    monkeypatch.setattr(bt, "_parent", swapped)
    bad = bt.upsilon3_doubletree(*cat, EDGES, 2, base=BASE)
    assert rel(bad, good) > 1e-3
