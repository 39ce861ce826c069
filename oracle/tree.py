"""Tree (reduced-catalogue) approximation of the per-centre multipoles,
FP64 oracle.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the library never
does, and it shares no code with the library.

It follows the practical implementation described in Sect. 3 of Porth et
al. (2025) (the subsection on tree-based acceleration), in its order:

1. a hierarchy of grids of cell side Delta_d = 2^(d-1) Delta_1, d = 1..D;
2. one reduced catalogue per grid: every non-empty cell becomes one
   pseudo-galaxy at the cell's centre of mass, carrying the cell-summed
   weighted shear (the cell-averaged shear times the cell weight);
3. each radial bin uses the coarsest level d with Theta_low / Delta_d >=
   r_min, or the discrete estimator when no level qualifies;
4. the blocks G_n of a bin are allocated with the standard formula, the sum
   running over the pseudo-galaxies of the bin's level; centres remain the
   original galaxies; contraction and corrections are unchanged.

Readings (the paper does not spell these out):
* the grids are anchored at the lower-left corner (min x, min y) of the
  catalogue; cell index floor((x - x_min) / Delta) per axis;
* "centre of mass" is weighted by w; a cell of zero total weight sits at the
  plain mean of its galaxies;
* the multiple-counting blocks of App. A.1 of an approximated bin use the
  cell sums of the corresponding per-galaxy weights ((w gamma)^2,
  |w gamma|^2, w^2, (w gamma)^3, |w gamma|^2 w gamma, w^3), so that the
  subtraction still removes exactly the terms in which one galaxy fills two
  slots (distinct galaxies of one cell remain distinct);
* r_min >= 2 is required, so that the centre's own cell (within sqrt(2)
  Delta of it) never falls into an approximated bin;
* with different resolutions per bin a galaxy can enter two bins (through
  its own position in one and its cell's centre of mass in another) or
  none; the multipole route counts such a galaxy in both, and its
  distinctness is over (galaxy, bin) memberships, which is what the
  corrections of App. A.1 remove.
"""
from __future__ import annotations

import numpy as np

from .brute import CONJ, projected
from .estimator import (_family_values, centre_multipoles, check_inputs, contract,
                        family_orders, squared_edges)

FAMS = ("G", "W", "Q", "A", "V", "T", "M", "U")


def tree_levels(edges, delta1: float, nlevels: int, rmin: float) -> list:
    """Level per radial bin: 0 = discrete, d >= 1 = grid of side
    delta1 * 2^(d-1), the coarsest d with edges[b] / Delta_d >= rmin."""
    lv = []
    for b in range(len(edges) - 1):
        best = 0
        for d in range(1, nlevels + 1):
            if edges[b] / (delta1 * 2.0 ** (d - 1)) >= rmin:
                best = d
        lv.append(best)
    return lv


def reduced_catalogue(x, y, g1, g2, w, delta: float, x0: float, y0: float) -> dict:
    """Pseudo-galaxies of the grid of side delta anchored at (x0, y0):
    positions 'x', 'y' (w-weighted centres of mass), the cell index 'cell'
    of each galaxy, and the cell sums of every family weight."""
    ix = np.floor((x - x0) / delta).astype(np.int64)
    iy = np.floor((y - y0) / delta).astype(np.int64)
    cells, inv = np.unique(np.stack([iy, ix], 1), axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nc = cells.shape[0]
    W = np.bincount(inv, weights=w, minlength=nc)
    cnt = np.bincount(inv, minlength=nc)
    sx = np.bincount(inv, weights=w * x, minlength=nc)
    sy = np.bincount(inv, weights=w * y, minlength=nc)
    mx = np.bincount(inv, weights=x, minlength=nc) / cnt
    my = np.bincount(inv, weights=y, minlength=nc) / cnt
    with np.errstate(divide="ignore", invalid="ignore"):
        px = np.where(W != 0.0, sx / np.where(W != 0.0, W, 1.0), mx)
        py = np.where(W != 0.0, sy / np.where(W != 0.0, W, 1.0), my)
    wg = w * (g1 + 1j * g2)
    sums = {}
    for fam in FAMS:
        v = _family_values(fam, wg, w)
        sums[fam] = (np.bincount(inv, weights=v.real, minlength=nc)
                     + 1j * np.bincount(inv, weights=v.imag, minlength=nc))
    return {"x": px, "y": py, "cell": inv, "sums": sums, "n": nc}


def reduced_hierarchy(x, y, g1, g2, w, delta1: float, nlevels: int) -> dict:
    x0, y0 = float(np.min(x)), float(np.min(y))
    return {d: reduced_catalogue(x, y, g1, g2, w, delta1 * 2.0 ** (d - 1), x0, y0)
            for d in range(1, nlevels + 1)}


def tree_centre_multipoles(x, y, g1, g2, w, e2, nmax, i, levels, red, ranges=None):
    """centre_multipoles with the bins of level d >= 1 replaced by sums over
    the pseudo-galaxies of level d."""
    if ranges is None:
        ranges = family_orders(nmax)
    nb = e2.size - 1
    out = centre_multipoles(x, y, g1, g2, w, e2, nmax, i, ranges)
    lv = np.asarray(levels)
    for d in sorted(set(levels) - {0}):
        R = red[d]
        dx = R["x"] - x[i]
        dy = R["y"] - y[i]
        r2 = dx * dx + dy * dy
        b = np.searchsorted(e2, r2, side="right") - 1
        ok = (b >= 0) & (b < nb)
        ok[ok] = lv[b[ok]] == d
        sel = np.nonzero(ok)[0]
        bins = np.nonzero(lv == d)[0]
        phi = np.arctan2(dy[sel], dx[sel])
        onehot = np.zeros((nb, sel.size))
        onehot[b[sel], np.arange(sel.size)] = 1.0
        out["counts"][bins] = np.bincount(b[sel], minlength=nb)[bins]
        for fam, (lo, hi) in ranges.items():
            ks = np.arange(lo, hi + 1)
            ph = np.exp(1j * np.multiply.outer(phi, ks))
            blk = onehot @ (R["sums"][fam][sel][:, None] * ph)
            out[fam][bins] = blk[bins]
    return out


def upsilon_tree(x, y, g1, g2, w, edges, nmax, delta1: float, nlevels: int, rmin: float,
                 centers=None, distinct=True, chunk=256):
    """4PCF multipoles with the tree approximation (layout as
    ``estimator.upsilon``)."""
    x, y, g1, g2, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    check_inputs(x, y, g1, g2, w, edges, nmax)
    if not (rmin >= 2.0):
        raise ValueError("rmin must be >= 2")
    e2 = squared_edges(edges)
    nb = e2.size - 1
    levels = tree_levels(edges, delta1, nlevels, rmin)
    red = reduced_hierarchy(x, y, g1, g2, w, delta1, nlevels)
    ranges = family_orders(nmax)
    if centers is None:
        centers = np.arange(x.size)
    centers = np.asarray(centers, dtype=np.int64)
    nn = 2 * nmax + 1
    out = np.zeros((9, nb, nb, nb, nn, nn), dtype=np.complex128)
    for s in range(0, len(centers), chunk):
        c = centers[s:s + chunk]
        per = [tree_centre_multipoles(x, y, g1, g2, w, e2, nmax, int(i), levels, red, ranges) for i in c]
        mp = {k: np.stack([p[k] for p in per]) for k in per[0]}
        mp["ranges"] = ranges
        out += contract(mp, g1, g2, w, c, nmax, nb, distinct)
    return out


def brute_tree_upsilon(x, y, g1, g2, w, edges, nmax, delta1, nlevels, rmin, distinct=True):
    """Quadruplet-by-quadruplet definition of the tree estimator: for a bin
    of level d >= 1, a galaxy j is a neighbour of centre i in that bin when
    its level-d cell's centre of mass lies in the bin, and it enters with
    the angle of that centre of mass; quadruplets are of distinct neighbours
    (cells may be shared), distinct as (galaxy, bin) memberships.  Tiny
    inputs only."""
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    e2 = squared_edges(edges)
    nb = e2.size - 1
    nn = 2 * nmax + 1
    ns = np.arange(-nmax, nmax + 1)
    levels = tree_levels(edges, delta1, nlevels, rmin)
    red = reduced_hierarchy(x, y, g1, g2, w, delta1, nlevels)
    gam = g1 + 1j * g2
    out = np.zeros((9, nb, nb, nb, nn, nn), dtype=np.complex128)
    for i in range(x.size):
        # (galaxy, bin, angle) memberships of centre i
        memb = []
        for j in range(x.size):
            for d in sorted(set(levels)):
                if d == 0:
                    px, py = x[j], y[j]
                else:
                    c = red[d]["cell"][j]
                    px, py = red[d]["x"][c], red[d]["y"][c]
                dx, dy = px - x[i], py - y[i]
                r2 = dx * dx + dy * dy
                b = int(np.searchsorted(e2, r2, side="right") - 1)
                if 0 <= b < nb and levels[b] == d and not (d == 0 and j == i):
                    memb.append((j, b, np.arctan2(dy, dx)))
        for u1, (j, b1, p1) in enumerate(memb):
            for u2, (k, b2, p2) in enumerate(memb):
                for u3, (l, b3, p3) in enumerate(memb):
                    if distinct and (u1 == u2 or u1 == u3 or u2 == u3):
                        continue
                    z0 = 0.5 * (p1 + p3)
                    s = (projected(gam[i], z0), projected(gam[j], p1), projected(gam[k], p2),
                         projected(gam[l], p3))
                    wt = w[i] * w[j] * w[k] * w[l]
                    e = np.exp(-1j * np.add.outer(ns * (p2 - p1), ns * (p3 - p1)))
                    for mu, pat in enumerate(CONJ):
                        pr = wt
                        for a in range(4):
                            pr = pr * (np.conj(s[a]) if pat[a] else s[a])
                        out[mu, b1, b2, b3] += pr * e
                    out[8, b1, b2, b3] += wt * e
    return out
