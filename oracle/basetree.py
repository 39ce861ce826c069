"""BaseTree and DoubleTree approximations of the shear 3PCF multipoles,
FP64 oracle.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the library never
does, and it shares no code with the library.

It follows the subsection on the algorithmic implementation in the appendix
on Nth-order statistics (App. F.3) at N = 3, in its order:

1. 'Tree': the blocks of a radial bin are allocated over a reduced catalogue
   of neighbours (grids Delta^L_d = 2^(d-1) Delta^L_1, the level of a bin as
   in Sect. 3.2: the coarsest grid with Theta_low / Delta^L_d >= r_min^L);
2. 'BaseTree': the sum over the base point X_0 runs over a second hierarchy
   of reduced catalogues (grids Delta^B_d), the grid chosen per radial bin
   by the same rule with its own Delta^B_1 and r_min^B; the value x of a
   base pseudo-galaxy is the cell sum of x (w gamma, or w);
3. the recursion: with Theta_1 <= Theta_2, x times the Theta_1 block is formed
   at the pseudo-galaxies of the Theta_1 grid (the product x X^1), summed over
   the cells of that grid inside each cell of the Theta_2 grid (the cached
   partial product), and multiplied by the Theta_2 block at the Theta_2
   grid's pseudo-galaxies;
4. 'DoubleTree' = 1 and 2 together.  Both reduce to the discrete estimator
   when no bin reaches a grid.

Readings (the paper does not spell these out):
* both hierarchies use the anchoring, centre of mass and level rule of the
  tree oracle (``oracle.tree``): grids anchored at (min x, min y), cells
  nested (a cell of grid d + 1 is the union of four cells of grid d);
* for Theta_1 > Theta_2 the recursion runs the other way: the Theta_2 block
  carries x and is summed into the Theta_1 grid.  The paper reaches this by
  reordering the radial bins and evaluating more multipoles; x F1 F2 is a
  product of commuting factors, so only the assignment of the factors to
  the grids matters;
* distinctness: the same-neighbour terms are removed where Theta_1 = Theta_2
  (both blocks then sit at the same base pseudo-galaxy), at that point, with
  the cell sums of the product weights ((w gamma)^2, |w gamma|^2, w^2) when
  the neighbours are pseudo-galaxies (as in ``oracle.tree``); for
  Theta_1 != Theta_2 the two blocks may see one galaxy from two base points
  and those terms stay: distinctness is over (galaxy, bin) memberships;
* every galaxy is a base point: the reduction replaces the sum over all of
  them (a centre subset is not defined here).
"""
from __future__ import annotations

import numpy as np

from .brute import projected
from .estimator import _family_values, check_inputs, squared_edges
from .nthorder import arg_coefficients, beta_matrix, norm_coefficients
from .tree import reduced_catalogue, tree_levels

FAMS = ("G", "W", "Q", "A", "V")


def _galaxies(x, y, g1, g2, w) -> dict:
    """The discrete catalogue in the layout of a reduced one (every galaxy
    its own cell)."""
    wg = w * (g1 + 1j * g2)
    sums = {f: _family_values(f, wg, w).astype(np.complex128) for f in FAMS}
    return {"x": x, "y": y, "cell": np.arange(x.size), "sums": sums, "n": x.size}


def _hierarchy(x, y, g1, g2, w, levels, delta1):
    """Level -> catalogue for every level in `levels` (0 = the galaxies)."""
    x0, y0 = float(np.min(x)), float(np.min(y))
    out = {}
    for d in sorted(set(levels)):
        out[d] = (_galaxies(x, y, g1, g2, w) if d == 0 else
                  reduced_catalogue(x, y, g1, g2, w, delta1 * 2.0 ** (d - 1), x0, y0))
    return out


def _orders(nmax):
    """Slot exponents c used by any (mu, n), the normalisation included."""
    B = beta_matrix(3)
    cs = set()
    for n in range(-nmax, nmax + 1):
        for r in B:
            c1, c2 = arg_coefficients(r, (n,))
            cs.update((c1 if r[1] > 0 else -c1, c2 if r[2] > 0 else -c2))
        cs.update(norm_coefficients((n,)))
    for r in B:
        c1, c2 = arg_coefficients(r, (0,))
        cs.update((c1 + c2, -(c1 + c2)))
    c1, c2 = norm_coefficients((0,))
    cs.add(c1 + c2)
    return sorted(cs)


def _blocks(px, py, nbr, e2, nb, orders):
    """Per base point (px, py): per bin and exponent c the family sums
    sum_j v_j e^{i c phi_j} over the neighbour catalogue `nbr`, as a dict
    fam -> complex [M, nb, len(orders)]."""
    M = px.size
    out = {f: np.zeros((M, nb, len(orders)), dtype=np.complex128) for f in FAMS}
    ords = np.asarray(orders)
    for c in range(M):
        dx = nbr["x"] - px[c]
        dy = nbr["y"] - py[c]
        r2 = dx * dx + dy * dy
        b = np.searchsorted(e2, r2, side="right") - 1
        sel = np.nonzero((b >= 0) & (b < nb))[0]
        if sel.size == 0:
            continue
        ph = np.exp(1j * np.multiply.outer(np.arctan2(dy[sel], dx[sel]), ords))   # [j, c]
        onehot = np.zeros((nb, sel.size))
        onehot[b[sel], np.arange(sel.size)] = 1.0
        for f in FAMS:
            out[f][c] = onehot @ (nbr["sums"][f][sel][:, None] * ph)
    return out


def _parent(cats, df, dc):
    """Index of the level-dc base pseudo-galaxy holding each level-df one
    (nested grids: all galaxies of a fine cell share one coarse cell)."""
    if df == dc:
        return np.arange(cats[df]["n"])
    par = np.zeros(cats[df]["n"], dtype=np.int64)
    par[cats[df]["cell"]] = cats[dc]["cell"]
    return par


def _aggregate(v, par, m):
    return (np.bincount(par, weights=v.real, minlength=m)
            + 1j * np.bincount(par, weights=v.imag, minlength=m))


def upsilon3_doubletree(x, y, g1, g2, w, edges, nmax, base=None, tree=None, distinct=True):
    """Shear 3PCF multipoles [5, nb, nb, 2 nmax + 1] (layout and sign of
    ``oracle.upsilon3``) with the BaseTree approximation of the base points
    (base = (Delta^B_1, levels, r_min^B)) and/or the Tree approximation of
    the neighbours (tree = (Delta^L_1, levels, r_min^L)); None switches one
    off."""
    x, y, g1, g2, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    check_inputs(x, y, g1, g2, w, edges, nmax)
    e2 = squared_edges(edges)
    nb = e2.size - 1
    nn = 2 * nmax + 1
    dB = tree_levels(edges, *base) if base is not None else [0] * nb
    dL = tree_levels(edges, *tree) if tree is not None else [0] * nb
    cats = _hierarchy(x, y, g1, g2, w, dB, base[0] if base is not None else 1.0)
    nbrs = _hierarchy(x, y, g1, g2, w, dL, tree[0] if tree is not None else 1.0)
    orders = _orders(nmax)
    col = {c: k for k, c in enumerate(orders)}
    # blocks of every bin at the base points of its own grid
    F = {}
    for d in sorted(set(dB)):
        cb = cats[d]
        for dl in sorted(set(dL[b] for b in range(nb) if dB[b] == d)):
            blk = _blocks(cb["x"], cb["y"], nbrs[dl], e2, nb, orders)
            for b in range(nb):
                if dB[b] == d and dL[b] == dl:
                    F[b] = {f: blk[f][:, b] for f in FAMS}          # [M_d, len(orders)]
    B = beta_matrix(3)
    sign = -1.0                     # (-1)^3: three projected shears
    out = np.zeros((5, nb, nb, nn), dtype=np.complex128)
    for mu in range(5):
        for d1 in sorted(set(dB)):
            for d2 in sorted(set(dB)):
                fine, coarse = min(d1, d2), max(d1, d2)
                cf = cats[fine]
                if mu < 4:
                    r = B[mu]
                    t = sign * cf["sums"]["G"]
                    t = t if r[0] > 0 else np.conj(t)
                else:
                    t = cf["sums"]["W"]
                par = _parent(cats, fine, coarse)
                mc = cats[coarse]["n"]
                for ni, n in enumerate(range(-nmax, nmax + 1)):
                    if mu < 4:
                        c1, c2 = arg_coefficients(B[mu], (n,))
                        slot = lambda b, beta, c: (F[b]["G"][:, col[c]] if beta > 0
                                                   else np.conj(F[b]["G"][:, col[-c]]))
                        f1 = lambda b: slot(b, B[mu][1], c1)
                        f2 = lambda b: slot(b, B[mu][2], c2)
                    else:
                        c1, c2 = norm_coefficients((n,))
                        f1 = lambda b: F[b]["W"][:, col[c1]]
                        f2 = lambda b: F[b]["W"][:, col[c2]]
                    for b1 in range(nb):
                        if dB[b1] != d1:
                            continue
                        for b2 in range(nb):
                            if dB[b2] != d2:
                                continue
                            if d1 <= d2:   # x rides on the Theta_1 block, summed into the Theta_2 grid
                                S = _aggregate(t * f1(b1), par, mc)
                                out[mu, b1, b2, ni] = np.sum(S * f2(b2))
                            else:          # the other way round
                                S = _aggregate(t * f2(b2), par, mc)
                                out[mu, b1, b2, ni] = np.sum(f1(b1) * S)
    if distinct:
        for b in range(nb):
            d = dB[b]
            cf = cats[d]
            for mu in range(5):
                if mu < 4:
                    r = B[mu]
                    c1, c2 = arg_coefficients(r, (0,))
                    # the product weight of one galaxy in both slots
                    fam, cj = (("Q", False) if r[1] > 0 and r[2] > 0 else
                               ("Q", True) if r[1] < 0 and r[2] < 0 else ("A", False))
                    t = sign * cf["sums"]["G"]
                    t = t if r[0] > 0 else np.conj(t)
                else:
                    c1, c2 = norm_coefficients((0,))
                    fam, cj = "V", False
                    t = cf["sums"]["W"]
                c = c1 + c2
                if cj:
                    Dv = np.conj(F[b][fam][:, col[-c]])
                else:
                    Dv = F[b][fam][:, col[c]]
                out[mu, b, b, :] -= np.sum(t * Dv)
    return out


def brute_upsilon3_doubletree(x, y, g1, g2, w, edges, nmax, base=None, tree=None, distinct=True):
    """The same approximation by enumeration, from the definitions: for every
    galaxy g as base point and bins (b1, b2), the neighbours of slot l are
    taken around the position of g's cell on the grid of b_l (g itself on
    the discrete level), from the bin's neighbour catalogue, and every ordered
    pair (j, k) contributes the product of the projected shears (Sect. 2.1)
    of g (angle (phi_j + phi_k)/2), j and k times the cell weight sums and
    e^{-i n (phi_k - phi_j)}.  Distinct: where b1 = b2, the terms in which one
    galaxy fills both slots are removed (j = k on the discrete catalogue; on
    a reduced one, the per-galaxy products summed over the cell).  Tiny
    inputs only."""
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    e2 = squared_edges(edges)
    nb = e2.size - 1
    nn = 2 * nmax + 1
    ns = np.arange(-nmax, nmax + 1)
    dB = tree_levels(edges, *base) if base is not None else [0] * nb
    dL = tree_levels(edges, *tree) if tree is not None else [0] * nb
    cats = _hierarchy(x, y, g1, g2, w, dB, base[0] if base is not None else 1.0)
    nbrs = _hierarchy(x, y, g1, g2, w, dL, tree[0] if tree is not None else 1.0)
    B = beta_matrix(3)
    gam = g1 + 1j * g2
    out = np.zeros((5, nb, nb, nn), dtype=np.complex128)

    def around(b, g):
        """Neighbours of bin b around g's base point on the grid of b:
        (values w gamma, weights w, product sums Q, A, V, angles)."""
        cb = cats[dB[b]]
        cell = cb["cell"][g]
        px, py = cb["x"][cell], cb["y"][cell]
        nc = nbrs[dL[b]]
        dx = nc["x"] - px
        dy = nc["y"] - py
        r2 = dx * dx + dy * dy
        bb = np.searchsorted(e2, r2, side="right") - 1
        sel = np.nonzero(bb == b)[0]
        s = nc["sums"]
        return (s["G"][sel], s["W"][sel].real, s["Q"][sel], s["A"][sel], s["V"][sel].real,
                np.arctan2(dy[sel], dx[sel]), sel)

    for g in range(x.size):
        xg = w[g] * gam[g]
        for b1 in range(nb):
            v1, u1, q1, a1, vv1, p1, s1 = around(b1, g)
            if p1.size == 0:
                continue
            for b2 in range(nb):
                v2, u2, q2, a2, vv2, p2, s2 = around(b2, g)
                if p2.size == 0:
                    continue
                J, K = (a.ravel() for a in np.meshgrid(np.arange(p1.size), np.arange(p2.size), indexing="ij"))
                P1, P2 = p1[J], p2[K]
                rot = (projected(xg, (P1 + P2) / 2), projected(v1[J], P1), projected(v2[K], P2))
                E = np.exp(-1j * np.multiply.outer(P2 - P1, ns))
                for mu, r in enumerate(B):
                    p = np.ones(J.size, dtype=np.complex128)
                    for l in range(3):
                        p = p * (rot[l] if r[l] > 0 else np.conj(rot[l]))
                    out[mu, b1, b2] += p @ E
                out[4, b1, b2] += (w[g] * u1[J] * u2[K]) @ E
                if distinct and b1 == b2:
                    # one galaxy in both slots: same entity (s1 == s2 here),
                    # per-galaxy products summed over it, angle phi_j twice
                    ph = p1
                    for mu, r in enumerate(B):
                        pc = projected(xg, ph)
                        pc = pc if r[0] > 0 else np.conj(pc)
                        # product of the two neighbour projections of one galaxy:
                        # (-v e^{-2i phi})(-v e^{-2i phi}) summed over the cell
                        rot2 = np.exp(-4j * ph)
                        if r[1] > 0 and r[2] > 0:
                            pp = q1 * rot2
                        elif r[1] < 0 and r[2] < 0:
                            pp = np.conj(q1 * rot2)
                        else:
                            pp = a1
                        out[mu, b1, b1] -= np.sum(pc * pp) * np.ones(nn)
                    out[4, b1, b1] -= np.sum(w[g] * vv1) * np.ones(nn)
    return out
