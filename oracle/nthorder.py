"""FP64 CPU oracle of the multipole-based estimator for shear correlation
functions of general order N, used for N = 3 (the shear 3PCF) and, as a
cross-check of the general construction against the explicit 4PCF factor
table, for N = 4.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the library never
does, and it shares no code with the library.

It follows the appendix "Multipole-based estimators for Nth-order shear
statistics" of Porth et al. (2025):

1. natural components (notation subsection): Gamma_0 has no conjugated
   shear; then, for p = 1 ... floor(N/2) conjugated shears, every placement
   of the p conjugations in the order of the stated procedure (read as the
   lexicographic order of the conjugated positions); for even N only the
   first half of the p = N/2 placements.  beta^mu_l = -1 where the l-th
   shear of Gamma_mu is conjugated, +1 otherwise (l = 1 is the centre);
2. generalised x-projection: zeta_0 = (phi_1 + phi_{N-1}) / 2 for the
   centre, zeta_l = phi_l for the l-th neighbour;
3. the exponent Arg_mu of that appendix: the coefficient of phi_1 is
   sum_l n_l - beta_1 - 2 beta_2, of phi_l (2 <= l <= N-2) it is
   -n_l - 2 beta_{l+1}, of phi_{N-1} it is -n_{N-1} - beta_1 - 2 beta_N;
4. a neighbour slot with coefficient c is G_c (beta = +1) or conj(G_{-c})
   (beta = -1), G_c = sum_j w_j gamma_j e^{i c phi_ij} over the slot's bin;
   the centre factor is w_i gamma_i or its conjugate (beta_1);  the
   normalisation uses W blocks and w_i with every beta term dropped;
5. N = 3, distinct pairs of neighbours (j != k): the j = k terms of the
   double sum, present only when both slots share a bin, are subtracted.

Reading: the appendix writes the multipoles through the blocks G and W and
only states the argument of the exponent; the natural components themselves
are products of N projected shears gamma = -gamma_c e^{-2 i zeta} (Sect. 2.1),
which carry the factor (-1)^N that the printed block formula omits.  The
definition decides: every shear component of order N is the block product
times (-1)^N (no change for N = 4; a minus sign for the N = 3 shear
components, none for the normalisation, whose summand has no shear).

All arithmetic is numpy float64 / complex128.
"""
from __future__ import annotations

import itertools

import numpy as np

from .brute import projected
from .estimator import check_inputs, centre_neighbours, squared_edges


def beta_matrix(N: int) -> np.ndarray:
    """[2^{N-1}, N] matrix of +-1: row mu is Gamma_mu, column l the l-th
    shear (0 = centre)."""
    if N < 2:
        raise ValueError("N >= 2")
    rows = [np.ones(N, dtype=np.int64)]
    for p in range(1, N // 2 + 1):
        combos = list(itertools.combinations(range(N), p))
        if 2 * p == N:
            combos = combos[: len(combos) // 2]
        for cc in combos:
            r = np.ones(N, dtype=np.int64)
            r[list(cc)] = -1
            rows.append(r)
    out = np.array(rows)
    assert out.shape[0] == 2 ** (N - 1)
    return out


def arg_coefficients(beta, ns) -> list:
    """Coefficients of phi_1 ... phi_{N-1} in Arg_mu for the multipole
    vector ns = (n_2, ..., n_{N-1}) and one row beta = (beta_1..beta_N)."""
    N = len(beta)
    if N < 3 or len(ns) != N - 2:
        raise ValueError("N >= 3 with N-2 multipole indices")
    c = [0] * (N - 1)
    c[0] = sum(ns) - beta[0] - 2 * beta[1]
    for l in range(2, N - 1):
        c[l - 1] = -ns[l - 2] - 2 * beta[l]
    c[N - 2] += -ns[N - 3] - beta[0] - 2 * beta[N - 1]
    return c


def norm_coefficients(ns) -> list:
    """Coefficients of the normalisation: Arg with every beta term dropped."""
    N = len(ns) + 2
    c = [0] * (N - 1)
    c[0] = sum(ns)
    for l in range(2, N - 1):
        c[l - 1] = -ns[l - 2]
    c[N - 2] += -ns[N - 3]
    return c


def _slot_blocks(phi, b, wg, w, nb, orders):
    """Per-bin complex sums G_c = sum_j wg_j e^{i c phi_j} and W_c for every
    order c in `orders`: dict c -> ([nb] G, [nb] W)."""
    out = {}
    for c in orders:
        e = np.exp(1j * c * phi)
        out[c] = (np.bincount(b, weights=(wg * e).real, minlength=nb)
                  + 1j * np.bincount(b, weights=(wg * e).imag, minlength=nb),
                  np.bincount(b, weights=(w * e).real, minlength=nb)
                  + 1j * np.bincount(b, weights=(w * e).imag, minlength=nb))
    return out


def _slot(blocks, beta, c):
    """Neighbour-slot factor per bin: G_c (beta = +1) or conj(G_{-c})."""
    return blocks[c][0] if beta > 0 else np.conj(blocks[-c][0])


def upsilon_n(x, y, g1, g2, w, edges, N, nmax, centers=None, coeff=arg_coefficients):
    """Raw multipoles (all neighbour tuples, no distinctness) of the shear
    NPCF: array [2^{N-1} + 1, nb, ..., nb, (2 nmax + 1), ...] with N-1 bin
    axes and N-2 multipole axes (n_l stored at offset +nmax); the last
    component is the normalisation.  Small inputs only (N <= 4)."""
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    check_inputs(x, y, g1, g2, w, edges, nmax)
    B = beta_matrix(N)
    nmu = B.shape[0]
    e2 = squared_edges(edges)
    nb = e2.size - 1
    nn = 2 * nmax + 1
    gam = g1 + 1j * g2
    out = np.zeros((nmu + 1,) + (nb,) * (N - 1) + (nn,) * (N - 2), dtype=np.complex128)
    if centers is None:
        centers = range(x.size)
    nvecs = list(itertools.product(range(-nmax, nmax + 1), repeat=N - 2))
    orders = set()
    for ns in nvecs:
        for r in B:
            for l, c in enumerate(coeff(r, ns)):
                orders.add(c if r[l + 1] > 0 else -c)
        orders.update(norm_coefficients(ns))
    sign = (-1.0) ** N          # the product of N projected shears -gamma_c e^{-2 i zeta}
    for i in centers:
        i = int(i)
        sel, b, dx, dy = centre_neighbours(x, y, e2, i)
        if sel.size == 0:
            continue
        phi = np.arctan2(dy, dx)
        blk = _slot_blocks(phi, b, w[sel] * gam[sel], w[sel], nb, sorted(orders))
        xg = sign * w[i] * gam[i]
        for ns in nvecs:
            idx = tuple(n + nmax for n in ns)
            for mu, r in enumerate(B):
                cs = coeff(r, ns)
                f = [_slot(blk, r[l + 1], cs[l]) for l in range(N - 1)]
                t = xg if r[0] > 0 else np.conj(xg)
                term = t * f[0]
                for l in range(1, N - 1):
                    term = np.multiply.outer(term, f[l])
                out[(mu, Ellipsis) + idx] += term
            cs = norm_coefficients(ns)
            term = w[i] * blk[cs[0]][1]
            for l in range(1, N - 1):
                term = np.multiply.outer(term, blk[cs[l]][1])
            out[(nmu, Ellipsis) + idx] += term
    return out


def upsilon3(x, y, g1, g2, w, edges, nmax, centers=None, distinct=True, coeff=arg_coefficients):
    """Shear 3PCF multipoles Upsilon_{mu,n}(Theta_1, Theta_2), mu = 0..3 and
    the normalisation (index 4): array [5, nb, nb, 2 nmax + 1] complex128.
    distinct: the j = k terms (same neighbour in both slots, so
    Theta_1 = Theta_2) are removed from the double sum over neighbours."""
    raw = upsilon_n(x, y, g1, g2, w, edges, 3, nmax, centers=centers, coeff=coeff)
    if not distinct:
        return raw
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    B = beta_matrix(3)
    e2 = squared_edges(edges)
    nb = e2.size - 1
    gam = g1 + 1j * g2
    diag = np.zeros((5, nb), dtype=np.complex128)
    if centers is None:
        centers = range(x.size)
    for i in centers:
        i = int(i)
        sel, b, dx, dy = centre_neighbours(x, y, e2, i)
        if sel.size == 0:
            continue
        phi = np.arctan2(dy, dx)
        wg = w[sel] * gam[sel]
        xg = -w[i] * gam[i]          # (-1)^3 of three projected shears
        for mu, r in enumerate(B):
            # j = k: both neighbour factors taken at the same galaxy; the
            # phase is the sum of the two slot coefficients (independent of n)
            c1, c2 = coeff(r, (0,))
            f1 = wg if r[1] > 0 else np.conj(wg)
            f2 = wg if r[2] > 0 else np.conj(wg)
            v = f1 * f2 * np.exp(1j * (c1 + c2) * phi)
            t = xg if r[0] > 0 else np.conj(xg)
            diag[mu] += t * (np.bincount(b, weights=v.real, minlength=nb)
                             + 1j * np.bincount(b, weights=v.imag, minlength=nb))
        c1, c2 = norm_coefficients((0,))
        v = w[sel] * w[sel] * np.exp(1j * (c1 + c2) * phi)
        diag[4] += w[i] * (np.bincount(b, weights=v.real, minlength=nb)
                           + 1j * np.bincount(b, weights=v.imag, minlength=nb))
    out = raw.copy()
    for bb in range(nb):
        out[:, bb, bb, :] -= diag[:, bb, None]
    return out


def brute_upsilon3(x, y, g1, g2, w, edges, nmax, centers=None, distinct=True):
    """Triplet-by-triplet sum from the definitions: for every centre i and
    ordered neighbour pair (j, k) with theta_ij in Theta_1, theta_ik in
    Theta_2 (j != k if distinct), the product of the projected shears
    gamma(X; zeta) = -gamma_c e^{-2 i zeta} of Sect. 2.1 (conjugated where
    beta = -1) with zeta_0 = (phi_ij + phi_ik)/2, zeta_1 = phi_ij,
    zeta_2 = phi_ik, times w_i w_j w_k and e^{-i n phi_ijk},
    phi_ijk = phi_ik - phi_ij.  O(N m^2): tiny inputs."""
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    B = beta_matrix(3)
    e2 = squared_edges(edges)
    nb = e2.size - 1
    nn = 2 * nmax + 1
    ns = np.arange(-nmax, nmax + 1)
    gam = g1 + 1j * g2
    out = np.zeros((5, nb, nb, nn), dtype=np.complex128)
    if centers is None:
        centers = range(x.size)
    for i in centers:
        i = int(i)
        dx = x - x[i]
        dy = y - y[i]
        r2 = dx * dx + dy * dy
        b = np.searchsorted(e2, r2, side="right") - 1
        nbr = np.nonzero((b >= 0) & (b < nb))[0]
        if nbr.size == 0:
            continue
        phi = np.arctan2(dy[nbr], dx[nbr])
        J, K = (a.ravel() for a in np.meshgrid(np.arange(nbr.size), np.arange(nbr.size), indexing="ij"))
        if distinct:
            keep = J != K
            J, K = J[keep], K[keep]
        if J.size == 0:
            continue
        p1, p2 = phi[J], phi[K]
        rot = (projected(gam[i], (p1 + p2) / 2),
               projected(gam[nbr][J], p1),
               projected(gam[nbr][K], p2))
        wt = w[i] * w[nbr][J] * w[nbr][K]
        E = np.exp(-1j * np.multiply.outer(p2 - p1, ns))
        bj, bk = b[nbr][J], b[nbr][K]
        for mu, r in enumerate(B):
            p = wt.astype(np.complex128)
            for l in range(3):
                p = p * (rot[l] if r[l] > 0 else np.conj(rot[l]))
            np.add.at(out[mu], (bj, bk), p[:, None] * E)
        np.add.at(out[4], (bj, bk), wt[:, None] * E)
    return out
