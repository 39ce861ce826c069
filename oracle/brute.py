"""Brute-force quadruplet enumeration of the shear 4PCF multipoles.

TEST INFRASTRUCTURE ONLY (see ``oracle/estimator.py``).  O(N m^3) in the
number m of neighbours per centre: for tiny catalogues only.

It evaluates the definitions directly, quadruplet by quadruplet, without the
multipole factorisation:

* projected shear gamma(X; zeta) = -gamma_c e^{-2 i zeta}     (Sect. 2.1);
* natural components Gamma_0..7 = products of four projected shears with
  the conjugation pattern of Sect. 2.2 (Gamma_0 read with X_2 in its third
  slot, Gamma_4 with zeta_1 in its second slot);
* x-projection zeta_0 = (phi_1 + phi_3)/2, zeta_k = phi_k      (Sect. 2.2);
* Upsilon_{mu,n} = sum_{i,j,k,l} w_i w_j w_k w_l P_mu
  B(theta_ij in T1) B(theta_ik in T2) B(theta_il in T3)
  e^{-i n2 phi_ijk - i n3 phi_ijl},  phi_ijk = phi_ik - phi_ij  (Sect. 3, the
  quadruplet estimator transformed to multipoles as in Sect. 3.1);
* N: the same with P = 1;
* ``distinct``: only j, k, l pairwise distinct (App. A.1).
"""
from __future__ import annotations

import numpy as np

# conjugated slots (X_0, X_1, X_2, X_3) for Gamma_0 ... Gamma_7
CONJ = [
    (0, 0, 0, 0),
    (1, 0, 0, 0),
    (0, 1, 0, 0),
    (0, 0, 1, 0),
    (0, 0, 0, 1),
    (1, 1, 0, 0),
    (1, 0, 1, 0),
    (1, 0, 0, 1),
]


def projected(gamma_c, zeta):
    """gamma(theta; zeta) = gamma_t + i gamma_x = -gamma_c exp(-2 i zeta)."""
    return -gamma_c * np.exp(-2j * zeta)


def brute_upsilon(x, y, g1, g2, w, edges, nmax, distinct=True, centers=None):
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    e2 = np.asarray(edges, dtype=np.float64) ** 2
    nb = e2.size - 1
    nn = 2 * nmax + 1
    ns = np.arange(-nmax, nmax + 1)
    gam = g1 + 1j * g2
    out = np.zeros((9, nb * nb * nb, nn, nn), dtype=np.complex128)
    if centers is None:
        centers = range(x.size)
    for i in centers:
        dx = x - x[i]
        dy = y - y[i]
        r2 = dx * dx + dy * dy
        b = np.searchsorted(e2, r2, side="right") - 1
        nbr = np.nonzero((b >= 0) & (b < nb))[0]
        m = nbr.size
        if m == 0:
            continue
        phi = np.arctan2(dy[nbr], dx[nbr])
        bj = b[nbr]
        J, K, L = (a.ravel() for a in np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"))
        if distinct:
            keep = (J != K) & (J != L) & (K != L)
            J, K, L = J[keep], K[keep], L[keep]
        if J.size == 0:
            continue
        p1, p2, p3 = phi[J], phi[K], phi[L]
        zeta = (0.5 * (p1 + p3), p1, p2, p3)
        gc = (np.full(J.size, gam[i]), gam[nbr][J], gam[nbr][K], gam[nbr][L])
        s = [projected(gc[a], zeta[a]) for a in range(4)]
        wt = w[i] * w[nbr][J] * w[nbr][K] * w[nbr][L]
        prods = np.empty((9, J.size), dtype=np.complex128)
        for mu, pattern in enumerate(CONJ):
            p = wt.astype(np.complex128)
            for a in range(4):
                p = p * (np.conj(s[a]) if pattern[a] else s[a])
            prods[mu] = p
        prods[8] = wt
        phi12 = p2 - p1
        phi13 = p3 - p1
        E2 = np.exp(-1j * np.multiply.outer(phi12, ns))       # [t, n2]
        E3 = np.exp(-1j * np.multiply.outer(phi13, ns))       # [t, n3]
        cidx = (bj[J] * nb + bj[K]) * nb + bj[L]
        order = np.argsort(cidx, kind="stable")
        cs = cidx[order]
        starts = np.flatnonzero(np.r_[True, cs[1:] != cs[:-1]])
        ends = np.r_[starts[1:], cs.size]
        for s0, s1 in zip(starts, ends):
            t = order[s0:s1]
            out[:, cs[s0]] += np.einsum("mt,tx,ty->mxy", prods[:, t], E2[t], E3[t])
    return out.reshape(9, nb, nb, nb, nn, nn)


def brute_angular_bins(x, y, g1, g2, w, edges, nphi, distinct=True, centers=None):
    """Quadruplet sums binned in (Theta_1, Theta_2, Theta_3, Phi_12, Phi_13)
    with nphi linear angular bins on [0, 2 pi): the numerator Upsilon_mu and
    the denominator N of the quadruplet estimator (Sect. 3), 9 x nb^3 x nphi^2."""
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    e2 = np.asarray(edges, dtype=np.float64) ** 2
    nb = e2.size - 1
    gam = g1 + 1j * g2
    out = np.zeros((9, nb, nb, nb, nphi, nphi), dtype=np.complex128)
    if centers is None:
        centers = range(x.size)
    two_pi = 2.0 * np.pi
    for i in centers:
        dx = x - x[i]
        dy = y - y[i]
        r2 = dx * dx + dy * dy
        b = np.searchsorted(e2, r2, side="right") - 1
        nbr = np.nonzero((b >= 0) & (b < nb))[0]
        m = nbr.size
        if m == 0:
            continue
        phi = np.arctan2(dy[nbr], dx[nbr])
        bj = b[nbr]
        J, K, L = (a.ravel() for a in np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"))
        if distinct:
            keep = (J != K) & (J != L) & (K != L)
            J, K, L = J[keep], K[keep], L[keep]
        if J.size == 0:
            continue
        p1, p2, p3 = phi[J], phi[K], phi[L]
        zeta = (0.5 * (p1 + p3), p1, p2, p3)
        gc = (np.full(J.size, gam[i]), gam[nbr][J], gam[nbr][K], gam[nbr][L])
        s = [projected(gc[a], zeta[a]) for a in range(4)]
        wt = w[i] * w[nbr][J] * w[nbr][K] * w[nbr][L]
        a12 = np.mod(p2 - p1, two_pi)
        a13 = np.mod(p3 - p1, two_pi)
        ia = np.minimum((a12 / two_pi * nphi).astype(np.int64), nphi - 1)
        ib = np.minimum((a13 / two_pi * nphi).astype(np.int64), nphi - 1)
        for mu in range(9):
            if mu < 8:
                p = wt.astype(np.complex128)
                for a in range(4):
                    p = p * (np.conj(s[a]) if CONJ[mu][a] else s[a])
            else:
                p = wt.astype(np.complex128)
            np.add.at(out[mu], (bj[J], bj[K], bj[L], ia, ib), p)
    return out
