"""FP64 CPU oracle of the multipole-based shear 4PCF estimator.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
reference the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the library never does, and it shares no code with the library.

It follows Porth et al. (2025), "Efficient estimation of fourth-order shear
correlation functions", Sect. 3 and Appendix A.1:

1. pair binning:   theta_ij in Theta_b, with half-open bins [e_b, e_{b+1})
                   decided on r^2 = dx*dx + dy*dy against squared edges
                   (Sect. 3, the bin selection function B);
2. per-centre multipoles G_k, W_k (Sect. 3.1, the derivation of the n-th
   multipole of Upsilon_0 and Eq. for N_n) and the multiple-counting
   families (Appendix A.1, Table 1), computed directly as
   sum_j v_j exp(i k phi_ij) with phi_ij = atan2(dy, dx);
3. contraction     Upsilon_{mu,n}(T1,T2,T3) = sum_i x_i A B C with the factor
                   table of Sect. 3.1 (the equations for Upsilon_0..7 and N);
4. the double- and triple-counting corrections of Appendix A.1 / Table 1,
   applied by inclusion-exclusion: minus the three pair terms, plus twice the
   triple term.

All arithmetic is numpy float64 / complex128.  Where the paper is silent or
garbled, the readings used are:
* G_k = sum_j w_j gamma_j e^{+ik phi_ij} and W_k = sum_j w_j e^{+ik phi_ij}
  (the "defined as in P24" blocks, fixed by the derivation of Upsilon_0);
* Gamma_0 reads gamma(X_2; zeta_2) in its third slot and Gamma_4 reads
  gamma(X_1; zeta_1) in its second slot (both as the multipole equations
  require);
* the App. A.1 multipole formula for the scalar corrections is read as the
  inclusion-exclusion of Table 1 summands: each pair correction is
  sum_i x_i * (Table 1 block at the equal bin) * (remaining factor at the
  other bin), the triple correction is sum_i x_i * (Table 1 block);
* "j != l != l" means j, k, l pairwise distinct.
"""
from __future__ import annotations

import numpy as np

NCORR = 9          # Upsilon_0..7 and the normalisation N (index 8)

# ---------------------------------------------------------------------------
# Factor table of Sect. 3.1 (multipole equations for Upsilon_0 ... Upsilon_7
# and N_n).  An order spec (a, b, c) means k = a*n2 + b*n3 + c.
# Centre factor: 'g' = w_i gamma_i, 'gc' = its conjugate, 'w' = w_i.
# Each multipole factor: (family, conjugate?, order spec).
# ---------------------------------------------------------------------------
FACTORS = [
    # mu  x      A (Theta_1)               B (Theta_2)             C (Theta_3)
    ("g",  ("G", False, (1, 1, -3)),  ("G", False, (-1, 0, -2)), ("G", False, (0, -1, -3))),
    ("gc", ("G", False, (1, 1, -1)),  ("G", False, (-1, 0, -2)), ("G", False, (0, -1, -1))),
    ("g",  ("G", True, (-1, -1, -1)), ("G", False, (-1, 0, -2)), ("G", False, (0, -1, -3))),
    ("g",  ("G", False, (1, 1, -3)),  ("G", True, (1, 0, -2)),   ("G", False, (0, -1, -3))),
    ("g",  ("G", False, (1, 1, -3)),  ("G", False, (-1, 0, -2)), ("G", True, (0, 1, -1))),
    ("gc", ("G", True, (-1, -1, -3)), ("G", False, (-1, 0, -2)), ("G", False, (0, -1, -1))),
    ("gc", ("G", False, (1, 1, -1)),  ("G", True, (1, 0, -2)),   ("G", False, (0, -1, -1))),
    ("gc", ("G", False, (1, 1, -1)),  ("G", False, (-1, 0, -2)), ("G", True, (0, 1, -3))),
    ("w",  ("W", False, (1, 1, 0)),   ("W", False, (-1, 0, 0)),  ("W", False, (0, -1, 0))),
]

# ---------------------------------------------------------------------------
# Table 1 (App. A.1): multiple-counting blocks for Theta_1=Theta_2,
# Theta_1=Theta_3, Theta_2=Theta_3 and Theta_1=Theta_2=Theta_3.
# Families: Q <-> (w e_c)^2, A <-> |w e_c|^2, T <-> (w e_c)^3,
# M <-> (w e_c)^2 (w e_c)^*, V <-> w^2, U <-> w^3; order spec as above.
# ---------------------------------------------------------------------------
TABLE1 = [
    (("Q", (0, 1, -5)), ("Q", (1, 0, -6)), ("Q", (-1, -1, -5)), ("T", (0, 0, -8))),
    (("Q", (0, 1, -3)), ("Q", (1, 0, -2)), ("Q", (-1, -1, -3)), ("T", (0, 0, -4))),
    (("A", (0, 1, -1)), ("A", (1, 0, -2)), ("Q", (-1, -1, -5)), ("M", (0, 0, -4))),
    (("A", (0, 1, -1)), ("Q", (1, 0, -6)), ("A", (-1, -1, -1)), ("M", (0, 0, -4))),
    (("Q", (0, 1, -5)), ("A", (1, 0, -2)), ("A", (-1, -1, -1)), ("M", (0, 0, -4))),
    (("A", (0, 1, 1)),  ("A", (1, 0, 2)),  ("Q", (-1, -1, -3)), ("M", (0, 0, 0))),
    (("A", (0, 1, 1)),  ("Q", (1, 0, -2)), ("A", (-1, -1, 1)),  ("M", (0, 0, 0))),
    (("Q", (0, 1, -3)), ("A", (1, 0, 2)),  ("A", (-1, -1, 1)),  ("M", (0, 0, 0))),
    (("V", (0, 1, 0)),  ("V", (1, 0, 0)),  ("V", (-1, -1, 0)),  ("U", (0, 0, 0))),
]


def family_orders(nmax: int) -> dict:
    """Range of multipole orders k needed by each family for |n2|,|n3| <= nmax
    (derived from the order specs above)."""
    ranges = {}
    specs = []
    for mu in range(NCORR):
        for f in FACTORS[mu][1:]:
            specs.append((f[0], f[2]))
        for f in TABLE1[mu]:
            specs.append(f)
    for fam, (a, b, c) in specs:
        vals = [a * n2 + b * n3 + c for n2 in (-nmax, nmax) for n3 in (-nmax, nmax)]
        lo, hi = min(vals), max(vals)
        if fam in ranges:
            lo = min(lo, ranges[fam][0])
            hi = max(hi, ranges[fam][1])
        ranges[fam] = (lo, hi)
    return ranges


def squared_edges(edges) -> np.ndarray:
    e = np.asarray(edges, dtype=np.float64)
    return e * e


def check_inputs(x, y, g1, g2, w, edges, nmax):
    e = np.asarray(edges, dtype=np.float64)
    if e.ndim != 1 or e.size < 2 or not np.all(np.isfinite(e)):
        raise ValueError("edges must be a finite 1-d array of length >= 2")
    if not (e[0] > 0.0) or not np.all(np.diff(e) > 0.0):
        raise ValueError("edges must be strictly increasing with edges[0] > 0")
    if nmax < 0:
        raise ValueError("nmax must be >= 0")
    for a in (x, y, g1, g2, w):
        if not np.all(np.isfinite(a)):
            raise ValueError("catalogue contains non-finite values")


def centre_neighbours(x, y, e2, i):
    """Neighbours j of centre i with theta_ij in [e_0, e_nb), their bins and
    separation vector.  r^2 is formed as two products and one sum (no fused
    multiply-add) and compared against the squared edges; the bin is the
    largest b with e2[b] <= r^2."""
    dx = x - x[i]
    dy = y - y[i]
    r2 = dx * dx + dy * dy
    nb = e2.size - 1
    b = np.searchsorted(e2, r2, side="right") - 1
    sel = np.nonzero((b >= 0) & (b < nb))[0]
    return sel, b[sel], dx[sel], dy[sel]


def bin_counts(x, y, edges, centers):
    """Integer number of neighbours per (centre, bin)."""
    e2 = squared_edges(edges)
    nb = e2.size - 1
    out = np.zeros((len(centers), nb), dtype=np.int64)
    for c, i in enumerate(centers):
        _, b, _, _ = centre_neighbours(x, y, e2, int(i))
        out[c] = np.bincount(b, minlength=nb)
    return out


def _family_values(fam, wg, w):
    if fam == "G":
        return wg
    if fam == "W":
        return w.astype(np.complex128)
    if fam == "Q":
        return wg * wg
    if fam == "A":
        return (np.abs(wg) ** 2).astype(np.complex128)
    if fam == "V":
        return (w * w).astype(np.complex128)
    if fam == "T":
        return wg * wg * wg
    if fam == "M":
        return wg * wg * np.conj(wg)
    if fam == "U":
        return (w * w * w).astype(np.complex128)
    raise KeyError(fam)


def centre_multipoles(x, y, g1, g2, w, e2, nmax, i, ranges=None):
    """All multipole families of centre i: dict fam -> complex [nb, K] over the
    orders ``ranges[fam]`` (inclusive), plus 'counts' -> int64 [nb].
    F_k(theta_i, Theta_b) = sum_{j: theta_ij in Theta_b} v_j exp(i k phi_ij)."""
    if ranges is None:
        ranges = family_orders(nmax)
    nb = e2.size - 1
    j, b, dx, dy = centre_neighbours(x, y, e2, i)
    phi = np.arctan2(dy, dx)
    onehot = np.zeros((nb, j.size))
    onehot[b, np.arange(j.size)] = 1.0
    wg = w[j] * (g1[j] + 1j * g2[j])
    wj = w[j]
    out = {"counts": np.bincount(b, minlength=nb).astype(np.int64)}
    for fam, (lo, hi) in ranges.items():
        ks = np.arange(lo, hi + 1)
        vals = _family_values(fam, wg, wj)
        ph = np.exp(1j * np.multiply.outer(phi, ks))
        out[fam] = onehot @ (vals[:, None] * ph)
    return out


def multipoles(x, y, g1, g2, w, edges, nmax, centers):
    """Stacked per-centre multipoles: dict fam -> complex [nc, nb, K]."""
    e2 = squared_edges(edges)
    ranges = family_orders(nmax)
    per = [centre_multipoles(x, y, g1, g2, w, e2, nmax, int(i), ranges) for i in centers]
    out = {k: np.stack([p[k] for p in per]) for k in per[0]} if per else {}
    out["ranges"] = ranges
    return out


def _centre_factor(kind, g1, g2, w, centers):
    c = np.asarray(centers)
    wg = w[c] * (g1[c] + 1j * g2[c])
    if kind == "g":
        return wg
    if kind == "gc":
        return np.conj(wg)
    return w[c].astype(np.complex128)


def _gather(mp, fam, spec, nmax, conj=False):
    """Block values at order k = a*n2 + b*n3 + c for all (n2, n3):
    complex [nc, nb, 2nmax+1, 2nmax+1]."""
    lo, _ = mp["ranges"][fam]
    n = np.arange(-nmax, nmax + 1)
    a, b, c = spec
    k = a * n[:, None] + b * n[None, :] + c
    vals = mp[fam][:, :, k - lo]
    return np.conj(vals) if conj else vals


def contract(mp, g1, g2, w, centers, nmax, nb, distinct=True):
    """Upsilon_{mu,(n2,n3)}(T1,T2,T3) summed over the given centres, for all
    nine correlators.  Returns complex [9, nb, nb, nb, 2nmax+1, 2nmax+1]."""
    nn = 2 * nmax + 1
    out = np.zeros((NCORR, nb, nb, nb, nn, nn), dtype=np.complex128)
    if len(centers) == 0:
        return out
    nc = len(centers)
    for mu in range(NCORR):
        xk, fa, fb, fc = FACTORS[mu]
        x = _centre_factor(xk, g1, g2, w, centers)
        A = _gather(mp, fa[0], fa[2], nmax, fa[1])      # [i, b1, n2, n3]
        B = _gather(mp, fb[0], fb[2], nmax, fb[1])      # [i, b2, n2, n3]
        C = _gather(mp, fc[0], fc[2], nmax, fc[1])      # [i, b3, n2, n3]
        xa = x[:, None, None, None] * A
        # raw sum over centres, one (n2, n3) at a time as a batched matmul:
        # out[b1, b2, b3, z] = sum_i (xA)[i,b1,z] B[i,b2,z] C[i,b3,z]
        L = (xa[:, :, None] * B[:, None]).reshape(nc, nb * nb, nn * nn)
        R = C.reshape(nc, nb, nn * nn)
        raw = np.matmul(L.transpose(2, 1, 0), R.transpose(2, 0, 1))   # [z, b1b2, b3]
        out[mu] = raw.transpose(1, 2, 0).reshape(nb, nb, nb, nn, nn)
        if not distinct:
            continue
        t12, t13, t23, t123 = TABLE1[mu]
        c12 = _gather(mp, t12[0], t12[1], nmax)
        c13 = _gather(mp, t13[0], t13[1], nmax)
        c23 = _gather(mp, t23[0], t23[1], nmax)
        t3 = _gather(mp, t123[0], t123[1], nmax)
        # Theta_1 = Theta_2 (j = k): sum_i x c12(T1) C(T3)
        p12 = np.einsum("i,iaz,icz->acz", x, c12.reshape(nc, nb, -1), R)
        # Theta_1 = Theta_3 (j = l): sum_i x c13(T1) B(T2)
        p13 = np.einsum("i,iaz,ibz->abz", x, c13.reshape(nc, nb, -1), B.reshape(nc, nb, -1))
        # Theta_2 = Theta_3 (k = l): sum_i x A(T1) c23(T2)
        p23 = np.einsum("iaz,ibz->abz", xa.reshape(nc, nb, -1), c23.reshape(nc, nb, -1))
        # Theta_1 = Theta_2 = Theta_3 (j = k = l): sum_i x t(T1)
        p3 = np.einsum("i,iaz->az", x, t3.reshape(nc, nb, -1))
        o = out[mu].reshape(nb, nb, nb, nn * nn)
        for a in range(nb):
            o[a, a, :, :] -= p12[a]
            o[a, :, a, :] -= p13[a]
            o[:, a, a, :] -= p23[:, a]
            o[a, a, a, :] += 2.0 * p3[a]
    return out


def contract_triplets(mp, g1, g2, w, centers, nmax, triplets, distinct=True):
    """The sums of ``contract`` at the listed radial-bin triplets (b1, b2, b3)
    only: complex [9, ntrip, 2nmax+1, 2nmax+1].  Each element is the sum over
    centres of x A(b1) B(b2) C(b3); for distinct quadruplets the App. A.1
    terms are removed where bins coincide: x c12(b1) C(b3) when b1 = b2,
    x c13(b1) B(b2) when b1 = b3, x A(b1) c23(b2) when b2 = b3, and twice
    x t(b1) added back when all three are equal."""
    t = np.asarray(triplets, dtype=np.int64).reshape(-1, 3)
    nn = 2 * nmax + 1
    out = np.zeros((NCORR, len(t), nn, nn), dtype=np.complex128)
    if len(centers) == 0 or len(t) == 0:
        return out
    b1, b2, b3 = t[:, 0], t[:, 1], t[:, 2]
    e12, e13, e23 = b1 == b2, b1 == b3, b2 == b3
    e123 = e12 & e23
    for mu in range(NCORR):
        xk, fa, fb, fc = FACTORS[mu]
        x = _centre_factor(xk, g1, g2, w, centers)[:, None, None, None]
        A = _gather(mp, fa[0], fa[2], nmax, fa[1])[:, b1]      # [i, t, n2, n3]
        B = _gather(mp, fb[0], fb[2], nmax, fb[1])[:, b2]
        C = _gather(mp, fc[0], fc[2], nmax, fc[1])[:, b3]
        out[mu] = np.sum(x * A * B * C, axis=0)
        if not distinct:
            continue
        t12, t13, t23, t123 = TABLE1[mu]
        c12 = _gather(mp, t12[0], t12[1], nmax)
        c13 = _gather(mp, t13[0], t13[1], nmax)
        c23 = _gather(mp, t23[0], t23[1], nmax)
        t3 = _gather(mp, t123[0], t123[1], nmax)
        out[mu][e12] -= np.sum(x * c12[:, b1[e12]] * C[:, e12], axis=0)
        out[mu][e13] -= np.sum(x * c13[:, b1[e13]] * B[:, e13], axis=0)
        out[mu][e23] -= np.sum(x * A[:, e23] * c23[:, b2[e23]], axis=0)
        out[mu][e123] += 2.0 * np.sum(x * t3[:, b1[e123]], axis=0)
    return out


def upsilon_triplets(x, y, g1, g2, w, edges, nmax, triplets, centers=None, distinct=True,
                     chunk=16):
    """``upsilon`` at the listed radial-bin triplets only: complex
    [9, ntrip, 2nmax+1, 2nmax+1], element t equal to
    upsilon(...)[:, b1_t, b2_t, b3_t].  For bin counts whose full tensor does
    not fit in memory (65 bins at nmax 15 is 38 GB)."""
    x, y, g1, g2, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    check_inputs(x, y, g1, g2, w, edges, nmax)
    if centers is None:
        centers = np.arange(x.size)
    centers = np.asarray(centers, dtype=np.int64)
    t = np.asarray(triplets, dtype=np.int64).reshape(-1, 3)
    nb = len(edges) - 1
    if t.size and (t.min() < 0 or t.max() >= nb):
        raise ValueError("triplet bin out of range")
    nn = 2 * nmax + 1
    out = np.zeros((NCORR, len(t), nn, nn), dtype=np.complex128)
    for s in range(0, len(centers), chunk):
        c = centers[s:s + chunk]
        mp = multipoles(x, y, g1, g2, w, edges, nmax, c)
        out += contract_triplets(mp, g1, g2, w, c, nmax, t, distinct)
    return out


def upsilon(x, y, g1, g2, w, edges, nmax, centers=None, distinct=True,
            chunk=256):
    """The 4PCF multipoles Upsilon_{mu,(n2,n3)}(T1,T2,T3), mu = 0..7, and
    N_{(n2,n3)} (index 8), complex128 [9, nb, nb, nb, 2nmax+1, 2nmax+1].
    ``centers``: indices of the galaxies used as the base point X_0 (default
    all); every galaxy stays a neighbour.  ``distinct``: subtract the
    double/triple-counting terms (quadruplets of four distinct galaxies)."""
    x, y, g1, g2, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    check_inputs(x, y, g1, g2, w, edges, nmax)
    nb = len(edges) - 1
    if centers is None:
        centers = np.arange(x.size)
    centers = np.asarray(centers, dtype=np.int64)
    nn = 2 * nmax + 1
    out = np.zeros((NCORR, nb, nb, nb, nn, nn), dtype=np.complex128)
    for s in range(0, len(centers), chunk):
        c = centers[s:s + chunk]
        mp = multipoles(x, y, g1, g2, w, edges, nmax, c)
        out += contract(mp, g1, g2, w, c, nmax, nb, distinct)
    return out


def abs_bound(x, y, g1, g2, w, edges, centers=None, order=4):
    """Scale of every term of the estimator, per radial-bin tuple: the sum over
    centres of the absolute values of the centre factor and of the per-bin
    block factors.  Since |e^{i k phi}| = 1, each block satisfies
    |F_k(theta_i, Theta_b)| <= sum_{j in b} |v_j|, so by the triangle
    inequality every element of Upsilon (raw or over distinct quadruplets, a
    subset of the terms) is bounded by
      S[0](b1,b2,b3) = sum_i |w_i gamma_i| Gbar_i(b1) Gbar_i(b2) Gbar_i(b3)
    for the shear correlators and by S[1] (the same with w, Wbar) for N,
    Gbar_i(b) = sum_{j in b} |w_j gamma_j|, Wbar_i(b) = sum_{j in b} |w_j|.
    With positive weights, S[1] equals the raw N_{(0,0)}.  order=3 gives the
    two-bin analogue [2, nb, nb] for the shear 3PCF."""
    x, y, g1, g2, w = (np.asarray(a, dtype=np.float64) for a in (x, y, g1, g2, w))
    e2 = squared_edges(edges)
    nb = e2.size - 1
    if centers is None:
        centers = range(x.size)
    ag = np.abs(w * (g1 + 1j * g2))
    aw = np.abs(w)
    out = np.zeros((2,) + (nb,) * (order - 1))
    for i in centers:
        i = int(i)
        j, b, _, _ = centre_neighbours(x, y, e2, i)
        for k, (xc, v) in enumerate(((ag[i], ag), (aw[i], aw))):
            s = np.bincount(b, weights=v[j], minlength=nb)
            t = xc * s
            for _ in range(order - 2):
                t = np.multiply.outer(t, s)
            out[k] += t
    return out


def _worker(args):
    x, y, g1, g2, w, edges, nmax, centers, distinct = args
    return upsilon(x, y, g1, g2, w, edges, nmax, centers, distinct)


def _bound_worker(args):
    x, y, g1, g2, w, edges, centers, order = args
    return abs_bound(x, y, g1, g2, w, edges, centers, order)


def abs_bound_parallel(x, y, g1, g2, w, edges, centers, order=4, processes=1):
    """``abs_bound`` over centre chunks in a process pool, added in chunk order."""
    centers = np.asarray(centers, dtype=np.int64)
    if processes <= 1:
        return abs_bound(x, y, g1, g2, w, edges, centers, order)
    import multiprocessing as mp
    chunks = np.array_split(centers, processes)
    with mp.get_context("fork").Pool(processes) as pool:
        res = pool.map(_bound_worker, [(x, y, g1, g2, w, edges, c, order) for c in chunks])
    out = res[0]
    for r in res[1:]:
        out = out + r
    return out


def _triplet_worker(args):
    x, y, g1, g2, w, edges, nmax, triplets, centers, distinct = args
    return upsilon_triplets(x, y, g1, g2, w, edges, nmax, triplets, centers, distinct)


def upsilon_triplets_parallel(x, y, g1, g2, w, edges, nmax, triplets, centers, distinct=True,
                              processes=1):
    """``upsilon_triplets`` over centre chunks in a process pool, added in
    chunk order."""
    centers = np.asarray(centers, dtype=np.int64)
    if processes <= 1:
        return upsilon_triplets(x, y, g1, g2, w, edges, nmax, triplets, centers, distinct)
    import multiprocessing as mp
    chunks = np.array_split(centers, processes)
    with mp.get_context("fork").Pool(processes) as pool:
        res = pool.map(_triplet_worker, [(x, y, g1, g2, w, edges, nmax, triplets, c, distinct)
                                         for c in chunks])
    out = res[0]
    for r in res[1:]:
        out = out + r
    return out


def upsilon_parallel(x, y, g1, g2, w, edges, nmax, centers=None, distinct=True,
                     processes=1, parts=None):
    """``upsilon`` over centre chunks in a process pool; partial results are
    added in chunk order (deterministic)."""
    if centers is None:
        centers = np.arange(len(x))
    centers = np.asarray(centers, dtype=np.int64)
    if processes <= 1:
        return upsilon(x, y, g1, g2, w, edges, nmax, centers, distinct)
    import multiprocessing as mp
    parts = parts or processes
    chunks = np.array_split(centers, parts)
    with mp.get_context("fork").Pool(processes) as pool:
        res = pool.map(_worker, [(x, y, g1, g2, w, edges, nmax, c, distinct) for c in chunks])
    out = res[0]
    for r in res[1:]:
        out = out + r
    return out
