"""Multipoles -> bin-averaged natural components (FP64 tail), oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/estimator.py``).

The multipole expansion of Sect. 3.1 gives the angular density
Upsilon(phi12, phi13) = (2 pi)^-2 sum_n Upsilon_n e^{i n2 phi12} e^{i n3 phi13}.
Integrating it over linear angular bins Phi_a x Phi_b (the angular part of the
bin average of Sect. 2.3) gives the binned quadruplet sums

    Ubar(Phi_a, Phi_b) = (2 pi)^-2 sum_n Upsilon_n I_{n2}(Phi_a) I_{n3}(Phi_b),
    I_0(Phi) = |Delta Phi|,  I_m(Phi) = (e^{i m Phi_up} - e^{i m Phi_low}) / (i m),

and the estimator of Sect. 3 is the ratio Gamma_mu = Ubar_mu / Nbar.  The
factors |Delta Phi| of the bin average cancel in that ratio.
"""
from __future__ import annotations

import numpy as np


def angular_integrals(nmax: int, nphi: int) -> np.ndarray:
    """I[m + nmax, a] = int_{Phi_a} e^{i m phi} dphi, linear bins on [0, 2 pi)."""
    ed = np.linspace(0.0, 2.0 * np.pi, nphi + 1)
    out = np.empty((2 * nmax + 1, nphi), dtype=np.complex128)
    for idx, m in enumerate(range(-nmax, nmax + 1)):
        if m == 0:
            out[idx] = ed[1:] - ed[:-1]
        else:
            out[idx] = (np.exp(1j * m * ed[1:]) - np.exp(1j * m * ed[:-1])) / (1j * m)
    return out


def binned_from_multipoles(ups: np.ndarray, nphi: int) -> np.ndarray:
    """[9, nb, nb, nb, 2n+1, 2n+1] multipoles -> [9, nb, nb, nb, nphi, nphi]
    binned quadruplet sums Ubar (index 8 = Nbar)."""
    nmax = (ups.shape[-1] - 1) // 2
    I = angular_integrals(nmax, nphi)
    return np.einsum("...xy,xa,yb->...ab", ups, I, I) / (2.0 * np.pi) ** 2


def natural_components(ups: np.ndarray, nphi: int):
    """(Gamma[8, nb, nb, nb, nphi, nphi] complex, Nbar[nb, nb, nb, nphi, nphi]
    real).  Gamma is Ubar_mu / Nbar where Nbar != 0, else 0."""
    return _ratio(binned_from_multipoles(ups, nphi))


def natural_components_triplets(ups: np.ndarray, nphi: int, triplets):
    """The conversion above for the listed radial-bin triplets (b1, b2, b3)
    only: (Gamma[8, ntrip, nphi, nphi], Nbar[ntrip, nphi, nphi])."""
    t = np.asarray(triplets, dtype=np.int64).reshape(-1, 3)
    return natural_components_selected(ups[:, t[:, 0], t[:, 1], t[:, 2]], nphi)


def natural_components_selected(sel: np.ndarray, nphi: int):
    """The same from the multipoles of the triplets alone, sel[9, ntrip,
    2n+1, 2n+1] (as ``upsilon_triplets`` returns them)."""
    return _ratio(binned_from_multipoles(sel[:, :, None, None], nphi)[:, :, 0, 0])


def _ratio(binned):
    nbar = binned[8].real
    with np.errstate(divide="ignore", invalid="ignore"):
        gam = np.where(nbar != 0.0, binned[:8] / np.where(nbar != 0.0, nbar, 1.0), 0.0)
    return gam, nbar
