"""Seeded synthetic galaxy catalogues and binning set-ups.

This module only draws inputs: positions, shears, weights and radial bin
edges.  It holds none of the estimator's arithmetic, so both the FP64 CPU
oracle (``oracle/``) and the GPU library may be fed from it without sharing
any code with each other.

Every generator takes an integer seed and uses ``numpy.random.default_rng``;
the draw order inside each generator is fixed and documented, so that a seed
fully determines the catalogue.

Units: flat-sky positions in arcmin, no periodic wrap; shear is the Cartesian
complex shear g1 + i g2; weights are positive reals.

Workloads (the paper's data are stand-ins; see the estimator paper, Sect. 4.1
for the GRF mock recipe it uses, and Sect. 6 for the DES-like shape noise):

* ``uniform_catalogue``  -- uniform positions, i.i.d. Gaussian shears;
* ``grf_catalogue``      -- uniform positions, shear from a Gaussian random
  convergence field with a power-law spectrum via Kaiser-Squires, plus shape
  noise (nearest-grid-point assignment of pixel shears);
* ``lognormal_catalogue`` -- positions drawn from a lognormal density field,
  shear as in ``grf_catalogue``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Catalogue", "log_edges", "uniform_catalogue", "grf_fields",
    "grf_catalogue", "lognormal_catalogue", "subset", "workload",
    "serving_requests",
]


@dataclasses.dataclass
class Catalogue:
    """Structure-of-arrays catalogue (all float64, length n)."""
    x: np.ndarray
    y: np.ndarray
    g1: np.ndarray
    g2: np.ndarray
    w: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return self.x, self.y, self.g1, self.g2, self.w


def log_edges(theta_min: float, theta_max: float, nbins: int) -> np.ndarray:
    """Logarithmically spaced radial bin edges e_b = tmin (tmax/tmin)^(b/nbins)."""
    b = np.arange(nbins + 1, dtype=np.float64)
    e = theta_min * (theta_max / theta_min) ** (b / nbins)
    e[0] = theta_min
    e[-1] = theta_max
    return e


def uniform_catalogue(seed: int, n: int, side: float, sigma: float = 0.26,
                      wlo: float = 0.5, whi: float = 1.5) -> Catalogue:
    """Uniform positions on [0, side)^2, shear components ~ N(0, sigma^2) i.i.d.,
    weights ~ U[wlo, whi).  Draw order: x, y, g1, g2, w."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, side, n)
    y = rng.uniform(0.0, side, n)
    g1 = rng.normal(0.0, sigma, n)
    g2 = rng.normal(0.0, sigma, n)
    w = rng.uniform(wlo, whi, n)
    return Catalogue(x, y, g1, g2, w)


def grf_fields(rng: np.random.Generator, ngrid: int, side: float,
               slope: float = -1.2, sigma: float = 0.02):
    """Gaussian random convergence field on an ngrid^2 periodic grid of the given
    side, power spectrum P(l) ~ l^slope (l = 0 mode removed), rescaled to a
    pixel standard deviation ``sigma``; and the matching shear field from the
    Kaiser-Squires kernel (l1 + i l2)^2 / l^2 with l1 along x (array axis 1).

    Returns (kappa[ny, nx] float64, gamma[ny, nx] complex128)."""
    white = rng.standard_normal((ngrid, ngrid))
    wk = np.fft.fft2(white)
    del white
    f = np.fft.fftfreq(ngrid, d=side / ngrid) * (2.0 * math.pi)
    l1 = f[None, :]
    l2 = f[:, None]
    lsq = l1 * l1 + l2 * l2
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where(lsq > 0.0, lsq ** (slope / 4.0), 0.0)
    wk *= amp
    del amp
    kappa = np.fft.ifft2(wk).real
    scale = sigma / kappa.std()
    kappa *= scale
    with np.errstate(divide="ignore", invalid="ignore"):
        ks = np.where(lsq > 0.0, ((l1 * l1 - l2 * l2) + 2j * l1 * l2) / lsq, 0.0)
    del lsq
    wk *= ks
    del ks
    gamma = np.fft.ifft2(wk)
    gamma *= scale
    return kappa, gamma


def _ngp(field: np.ndarray, x: np.ndarray, y: np.ndarray, side: float):
    ng = field.shape[0]
    ix = np.clip((x * (ng / side)).astype(np.int64), 0, ng - 1)
    iy = np.clip((y * (ng / side)).astype(np.int64), 0, ng - 1)
    return field[iy, ix]


def grf_catalogue(seed: int, n: int, side: float, ngrid: int = 4096,
                  slope: float = -1.2, sigma_kappa: float = 0.02,
                  sigma_e: float = 0.26, wlo: float = 0.5,
                  whi: float = 1.5) -> Catalogue:
    """Uniform positions on [0, side)^2; shear = nearest-grid-point pixel shear
    of a power-law GRF (``grf_fields``) plus N(0, sigma_e^2) noise per
    component; weights ~ U[wlo, whi).
    Draw order: white noise grid, x, y, noise1, noise2, w."""
    rng = np.random.default_rng(seed)
    _, gamma = grf_fields(rng, ngrid, side, slope, sigma_kappa)
    x = rng.uniform(0.0, side, n)
    y = rng.uniform(0.0, side, n)
    gp = _ngp(gamma, x, y, side)
    del gamma
    g1 = gp.real + rng.normal(0.0, sigma_e, n)
    g2 = gp.imag + rng.normal(0.0, sigma_e, n)
    w = rng.uniform(wlo, whi, n)
    return Catalogue(x, y, np.ascontiguousarray(g1), np.ascontiguousarray(g2), w)


def lognormal_catalogue(seed: int, n: int, side: float, ngrid: int = 4096,
                        sigma_ln: float = 0.5, slope: float = -1.2,
                        sigma_kappa: float = 0.02, sigma_e: float = 0.26,
                        wlo: float = 0.5, whi: float = 1.5) -> Catalogue:
    """Clustered catalogue: density rho = exp(g - sigma_ln^2/2) with g a
    power-law GRF rescaled to sigma_ln; exactly n positions from a multinomial
    over pixels with p ~ rho, uniform inside the pixel; shear from an
    independent GRF (as ``grf_catalogue``) plus noise.
    Draw order: density white noise, shear white noise, multinomial counts,
    in-pixel offsets x, y, noise1, noise2, w."""
    rng = np.random.default_rng(seed)
    g, _ = grf_fields(rng, ngrid, side, slope, sigma_ln)
    rho = np.exp(g - 0.5 * sigma_ln * sigma_ln)
    del g
    _, gamma = grf_fields(rng, ngrid, side, slope, sigma_kappa)
    p = (rho / rho.sum()).ravel()
    counts = rng.multinomial(n, p)
    del p, rho
    pix = np.repeat(np.arange(ngrid * ngrid, dtype=np.int64), counts)
    del counts
    iy = pix // ngrid
    ix = pix - iy * ngrid
    del pix
    d = side / ngrid
    x = (ix + rng.uniform(0.0, 1.0, n)) * d
    y = (iy + rng.uniform(0.0, 1.0, n)) * d
    gp = gamma[iy, ix]
    del gamma
    g1 = gp.real + rng.normal(0.0, sigma_e, n)
    g2 = gp.imag + rng.normal(0.0, sigma_e, n)
    w = rng.uniform(wlo, whi, n)
    return Catalogue(x, y, np.ascontiguousarray(g1), np.ascontiguousarray(g2), w)


def subset(cat: Catalogue, idx: np.ndarray) -> Catalogue:
    idx = np.asarray(idx)
    return Catalogue(*(np.ascontiguousarray(a[idx]) for a in cat.arrays()))


# --------------------------------------------------------------------------
# Named workloads.  Each returns (catalogue, edges, nmax, description).
# --------------------------------------------------------------------------

def workload(name: str, ngrid: int | None = None):
    """The named synthetic workloads used by tests and the benchmark.

    uniform-2k : 60'x60', N=2000 uniform, sigma 0.26, 4 log bins 1-30', nmax 3
    grf-1m     : 600'x600', N=1e6, power-law GRF shear (4096^2 grid) + noise,
                 12 log bins 1-100', nmax 10
    lognormal-10m : 2400'x2400', N=1e7 lognormal positions, 16 log bins
                 0.5-200', nmax 15
    grf-65bin  : 600'x600', N=108000 (0.3 per arcmin^2), GRF shear as grf-1m,
                 65 log bins 0.25-166.29', nmax 15 (the binning of the
                 paper's mock and survey measurements, Sect. 5 and 6)
    """
    if name == "uniform-2k":
        cat = uniform_catalogue(0, 2000, 60.0)
        return cat, log_edges(1.0, 30.0, 4), 3, "60'x60' uniform N=2000, 4 log bins 1-30', nmax=3"
    if name == "grf-1m":
        cat = grf_catalogue(1, 1_000_000, 600.0, ngrid=ngrid or 4096)
        return cat, log_edges(1.0, 100.0, 12), 10, "600'x600' GRF N=1e6, 12 log bins 1-100', nmax=10"
    if name == "lognormal-10m":
        cat = lognormal_catalogue(4, 10_000_000, 2400.0, ngrid=ngrid or 4096)
        return cat, log_edges(0.5, 200.0, 16), 15, "2400'x2400' lognormal N=1e7, 16 log bins 0.5-200', nmax=15"
    if name == "grf-65bin":
        cat = grf_catalogue(5, 108_000, 600.0, ngrid=ngrid or 4096)
        return (cat, log_edges(0.25, 166.29, 65), 15,
                "600'x600' GRF N=108000, 65 log bins 0.25-166.29', nmax=15")
    raise KeyError(name)


def serving_requests(nreq: int = 256, seed0: int = 1000, ngrid: int = 1024,
                     nmin: float = 1e5, nmax_gal: float = 2e6,
                     amin: float = 4.0, amax: float = 100.0,
                     nmax: int = 8, n_scale: float = 1.0):
    """Parameters of the mock-catalogue request stream (catalogues are drawn
    lazily by ``make``).  Request r uses seed seed0 + r:
    N_r = round(exp U[ln nmin, ln nmax_gal]) * n_scale, area exp U[ln amin, ln amax]
    deg^2 (square patch), nbins ~ U{8..16} log bins over 1-100', nmax fixed."""
    out = []
    for r in range(nreq):
        rng = np.random.default_rng(seed0 + r)
        ng = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax_gal)))) * n_scale)
        area = math.exp(rng.uniform(math.log(amin), math.log(amax)))
        nb = int(rng.integers(8, 17))
        side = math.sqrt(area) * 60.0
        out.append(dict(rid=r, seed=seed0 + r, n=max(ng, 4), side=side,
                        nbins=nb, nmax=nmax, ngrid=ngrid))
    return out


def make_request_catalogue(req: dict) -> Catalogue:
    return grf_catalogue(req["seed"], req["n"], req["side"], ngrid=req["ngrid"])
