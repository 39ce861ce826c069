"""Shared test helpers (no estimator arithmetic here)."""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel_per_mu(a, b):
    """Normwise relative error per correlator: ||a_mu - b_mu||_F / ||b_mu||_F."""
    a = np.asarray(a)
    b = np.asarray(b)
    return np.array([np.linalg.norm(a[m] - b[m]) / max(np.linalg.norm(b[m]), 1e-300)
                     for m in range(a.shape[0])])


def maxabs_per_mu(a, b):
    """Largest element error per correlator over the largest reference
    element: max|a_mu - b_mu| / max|b_mu|."""
    return np.array([np.abs(a[m] - b[m]).max() / max(np.abs(b[m]).max(), 1e-300)
                     for m in range(a.shape[0])])


def elem_per_mu(a, b, floor=1e-3):
    """Element-wise relative error per correlator over the entries that are at
    least `floor` times the correlator's largest entry: max |a - b| / |b|
    there (smaller entries are mostly noise around zero, where a relative
    error says nothing)."""
    out = []
    for m in range(a.shape[0]):
        mag = np.abs(b[m])
        sel = mag >= floor * max(mag.max(), 1e-300)
        out.append((np.abs(a[m] - b[m])[sel] / mag[sel]).max() if sel.any() else 0.0)
    return np.array(out)


def cond_per_mu(a, b, scale):
    """Largest element error per correlator measured in the element's own
    term scale: max |a - b| / S, with S the oracle's sum of absolute term
    values (oracle.abs_bound), broadcast over the multipole axes."""
    return np.array([(np.abs(a[m] - b[m]) / np.maximum(scale[m], 1e-300)).max() for m in range(a.shape[0])])


def equal_bin_mask(nb, nbin=3):
    """Radial-bin tuples with at least two equal bins: where the degenerate
    terms are subtracted (App. A.1; 3 nb^2 - 2 nb of nb^3 triplets for the
    4PCF, the nb diagonal pairs for the 3PCF)."""
    g = np.meshgrid(*[np.arange(nb)] * nbin, indexing="ij")
    m = np.zeros(g[0].shape, dtype=bool)
    for i in range(nbin):
        for j in range(i + 1, nbin):
            m |= g[i] == g[j]
    return m


# Bars per precision.  norm: the spec bar (relative error per
# correlator, read normwise).  cond: derived from the arithmetic (see the
# design notes, section 7): every term x A B C carries a relative perturbation
# of at most ~2^-20 from the binary32 records, ~2^-20 (fp16) or ~2^-16.4 (bf16)
# from the hi/lo operand splits and ~2^-17.2 from the binary32 accumulation
# of 512-centre blocks and 16-block running sums, so each element's error is
# below that times its term scale S: 2^-16 (fp16), 2^-15 (bf16); binary64:
# 1e-10.  max and elem are regression bars, about ten times the largest values
# measured at the 2000-galaxy, 1e6-galaxy and 1e7-galaxy workloads (fp16 1.2e-6
# and 1.1e-4, bf16 1.1e-5 and 5.7e-4, fp64 5e-15 and 5e-13).
BARS = {
    "fp64": {"norm": 1e-10, "max": 1e-10, "elem": 1e-8, "cond": 1e-10},
    "fp16": {"norm": 1e-5, "max": 1e-5, "elem": 1e-3, "cond": 2.0 ** -16},
    "bf16": {"norm": 1e-5, "max": 1e-4, "elem": 5e-3, "cond": 2.0 ** -15},
}


def _scale_for(bound, ncorr, shape_tail):
    """abs_bound's [2, bins...] -> per correlator, broadcast over multipoles."""
    if bound is None:
        return None
    extra = (1,) * len(shape_tail)
    return np.stack([bound[1 if m == ncorr - 1 else 0].reshape(bound.shape[1:] + extra)
                     for m in range(ncorr)])


def parity_metrics(a, b, bound=None, nbin=3, eq=None):
    """Per correlator: normwise, max-element, element-wise (entries >= 1e-3
    max) and, given the oracle's term scale `bound`, scaled element errors, of
    a against the reference b ([ncorr, nb x nbin, multipoles...]); each also
    over the equal-bin tuples alone (prefix eq_).  For a list of bin tuples
    instead ([ncorr, ntuple, multipoles...], `bound` [2, ntuple]) pass `eq`,
    the mask of the tuples with equal bins."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = b.shape[1]
    if eq is None:
        eq = equal_bin_mask(nb, nbin)
    eq = np.asarray(eq, dtype=bool)
    tail = b.shape[1 + eq.ndim:]
    S = _scale_for(bound, b.shape[0], tail)
    ae, be = a[:, eq], b[:, eq]
    out = {"norm": rel_per_mu(a, b), "max": maxabs_per_mu(a, b), "elem": elem_per_mu(a, b),
           "eq_norm": rel_per_mu(ae, be), "eq_max": maxabs_per_mu(ae, be), "eq_elem": elem_per_mu(ae, be)}
    if S is not None:
        S = np.broadcast_to(S, b.shape)
        out["cond"] = cond_per_mu(a, b, S)
        out["eq_cond"] = cond_per_mu(ae, be, S[:, eq])
    return out


def assert_parity(a, b, prec, bound=None, nbin=3, label="", bars=None, eq=None):
    """Every metric of parity_metrics within the bars of `prec` (the
    equal-bin tuples within the same bars as the whole tensor)."""
    bars = dict(BARS[prec], **(bars or {}))
    m = parity_metrics(a, b, bound, nbin, eq)
    print(label, prec, {k: float(v.max()) for k, v in m.items()}, flush=True)
    for key, tol in bars.items():
        for k in (key, "eq_" + key):
            if k in m:
                assert np.all(m[k] < tol), (label, prec, k, m[k])
    return m


def ensure_built():
    from paper_2509_07974_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2509_07974_amd.build import build
        build()
    return _lib.lib()


def header_functions():
    """Function names declared in include/*.h."""
    import re
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(inc, fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", src):
            name = m.group(1)
            prefix = src[max(0, m.start() - 80):m.start()]
            if name in ("if", "sizeof", "defined", "return"):
                continue
            if re.search(r"(fpcf4_status|void|int64_t|const char\s*\*)\s*\*?\s*$", prefix):
                names.append(name)
    return sorted(set(names))
