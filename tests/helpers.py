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
    return np.array([np.abs(a[m] - b[m]).max() / max(np.abs(b[m]).max(), 1e-300)
                     for m in range(a.shape[0])])


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
