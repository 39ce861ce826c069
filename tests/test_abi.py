"""C-ABI library: loads, exports every declared symbol, rejects invalid
arguments before touching a device (runs without a GPU)."""
import ctypes as C

import numpy as np
import pytest

from helpers import ensure_built, header_functions


def test_header_declares_expected_api():
    names = header_functions()
    for n in ["estimate_4pcf_multipoles", "fpcf4_debug_multipoles", "fpcf4_to_natural",
              "fpcf4_plan", "fpcf4_request_create", "fpcf4_request_step",
              "fpcf4_request_finalize", "fpcf4_request_destroy", "fpcf4_last_error"]:
        assert n in names


def test_library_exports_all_header_symbols():
    lib = ensure_built()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_version_and_output_elems():
    lib = ensure_built()
    assert b"gfx950" in lib.fpcf4_version()
    assert lib.fpcf4_output_elems(4, 3) == 9 * 64 * 49
    assert lib.fpcf4_output_elems(12, 10) == 9 * 1728 * 441


def _call(edges, nmax=2, n=10, precision=0, xs=None):
    from paper_2509_07974_amd import _lib
    ensure_built()
    rng = np.random.default_rng(0)
    arrs = [rng.uniform(0, 10, n) for _ in range(5)] if xs is None else xs
    cat = _lib.Catalogue(n, *[a.ctypes.data for a in arrs], _lib.MEM_HOST)
    e = np.asarray(edges, dtype=np.float64)
    bins = _lib.Bins(e.size - 1, e.ctypes.data)
    opts = _lib.Options(nmax, precision, 1, 0, None, 0, 0, None)
    out = np.zeros(max(1, 9 * (e.size - 1) ** 3 * (2 * max(nmax, 0) + 1) ** 2), complex)
    st = _lib.lib().estimate_4pcf_multipoles(C.byref(cat), C.byref(bins), C.byref(opts),
                                             C.c_void_p(out.ctypes.data), _lib.MEM_HOST)
    return st, _lib.lib().fpcf4_last_error().decode()


@pytest.mark.parametrize("edges,nmax,code", [
    ([1.0, 0.5, 2.0], 2, -1),          # not increasing
    ([0.0, 1.0, 2.0], 2, -1),          # edges[0] <= 0
    ([-1.0, 1.0], 2, -1),
    ([1.0, np.nan, 3.0], 2, -1),       # non-finite edge
    ([1.0, 2.0], -1, -1),              # nmax < 0
    ([1.0, 2.0], 17, -2),              # beyond compiled nmax
    (list(np.geomspace(1, 10, 130)), 2, -2),  # 129 bins > 128
    ([1.0], 2, -1),                    # no bin
])
def test_invalid_arguments_rejected(edges, nmax, code):
    st, msg = _call(edges, nmax)
    assert st == code and msg


def test_bad_precision_and_null_output():
    from paper_2509_07974_amd import _lib
    st, _ = _call([1.0, 2.0], 2, precision=7)
    assert st == _lib.E_INVALID_ARG
    lib = ensure_built()
    st = lib.estimate_4pcf_multipoles(None, None, None, None, 0)
    assert st == _lib.E_INVALID_ARG


def test_python_binding_rejects_mismatched_lengths():
    import paper_2509_07974_amd as m
    ensure_built()
    with pytest.raises(ValueError):
        m.estimate_4pcf_multipoles(np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3), np.zeros(3),
                                   [1.0, 2.0], 1)


def _call3(edges, nmax=2, n=10, precision=0):
    from paper_2509_07974_amd import _lib
    ensure_built()
    rng = np.random.default_rng(0)
    arrs = [rng.uniform(0, 10, n) for _ in range(5)]
    cat = _lib.Catalogue(n, *[a.ctypes.data for a in arrs], _lib.MEM_HOST)
    e = np.asarray(edges, dtype=np.float64)
    bins = _lib.Bins(e.size - 1, e.ctypes.data)
    opts = _lib.Options(nmax, precision, 1, 0, None, 0, 0, None)
    out = np.zeros(max(1, 5 * (e.size - 1) ** 2 * (2 * max(nmax, 0) + 1)), complex)
    st = _lib.lib().estimate_3pcf_multipoles(C.byref(cat), C.byref(bins), C.byref(opts),
                                             C.c_void_p(out.ctypes.data), _lib.MEM_HOST)
    return st, _lib.lib().fpcf4_last_error().decode()


@pytest.mark.parametrize("edges,nmax,code", [
    ([1.0, 0.5, 2.0], 4, -1),          # not increasing
    ([0.0, 1.0, 2.0], 4, -1),          # edges[0] <= 0
    ([1.0, 2.0], -1, -1),              # nmax < 0
    ([1.0, 2.0], 33, -2),              # beyond the compiled 3PCF multipoles
    (list(np.geomspace(1, 10, 130)), 2, -2),  # 129 bins > 128
])
def test_3pcf_invalid_arguments_rejected(edges, nmax, code):
    st, msg = _call3(edges, nmax)
    assert st == code and msg


def test_3pcf_output_elems_and_null_output():
    from paper_2509_07974_amd import _lib
    lib = ensure_built()
    assert lib.fpcf4_output3_elems(12, 10) == 5 * 144 * 21
    assert lib.fpcf4_output3_elems(-1, 2) == 0
    assert lib.estimate_3pcf_multipoles(None, None, None, None, 0) == _lib.E_INVALID_ARG


@pytest.mark.parametrize("nphi,trip,code", [
    (8, [[0, 0, 3]], -1),      # bin index out of range
    (8, [[-1, 0, 0]], -1),
    (0, [[0, 0, 0]], -1),      # no angular bin
])
def test_natural_triplets_invalid_arguments(nphi, trip, code):
    from paper_2509_07974_amd import _lib
    lib = ensure_built()
    nb, nmax = 3, 1
    ups = np.zeros(9 * nb ** 3 * 9, complex)
    t = np.asarray(trip, dtype=np.int32)
    gam = np.zeros(8 * len(trip) * max(nphi, 1) ** 2, complex)
    st = lib.fpcf4_to_natural_triplets(C.c_void_p(ups.ctypes.data), _lib.MEM_HOST, nb, nmax, nphi,
                                       C.c_void_p(t.ctypes.data), len(trip), C.c_void_p(gam.ctypes.data),
                                       None, _lib.MEM_HOST, None)
    assert st == code
    assert lib.fpcf4_to_natural_triplets(None, 0, nb, nmax, 8, None, 0, None, None, 0, None) == -1


@pytest.mark.parametrize("prec,tree,code", [
    (1, (0.5, 0, 10.0), -1),     # no level
    (1, (0.5, 5, 10.0), -1),     # more levels than supported
    (1, (0.0, 2, 10.0), -1),     # zero cell side
    (1, (0.5, 2, 1.5), -1),      # r_min below 2
    (0, (0.5, 2, 10.0), -2),     # FP64 path
])
def test_tree_invalid_arguments_rejected(prec, tree, code):
    from paper_2509_07974_amd import _lib
    lib = ensure_built()
    rng = np.random.default_rng(0)
    n = 10
    arrs = [rng.uniform(0, 10, n) for _ in range(5)]
    cat = _lib.Catalogue(n, *[a.ctypes.data for a in arrs], _lib.MEM_HOST)
    e = np.array([1.0, 2.0, 4.0])
    bins = _lib.Bins(2, e.ctypes.data)
    opts = _lib.Options(1, prec, 1, 0, None, 0, 0, None)
    t = _lib.Tree(tree[1], 0, tree[0], tree[2])
    out = np.zeros(9 * 8 * 9, complex)
    st = lib.estimate_4pcf_multipoles_tree(C.byref(cat), C.byref(bins), C.byref(opts), C.byref(t),
                                           C.c_void_p(out.ctypes.data), _lib.MEM_HOST)
    assert st == code, lib.fpcf4_last_error()


def test_noalloc_rejects_oversized_workspace_before_device_work():
    """The allocation-free entry point checks the planned workspace against
    its static scratch on the host: a catalogue of 2e6 galaxies needs more
    than 64 MiB at any centre tile (galaxy records and cell list alone), so
    the call fails with E_BUDGET before any device work (no GPU here)."""
    from paper_2509_07974_amd import _lib
    lib = ensure_built()
    z = np.zeros(1)
    e = np.array([1.0, 2.0, 4.0])
    cat = _lib.Catalogue(2_000_000, *[z.ctypes.data] * 5, _lib.MEM_HOST)
    bins = _lib.Bins(2, e.ctypes.data)
    opts = _lib.Options(2, _lib.MIXED_FP16, 1, 0, None, 0, 0, None)
    out = np.zeros(9 * 8 * 25, complex)
    st = lib.estimate_4pcf_multipoles_noalloc(C.byref(cat), C.byref(bins), C.byref(opts),
                                              C.c_void_p(out.ctypes.data), _lib.MEM_HOST)
    assert st == _lib.E_BUDGET
    assert "static scratch" in lib.fpcf4_last_error().decode()
    st = lib.estimate_4pcf_multipoles_noalloc(C.byref(cat), C.byref(bins), C.byref(opts), None, _lib.MEM_HOST)
    assert st == _lib.E_INVALID_ARG


@pytest.mark.parametrize("bad", ["shape", "dtype", "layout", "readonly", "torch"])
def test_out_buffer_is_validated(bad):
    """A caller-supplied `out` must match the result exactly (shape,
    complex128, C-contiguous, writeable, host for host inputs): the library
    writes through a raw pointer, so anything else is rejected before the
    call."""
    import paper_2509_07974_amd as m
    ensure_built()
    x = np.zeros(3)
    edges = [1.0, 2.0, 4.0]
    shape = m.output_shape(2, 1)
    if bad == "shape":
        out = np.zeros((9, 2, 2, 2, 3, 2), complex)
    elif bad == "dtype":
        out = np.zeros(shape, np.complex64)
    elif bad == "layout":
        out = np.zeros(shape[::-1], complex).T
    elif bad == "readonly":
        out = np.zeros(shape, complex)
        out.flags.writeable = False
    else:
        import torch
        out = torch.zeros(shape, dtype=torch.complex128)
    for f in (m.estimate_4pcf_multipoles, m.estimate_4pcf_multipoles_noalloc):
        with pytest.raises(ValueError):
            f(x, x, x, x, x, edges, 1, out=out)
    with pytest.raises(ValueError):
        m.estimate_3pcf_multipoles(x, x, x, x, x, edges, 1, out=np.zeros((5, 2, 2, 4), complex))


@pytest.mark.gpu
def test_valid_host_out_is_filled_in_place():
    import paper_2509_07974_amd as m
    ensure_built()
    x = np.array([0.0, 100.0, 200.0])   # no pair in range: the result is zero
    out = np.full(m.output_shape(2, 1), 7 + 7j)
    got = m.estimate_4pcf_multipoles(x, x, x, x, x + 1, [1.0, 2.0, 4.0], 1, out=out)
    assert got is out and not np.any(out)


def test_basetree_rejects_centre_subsets_and_fp64():
    import paper_2509_07974_amd as fp
    x = np.arange(10.0)
    for kw, code in (({"centers": [1, 2]}, -1), ({"precision": "fp64"}, -2)):
        kw.setdefault("precision", "fp16")
        with pytest.raises(fp.Fpcf4Error) as ei:
            fp.estimate_3pcf_multipoles(x, x, x * 0, x * 0, x * 0 + 1, [1.0, 2.0, 4.0], 2,
                                        base=(0.5, 2, 4.0), **kw)
        assert ei.value.status == code
    with pytest.raises(fp.Fpcf4Error) as ei:
        fp.estimate_3pcf_multipoles(x, x, x * 0, x * 0, x * 0 + 1, [1.0, 2.0, 4.0], 2,
                                    precision="fp16", base=(0.5, 9, 4.0))
    assert ei.value.status == -1


def test_debug_sort_rejects_bad_arguments():
    """The sort check export validates on the host before any device work."""
    from paper_2509_07974_amd import _lib
    lib = ensure_built()
    k = np.array([1, 2, 40], dtype=np.uint64)
    v = np.zeros(3, np.int32)
    ko = np.zeros(3, np.uint64)
    vo = np.zeros(3, np.int32)

    def call(n, bits, kbytes, keys=k.ctypes.data, outk=ko.ctypes.data):
        return lib.fpcf4_debug_sort_pairs(keys, v.ctypes.data, n, bits, kbytes, outk, vo.ctypes.data)

    assert call(3, 5, 8) == _lib.E_INVALID_ARG      # 40 is not below 2^5
    assert call(3, 33, 4) == _lib.E_INVALID_ARG     # 32-bit keys take at most 32 bits
    assert call(3, 0, 8) == _lib.E_INVALID_ARG
    assert call(3, 65, 8) == _lib.E_INVALID_ARG
    assert call(3, 6, 2) == _lib.E_INVALID_ARG
    assert call(-1, 6, 8) == _lib.E_INVALID_ARG
    assert call(3, 6, 8, keys=None) == _lib.E_INVALID_ARG
    assert call(3, 6, 8, outk=None) == _lib.E_INVALID_ARG
    assert call(0, 6, 8) == _lib.OK                 # nothing to sort: no device work
