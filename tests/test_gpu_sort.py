"""The cell-list build's stable radix sort on the GPU, bit for bit against
NumPy's stable argsort (the definition of a stable sort by key).

The sort orders the catalogue by search cell (32-bit keys), the centres by
the Morton key of their cell (32-bit) and the galaxies by reduced-catalogue
cell (64-bit); equal keys must keep their catalogue order, so that every
cell's neighbours, and the galaxies summed into one pseudo-galaxy, come in
the same order on every run.  Sizes span one tile (4096), its ragged
neighbours, and enough tiles that the scan of the per-tile digit counts
itself spans several tiles.
"""
import numpy as np
import pytest

from helpers import ensure_built

pytestmark = pytest.mark.gpu


def _check(keys, bits, kbytes):
    import paper_2509_07974_amd as fp
    vals = np.arange(keys.size, dtype=np.int32)
    print(f"sort n={keys.size} bits={bits} key_bytes={kbytes}", flush=True)
    ko, vo = fp.debug_sort_pairs(keys, vals, bits, kbytes)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(vo, order.astype(np.int32))
    assert np.array_equal(ko, keys[order])


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 100_003])
@pytest.mark.parametrize("bits", [1, 7, 17, 32])
def test_sort_32bit_keys(n, bits):
    rng = np.random.default_rng(1000 * n + bits)
    keys = rng.integers(0, 2 ** bits, n, dtype=np.uint64)
    _check(keys, bits, 4)


@pytest.mark.parametrize("bits", [21, 33, 64])
def test_sort_64bit_keys(bits):
    rng = np.random.default_rng(bits)
    n = 70_001
    keys = rng.integers(0, 2 ** 63, n, dtype=np.uint64)
    if bits < 64:
        keys >>= np.uint64(63 - bits)
    else:
        keys |= rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(63)
    _check(keys, bits, 8)


def test_sort_many_tiles_and_heavy_duplicates():
    """1.5e6 keys (367 tiles: 5872 digit counts, two scan tiles), few
    distinct values so that stability decides almost every position."""
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 37, 1_500_000, dtype=np.uint64)
    _check(keys, 6, 4)


def test_sort_cell_keys_of_a_catalogue():
    """Keys shaped like the cell keys of a clustered catalogue: runs of equal
    keys and empty cells, already partly sorted."""
    rng = np.random.default_rng(11)
    ncx = 288
    cx = np.clip(rng.normal(140, 40, 300_000), 0, ncx - 1).astype(np.uint64)
    cy = np.clip(rng.normal(120, 30, 300_000), 0, ncx - 1).astype(np.uint64)
    keys = cy * np.uint64(ncx) + cx
    keys[:50_000].sort()
    _check(keys, 17, 4)
