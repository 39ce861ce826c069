"""The allocation-free entry point (estimate_4pcf_multipoles_noalloc, static
device scratch as workspace) against estimate_4pcf_multipoles, through the C
ABI: the same kernels in the same order on the same inputs, so the results
must agree bit for bit (which is within every parity bar).  Two calls in a
row, the second on a smaller input, show that what one call leaves in the
shared scratch does not leak into the next."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2509_07974_amd as m
    m.lib()
    return m


def _cases():
    big = synth.uniform_catalogue(301, 2000, 60.0)
    small = synth.uniform_catalogue(302, 500, 30.0)
    return ((big, synth.log_edges(1.0, 30.0, 4), 3), (small, synth.log_edges(1.0, 15.0, 3), 2))


@pytest.mark.parametrize("prec", ["fp64", "fp16", "bf16"])
def test_noalloc_equals_allocating_entry_point_twice(fp, prec):
    for cat, edges, nmax in _cases():
        print("noalloc host", prec, cat.n, len(edges) - 1, nmax, flush=True)
        got = fp.estimate_4pcf_multipoles_noalloc(*cat.arrays(), edges, nmax, precision=prec)
        ref = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision=prec)
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), (prec, cat.n)


def test_noalloc_device_inputs_explicit_stream_and_out(fp):
    """Device catalogue, caller-provided device output and an explicit stream
    other than torch's current one (the binding orders that stream after
    the input copies)."""
    import torch
    for cat, edges, nmax in _cases():
        print("noalloc device", cat.n, len(edges) - 1, nmax, flush=True)
        dev = [torch.from_numpy(a).cuda() for a in cat.arrays()]
        s = torch.cuda.Stream()
        out = torch.empty(fp.output_shape(len(edges) - 1, nmax), dtype=torch.complex128, device="cuda")
        got = fp.estimate_4pcf_multipoles_noalloc(*dev, edges, nmax, precision="fp16", stream=s, out=out)
        assert got is out
        ref = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp16")
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref)


def test_noalloc_shrinks_the_tile_to_fit(fp):
    """A catalogue whose single-tile workspace exceeds the scratch: the entry
    point halves the centre tile until it fits; the result equals the
    allocating entry point at that tile."""
    cat = synth.uniform_catalogue(303, 20000, 120.0)
    edges, nmax = synth.log_edges(1.0, 10.0, 4), 3
    full, _ = fp.plan(cat.n, edges, nmax, "fp64")
    assert full > fp.NOALLOC_SCRATCH_BYTES
    tile = cat.n
    while True:
        tile //= 2
        b, _ = fp.plan(cat.n, edges, nmax, "fp64", tile_centers=tile)
        if b <= fp.NOALLOC_SCRATCH_BYTES:
            break
    print("noalloc tile", tile, flush=True)
    got = fp.estimate_4pcf_multipoles_noalloc(*cat.arrays(), edges, nmax, precision="fp64")
    ref = fp.estimate_4pcf_multipoles(*cat.arrays(), edges, nmax, precision="fp64", tile_centers=tile)
    assert np.array_equal(got, ref)
