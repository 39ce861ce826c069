"""MI355X-native multipole estimator of the shear four-point correlation
function (Porth et al. 2025, arXiv:2509.07974, Sect. 3).

Thin Python binding over libfpcf4.so (include/fpcf4.h).  Every step of the
estimator runs in the library's HIP kernels; this module only marshals
arguments.  Inputs may be NumPy arrays (host) or CUDA/HIP torch tensors
(device); PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (FP64, MIXED_FP16, MIXED_BF16, MEM_HOST, MEM_DEVICE, NMAX_SUPPORTED, NOALLOC_SCRATCH_BYTES,
                   NBINS_SUPPORTED, Fpcf4Error, check, lib)

__all__ = ["estimate_4pcf_multipoles", "estimate_4pcf_multipoles_noalloc", "estimate_3pcf_multipoles",
           "debug_multipoles", "debug_pair_plan", "debug_corr_plan", "debug_sort_pairs", "to_natural",
           "to_natural_triplets", "natural_blocks", "plan", "Request",
           "profile_enable", "profile_read",
           "PRECISIONS", "Fpcf4Error", "output_shape", "output3_shape", "lib", "version",
           "NOALLOC_SCRATCH_BYTES"]

PRECISIONS = {"fp64": FP64, "fp16": MIXED_FP16, "bf16": MIXED_BF16}


def version() -> str:
    return lib().fpcf4_version().decode()


def output_shape(nbins: int, nmax: int):
    nn = 2 * nmax + 1
    return (9, nbins, nbins, nbins, nn, nn)


def output3_shape(nbins: int, nmax: int):
    return (5, nbins, nbins, 2 * nmax + 1)


def _stream_handle(stream):
    """Raw hipStream_t of `stream` (a torch stream object or an integer handle)."""
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream))


def _order_after_current(stream, device):
    """Make the caller's stream wait for the work torch has queued on its
    current stream (the input copies and the output allocation), so that the
    library, which runs on `stream`, never reads inputs before they are
    written or writes memory torch's allocator handed out on another stream."""
    import torch
    cur = torch.cuda.current_stream(device)
    if stream is None or stream == cur.cuda_stream:
        return
    torch.cuda.ExternalStream(stream, device=device).wait_stream(cur)


def _check_out(out, shape, device, torch_device=None):
    """Reject an `out` buffer the library could not write safely: wrong
    shape, dtype, layout or memory space (the library writes
    prod(shape) complex128 values through a raw pointer)."""
    shape = tuple(int(d) for d in shape)
    if device:
        import torch
        if not isinstance(out, torch.Tensor) or not out.is_cuda or out.device != torch_device:
            raise ValueError(f"out must be a torch tensor on {torch_device}")
        if out.dtype != torch.complex128:
            raise ValueError(f"out must be complex128, not {out.dtype}")
        if tuple(out.shape) != shape:
            raise ValueError(f"out has shape {tuple(out.shape)}, expected {shape}")
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
        return out
    if not isinstance(out, np.ndarray):
        raise ValueError("out must be a NumPy array for host inputs")
    if out.dtype != np.complex128:
        raise ValueError(f"out must be complex128, not {out.dtype}")
    if out.shape != shape:
        raise ValueError(f"out has shape {out.shape}, expected {shape}")
    if not out.flags.c_contiguous or not out.flags.writeable:
        raise ValueError("out must be C-contiguous and writeable")
    return out


def _is_torch_device(a) -> bool:
    try:
        import torch
    except ImportError:  # pragma: no cover
        return False
    return isinstance(a, torch.Tensor) and a.is_cuda


class _Marshal:
    """Keeps the arrays behind the raw pointers alive for the call."""

    def __init__(self, x, y, g1, g2, w, edges, nmax, precision, subtract_degenerate,
                 centers, tile_centers, stream):
        arrs = (x, y, g1, g2, w)
        self.device = all(_is_torch_device(a) for a in arrs)
        self.keep = []
        if self.device:
            import torch
            dev = [a.detach().to(torch.float64).contiguous() for a in arrs]
            n = dev[0].numel()
            if any(a.numel() != n for a in dev):
                raise ValueError("catalogue arrays differ in length")
            self.keep += dev
            ptrs = [a.data_ptr() for a in dev]
            mem = MEM_DEVICE
            stream = _stream_handle(stream)
            if stream is None:
                stream = torch.cuda.current_stream(dev[0].device).cuda_stream
            self.torch_device = dev[0].device
        else:
            stream = _stream_handle(stream)
            host = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in arrs]
            n = host[0].size
            if any(a.size != n for a in host):
                raise ValueError("catalogue arrays differ in length")
            self.keep += host
            ptrs = [a.ctypes.data for a in host]
            mem = MEM_HOST
        self.n = n
        self.cat = _lib.Catalogue(n, *ptrs, mem)
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        self.keep.append(e)
        self.nbins = e.size - 1
        self.bins = _lib.Bins(self.nbins, e.ctypes.data)
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        cptr, nc = None, 0
        if centers is not None:
            if self.device:
                import torch
                ct = torch.as_tensor(centers, dtype=torch.int64, device=self.torch_device).contiguous()
                self.keep.append(ct)
                cptr, nc = ct.data_ptr(), ct.numel()
            else:
                ca = np.ascontiguousarray(np.asarray(centers, dtype=np.int64))
                self.keep.append(ca)
                cptr, nc = ca.ctypes.data, ca.size
        self.ncent = nc if centers is not None else n
        self.nmax = int(nmax)
        self.stream = stream
        self.opts = _lib.Options(self.nmax, prec, 1 if subtract_degenerate else 0, 0, cptr, nc,
                                 int(tile_centers), stream)

    def refs(self):
        return C.byref(self.cat), C.byref(self.bins), C.byref(self.opts)

    def output(self, shape, out):
        """The output buffer (validated `out`, or a new one), after ordering
        the library's stream behind torch's current stream."""
        if self.device:
            import torch
            res = (_check_out(out, shape, True, self.torch_device) if out is not None
                   else torch.empty(shape, dtype=torch.complex128, device=self.torch_device))
            _order_after_current(self.stream, self.torch_device)
            return res, res.data_ptr(), MEM_DEVICE
        res = _check_out(out, shape, False) if out is not None else np.empty(shape, dtype=np.complex128)
        return res, res.ctypes.data, MEM_HOST


def estimate_4pcf_multipoles(x, y, g1, g2, w, edges, nmax: int, precision="fp64",
                             subtract_degenerate: bool = True, centers=None,
                             tile_centers: int = 0, stream=None, out=None, tree=None):
    """Upsilon_{mu,(n2,n3)}(T1,T2,T3), mu = 0..7, and N (index 8) as a
    complex128 array [9, nb, nb, nb, 2nmax+1, 2nmax+1] (NumPy for host inputs,
    a torch tensor on the inputs' device for device inputs).
    tree = (delta1, nlevels, rmin) selects the tree approximation (reduced
    catalogues on grids delta1 * 2^(d-1); mixed precisions only).
    out: optional preallocated result (same type, shape, complex128,
    contiguous, on the inputs' device); stream: a torch stream or a raw
    hipStream_t (default: torch's current stream)."""
    m = _Marshal(x, y, g1, g2, w, edges, nmax, precision, subtract_degenerate, centers,
                 tile_centers, stream)
    res, ptr, mem = m.output(output_shape(m.nbins, m.nmax), out)
    if tree is not None:
        delta1, nlevels, rmin = tree
        t = _lib.Tree(int(nlevels), 0, float(delta1), float(rmin))
        check(lib().estimate_4pcf_multipoles_tree(*m.refs(), C.byref(t), C.c_void_p(ptr), mem))
    else:
        check(lib().estimate_4pcf_multipoles(*m.refs(), C.c_void_p(ptr), mem))
    return res


def estimate_4pcf_multipoles_noalloc(x, y, g1, g2, w, edges, nmax: int, precision="fp64",
                                     subtract_degenerate: bool = True, centers=None,
                                     tile_centers: int = 0, stream=None, out=None):
    """estimate_4pcf_multipoles with the library's static device scratch
    (NOALLOC_SCRATCH_BYTES) as workspace: the library allocates no device
    memory.  Workloads whose workspace does not fit raise Fpcf4Error
    (E_BUDGET).  Pass `out` to keep the call free of allocations on the
    Python side as well."""
    m = _Marshal(x, y, g1, g2, w, edges, nmax, precision, subtract_degenerate, centers,
                 tile_centers, stream)
    res, ptr, mem = m.output(output_shape(m.nbins, m.nmax), out)
    check(lib().estimate_4pcf_multipoles_noalloc(*m.refs(), C.c_void_p(ptr), mem))
    return res


def estimate_3pcf_multipoles(x, y, g1, g2, w, edges, nmax: int, precision="fp64",
                             subtract_degenerate: bool = True, centers=None,
                             tile_centers: int = 0, stream=None, out=None, base=None, tree=None):
    """Shear 3PCF multipoles Upsilon_{mu,n}(T1,T2), mu = 0..3, and N (index 4)
    as a complex128 array [5, nb, nb, 2nmax+1] (NumPy for host inputs, a
    torch tensor on the inputs' device for device inputs).  nmax <= 32.
    base = (delta1, nlevels, rmin) selects the BaseTree approximation of the
    base points (grids delta1 * 2^(d-1); every galaxy a base point),
    tree = (delta1, nlevels, rmin) the tree approximation of the neighbours;
    both together are the DoubleTree (mixed precisions only)."""
    m = _Marshal(x, y, g1, g2, w, edges, nmax, precision, subtract_degenerate, centers,
                 tile_centers, stream)
    res, ptr, mem = m.output(output3_shape(m.nbins, m.nmax), out)
    if base is not None or tree is not None:
        def tr(t):
            return None if t is None else C.byref(_lib.Tree(int(t[1]), 0, float(t[0]), float(t[2])))
        check(lib().estimate_3pcf_multipoles_doubletree(*m.refs(), tr(base), tr(tree), C.c_void_p(ptr), mem))
    else:
        check(lib().estimate_3pcf_multipoles(*m.refs(), C.c_void_p(ptr), mem))
    return res


def debug_multipoles(x, y, g1, g2, w, edges, nmax: int, precision="fp64", centers=None,
                     tile_centers: int = 0, stream=None):
    """Stage (a) only: (counts int64 [nc, nb], G complex128 [nc, nb, 4nmax+3]
    for k = -2nmax-3..2nmax-1, W complex128 [nc, nb, 4nmax+1] for
    k = -2nmax..2nmax), for the centres in the given order."""
    m = _Marshal(x, y, g1, g2, w, edges, nmax, precision, True, centers, tile_centers, stream)
    nc, nb, n = m.ncent, m.nbins, m.nmax
    counts = np.zeros((nc, nb), dtype=np.int64)
    G = np.zeros((nc, nb, 4 * n + 3), dtype=np.complex128)
    W = np.zeros((nc, nb, 4 * n + 1), dtype=np.complex128)
    check(lib().fpcf4_debug_multipoles(*m.refs(), C.c_void_p(counts.ctypes.data),
                                       C.c_void_p(G.ctypes.data), C.c_void_p(W.ctypes.data)))
    return counts, G, W


def to_natural(upsilon, nphi: int, stream=None):
    """(Gamma complex128 [8, nb, nb, nb, nphi, nphi], Nbar float64
    [nb, nb, nb, nphi, nphi]) from the multipoles (host array)."""
    u = np.ascontiguousarray(np.asarray(upsilon, dtype=np.complex128))
    nb = u.shape[1]
    nmax = (u.shape[-1] - 1) // 2
    gam = np.empty((8, nb, nb, nb, nphi, nphi), dtype=np.complex128)
    nrm = np.empty((nb, nb, nb, nphi, nphi), dtype=np.float64)
    check(lib().fpcf4_to_natural(C.c_void_p(u.ctypes.data), nb, nmax, int(nphi),
                                 C.c_void_p(gam.ctypes.data), C.c_void_p(nrm.ctypes.data),
                                 _stream_handle(stream)))
    return gam, nrm


def to_natural_triplets(upsilon, nphi: int, triplets, stream=None):
    """Natural components for the listed radial-bin triplets only:
    (Gamma complex128 [8, ntrip, nphi, nphi], Nbar float64 [ntrip, nphi, nphi]).
    upsilon is the multipole tensor (NumPy, or a torch tensor on the GPU, in
    which case the results are torch tensors on the same device)."""
    t = np.ascontiguousarray(np.asarray(triplets, dtype=np.int32).reshape(-1, 3))
    ntrip = t.shape[0]
    if _is_torch_device(upsilon):
        import torch
        u = upsilon.contiguous()
        nb, nmax = u.shape[1], (u.shape[-1] - 1) // 2
        gam = torch.empty((8, ntrip, nphi, nphi), dtype=torch.complex128, device=u.device)
        nrm = torch.empty((ntrip, nphi, nphi), dtype=torch.float64, device=u.device)
        stream = _stream_handle(stream)
        if stream is None:
            stream = torch.cuda.current_stream(u.device).cuda_stream
        _order_after_current(stream, u.device)
        check(lib().fpcf4_to_natural_triplets(C.c_void_p(u.data_ptr()), MEM_DEVICE, nb, nmax, int(nphi),
                                              C.c_void_p(t.ctypes.data), ntrip, C.c_void_p(gam.data_ptr()),
                                              C.c_void_p(nrm.data_ptr()), MEM_DEVICE, stream))
        return gam, nrm
    u = np.ascontiguousarray(np.asarray(upsilon, dtype=np.complex128))
    nb, nmax = u.shape[1], (u.shape[-1] - 1) // 2
    gam = np.empty((8, ntrip, nphi, nphi), dtype=np.complex128)
    nrm = np.empty((ntrip, nphi, nphi), dtype=np.float64)
    check(lib().fpcf4_to_natural_triplets(C.c_void_p(u.ctypes.data), MEM_HOST, nb, nmax, int(nphi),
                                          C.c_void_p(t.ctypes.data), ntrip, C.c_void_p(gam.ctypes.data),
                                          C.c_void_p(nrm.ctypes.data), MEM_HOST, _stream_handle(stream)))
    return gam, nrm


def natural_blocks(upsilon, nphi: int, block: int = 4096, stream=None):
    """Yield (triplets [k, 3], Gamma [8, k, nphi, nphi], Nbar [k, nphi, nphi])
    over all radial-bin triplets in blocks of at most `block`, so that the
    natural components of a large tensor can be consumed on the fly."""
    nb = upsilon.shape[1]
    allt = np.stack(np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb), indexing="ij"), -1).reshape(-1, 3)
    for s in range(0, allt.shape[0], block):
        t = allt[s:s + block]
        gam, nrm = to_natural_triplets(upsilon, nphi, t, stream)
        yield t, gam, nrm


def debug_pair_plan(nmax: int):
    """The stage (b) contraction plan (host only): an int32 array
    [9, 2nmax+1, 2nmax+1, 16] as fpcf4_debug_pair_plan documents it, and the
    number of work items."""
    out = np.zeros((9, 2 * nmax + 1, 2 * nmax + 1, 16), dtype=np.int32)
    nit = C.c_int64(0)
    check(lib().fpcf4_debug_pair_plan(int(nmax), out.ctypes.data, C.byref(nit)))
    return out, int(nit.value)


def debug_corr_plan(nmax: int):
    """The distinct degenerate-term sums (host only): an int32 array
    [9, 8 nmax + 4, 8] as fpcf4_debug_corr_plan documents it, and the number
    of distinct sums."""
    out = np.zeros((9, 8 * nmax + 4, 8), dtype=np.int32)
    ns = C.c_int64(0)
    check(lib().fpcf4_debug_corr_plan(int(nmax), out.ctypes.data, C.byref(ns)))
    return out, int(ns.value)


def debug_sort_pairs(keys, vals, key_bits: int, key_bytes: int = 8):
    """The cell-list build's stable radix sort on the device (host arrays in
    and out): keys (uint64, each below 2^key_bits) and int32 vals sorted by
    key, equal keys in input order; key_bytes 4 runs the 32-bit-key sort."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    v = np.ascontiguousarray(vals, dtype=np.int32)
    if k.ndim != 1 or v.shape != k.shape:
        raise ValueError("keys and vals must be 1-D arrays of one length")
    ko = np.empty_like(k)
    vo = np.empty_like(v)
    check(lib().fpcf4_debug_sort_pairs(k.ctypes.data, v.ctypes.data, k.size, int(key_bits), int(key_bytes),
                                       ko.ctypes.data, vo.ctypes.data))
    return ko, vo


def profile_enable(on: bool = True):
    """Enable per-stage hipEvent timing in the library (resets the totals)."""
    check(lib().fpcf4_profile_enable(1 if on else 0))


def profile_read() -> dict:
    p = _lib.Profile()
    check(lib().fpcf4_profile_read(C.byref(p)))
    return {k: getattr(p, k) for k, _ in _lib.Profile._fields_}


def plan(n: int, edges, nmax: int, precision="fp64", ncenters=None, tile_centers: int = 0):
    """(device_bytes, ntiles) a request with these sizes needs."""
    z = np.zeros(1)
    m = _Marshal(z, z, z, z, z, edges, nmax, precision, True, None, tile_centers, None)
    m.cat.n = int(n)
    m.cat.mem = MEM_HOST
    if ncenters is not None:
        m.opts.ncenters = int(ncenters)
        m.opts.centers = C.c_void_p(8)   # only the count is read by the planner
    nbytes = C.c_size_t(0)
    ntiles = C.c_int64(0)
    check(lib().fpcf4_plan(*m.refs(), C.byref(nbytes), C.byref(ntiles)))
    return int(nbytes.value), int(ntiles.value)


class Request:
    """One estimate advanced tile by tile on its own stream, in a caller-owned
    device workspace (torch uint8 tensor): the serving building block."""

    def __init__(self, x, y, g1, g2, w, edges, nmax, precision="fp16", subtract_degenerate=True,
                 centers=None, tile_centers: int = 0, stream=None, workspace=None):
        import torch
        self.m = _Marshal(x, y, g1, g2, w, edges, nmax, precision, subtract_degenerate, centers,
                          tile_centers, stream)
        nbytes = C.c_size_t(0)
        ntiles = C.c_int64(0)
        check(lib().fpcf4_plan(*self.m.refs(), C.byref(nbytes), C.byref(ntiles)))
        self.bytes = int(nbytes.value)
        self.ntiles = int(ntiles.value)
        if workspace is None:
            workspace = torch.empty(self.bytes, dtype=torch.uint8, device="cuda")
        if workspace.numel() < self.bytes:
            raise Fpcf4Error(_lib.E_BUDGET, "workspace too small")
        self.workspace = workspace
        s = self.m.stream
        if s is not None and s != torch.cuda.current_stream(workspace.device).cuda_stream:
            # the request's kernels run on its own stream: order them after
            # the inputs and the workspace, and keep torch's allocator from
            # reusing those blocks while that stream may still use them
            ext = torch.cuda.ExternalStream(s, device=workspace.device)
            ext.wait_stream(torch.cuda.current_stream(workspace.device))
            workspace.record_stream(ext)
            for a in self.m.keep:
                if isinstance(a, torch.Tensor) and a.is_cuda:
                    a.record_stream(ext)
        self.handle = C.c_void_p()
        check(lib().fpcf4_request_create(*self.m.refs(), C.c_void_p(workspace.data_ptr()),
                                         self.bytes, C.byref(self.handle)))
        self.next_tile = 0

    def step(self, tile=None):
        t = self.next_tile if tile is None else tile
        check(lib().fpcf4_request_step(self.handle, t))
        self.next_tile = t + 1
        return self.next_tile < self.ntiles

    def finalize(self):
        shape = output_shape(self.m.nbins, self.m.nmax)
        res = np.empty(shape, dtype=np.complex128)
        check(lib().fpcf4_request_finalize(self.handle, C.c_void_p(res.ctypes.data), MEM_HOST))
        return res

    def close(self):
        if self.handle:
            lib().fpcf4_request_destroy(self.handle)
            self.handle = C.c_void_p()
        self.workspace = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
