"""Thin Python binding of libfmm.so (ctypes): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; torch is
used for device memory and streams. There is no CPU fallback: if the shared
library is missing, loading it raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EHIP, FMM_EUNSUPPORTED = 0, -1, -2, -3, -4
FMM_FP64, FMM_SPLIT_FP32, FMM_FP64_HARMONIC, FMM_EXACT_SLICE = 0, 1, 2, 3
FMM_OPT_M2L_KERNEL, FMM_OPT_USE_GRAPH, FMM_OPT_TILE_CONFIG, FMM_OPT_ADJOINT_FORM = 1, 2, 3, 4
FMM_OPT_P2M_WINDOW = 5
FMM_OPT_ROUND_SPLIT = 6
FMM_OPT_SLICES = 7

FRAME, NCELL, NTARGET, NSTENCIL = 24, 24 ** 3, 512, 892
NOALLOC_MAX_SUBGRIDS = 16384
FULL_MASK = (1 << 27) - 1

EXPORTS = [
    "fmm_create", "fmm_destroy", "fmm_status_string", "fmm_last_error", "fmm_set_option",
    "fmm_stencil", "fmm_pair_count", "fmm_p2m", "fmm_m2l", "fmm_m2l_noalloc", "fmm_p2m_m2l",
    "fmm_m2l_backward", "fmm_m2l_p2m_backward",
    "fmm_p2m_backward", "fmm_stencil_tables", "fmm_autotune", "fmm_evaluate",
    "fmm_tree_size", "fmm_tree_upward", "fmm_tree_m2l", "fmm_tree_downward", "fmm_tree_evaluate",
    "fmm_tree_solve",
]

DESC_DTYPE = np.dtype([("p", "<i4"), ("log2_inv_h", "<i4"), ("mask", "<u4"), ("reserved", "<i4"),
                       ("m_off", "<i8"), ("l_off", "<i8"), ("part_off", "<i8")])
assert DESC_DTYPE.itemsize == 40


class Tree(ctypes.Structure):
    """fmm_tree: a uniform n^3 domain of finest spacing 2^log2_h, order p, ppc
    particles per finest cell; harmonic = 1 selects the harmonic form of M2L."""
    _fields_ = [("p", ctypes.c_int32), ("n", ctypes.c_int32), ("ppc", ctypes.c_int32),
                ("log2_h", ctypes.c_int32), ("harmonic", ctypes.c_int32)]


class FMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (status_string(status), msg))
        self.status = status


_lib = None


def load_library(path=LIB_PATH):
    """Load libfmm.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libfmm.so not found at %s: build it with "
                          "`python -m paper_2304_11002_amd.build`" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "fmm_create": ([ctypes.POINTER(vp), i32], i32),
        "fmm_destroy": ([vp], i32),
        "fmm_status_string": ([i32], ctypes.c_char_p),
        "fmm_last_error": ([vp], ctypes.c_char_p),
        "fmm_set_option": ([vp, i32, i64], i32),
        "fmm_stencil": ([ctypes.POINTER(i32), vp], i32),
        "fmm_pair_count": ([vp, i64, ctypes.POINTER(i64)], i32),
        "fmm_p2m": ([vp, vp, i64, vp, vp, i32, vp, vp], i32),
        "fmm_m2l": ([vp, vp, i64, vp, vp, i32, vp], i32),
        "fmm_m2l_noalloc": ([vp, vp, i64, vp, vp, i32, vp], i32),
        "fmm_p2m_m2l": ([vp, vp, i64, vp, vp, i32, vp, vp, i32, vp], i32),
        "fmm_m2l_backward": ([vp, vp, i64, vp, vp, vp], i32),
        "fmm_p2m_backward": ([vp, vp, i64, vp, i32, vp, vp, vp], i32),
        "fmm_m2l_p2m_backward": ([vp, vp, i64, vp, i32, vp, vp, vp, vp], i32),
        "fmm_stencil_tables": ([vp, i32, vp, vp], i32),
        "fmm_autotune": ([vp, vp, i64, vp, vp, i32, vp, ctypes.POINTER(i32)], i32),
        "fmm_evaluate": ([vp, vp, i64, vp, vp, i32, vp, vp, vp], i32),
        "fmm_tree_size": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i64)], i32),
        "fmm_tree_upward": ([vp, vp, vp, vp, vp, vp], i32),
        "fmm_tree_m2l": ([vp, vp, vp, vp, vp], i32),
        "fmm_tree_downward": ([vp, vp, vp, vp], i32),
        "fmm_tree_evaluate": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "fmm_tree_solve": ([vp, vp, vp, vp, vp, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def status_string(status):
    return load_library().fmm_status_string(status).decode()


def _desc_ptr(desc):
    if desc is None or len(desc) == 0:
        return None, 0
    if not isinstance(desc, np.ndarray) or desc.dtype != DESC_DTYPE or not desc.flags.c_contiguous:
        raise TypeError("descriptors must be a C-contiguous numpy array of DESC_DTYPE")
    return desc.ctypes.data, len(desc)


def _ptr(t):
    """Device (or host) address of a tensor, or of None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _ncomp(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def _desc_extents(desc, ppc=None):
    """float64 elements each ragged buffer must hold for these descriptors:
    M and L up to the furthest block end, particles up to the furthest
    sub-grid's last particle. None where the descriptors (or ppc) are not
    valid: the library rejects those itself."""
    if desc is None or len(desc) == 0:
        return {}
    p = desc["p"].astype(np.int64)
    if p.min() < 2 or p.max() > 4:
        return {}
    C = _ncomp(p)
    ext = {}
    if (desc["m_off"] >= 0).all():
        ext["M"] = int((desc["m_off"] + C * NCELL).max())
    if (desc["l_off"] >= 0).all():
        ext["L"] = int((desc["l_off"] + C * NTARGET).max())
    if ppc is not None and 1 <= int(ppc) <= 64 and (desc["part_off"] >= 0).all():
        last = int((desc["part_off"] + NCELL * int(ppc)).max())
        ext["pos"], ext["mass"] = 3 * last, last
        ext["out"] = 4 * NTARGET * int(ppc) * len(desc)
    return ext


def _tree_extents(tree):
    t = (tree.p, tree.n, tree.ppc)
    if not (2 <= t[0] <= 4 and t[1] in (8, 16, 32, 64, 128) and 1 <= t[2] <= 64):
        return {}
    cells = t[1] ** 3
    ext = {"pos": 3 * cells * t[2], "mass": cells * t[2], "out": 4 * cells * t[2]}
    try:
        ext["M"] = ext["L"] = tree_size(tree)[1]
    except FMMError:
        pass
    return ext


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def stencil():
    """The 892 stencil offsets (dx, dy, dz) in the library's order."""
    lib = load_library()
    n = ctypes.c_int32()
    _check(lib.fmm_stencil(ctypes.byref(n), None), None)
    out = np.zeros((n.value, 3), np.int32)
    _check(lib.fmm_stencil(ctypes.byref(n), out.ctypes.data), None)
    return out


def pair_count(desc):
    lib = load_library()
    pd, n = _desc_ptr(desc)
    out = ctypes.c_int64()
    _check(lib.fmm_pair_count(pd, n, ctypes.byref(out)), None)
    return out.value


def tree_size(tree):
    """(levels, float64 elements of one M or L workspace) of a Tree."""
    lib = load_library()
    nl, ne = ctypes.c_int32(), ctypes.c_int64()
    _check(lib.fmm_tree_size(ctypes.byref(tree), ctypes.byref(nl), ctypes.byref(ne)), None)
    return nl.value, ne.value


def _check(status, ctx_handle):
    if status != FMM_OK:
        msg = load_library().fmm_last_error(ctx_handle).decode()
        raise FMMError(status, msg)


def ncomp(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def make_descriptors(p, log2_inv_h, mask, ppc=8):
    """Descriptors with packed, ragged M/L offsets and particle offsets.

    Returns (desc, m_elems, l_elems): total float64 elements of M and L.
    """
    p = np.asarray(p, np.int32)
    B = len(p)
    desc = np.zeros(B, DESC_DTYPE)
    desc["p"] = p
    desc["log2_inv_h"] = np.asarray(log2_inv_h, np.int32)
    desc["mask"] = np.asarray(mask, np.uint32)
    C = (p.astype(np.int64) + 1) * (p + 2) * (p + 3) // 6
    m_sz, l_sz = C * NCELL, C * NTARGET
    desc["m_off"] = np.concatenate([[0], np.cumsum(m_sz)[:-1]]) if B else []
    desc["l_off"] = np.concatenate([[0], np.cumsum(l_sz)[:-1]]) if B else []
    desc["part_off"] = np.arange(B, dtype=np.int64) * NCELL * ppc
    return desc, int(m_sz.sum()), int(l_sz.sum())


class Context:
    """One library context on one device (device=-1: host-only, checks only)."""

    def __init__(self, device=0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.fmm_create(ctypes.byref(h), int(device))
        if st != FMM_OK:
            raise FMMError(st, self.lib.fmm_last_error(None).decode())
        self.handle = h
        self.device = device
        self._options = {}

    def close(self):
        if self.handle:
            self.lib.fmm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _s(self, stream, n):
        # a host-only context never reaches a stream; empty batches need none
        if self.device < 0 or not n:
            return None
        return _stream(stream)

    def last_error(self):
        return self.lib.fmm_last_error(self.handle).decode()

    def _run(self, status):
        _check(status, self.handle)

    def _buf(self, t, ext, kind, name):
        """Address of a float64 buffer after the checks the C ABI cannot make
        (element type, contiguity, device, size). Integers pass through as raw
        addresses, which the caller vouches for."""
        if t is None or isinstance(t, int):
            return t
        if str(t.dtype) != "torch.float64":
            raise TypeError("%s must be float64, got %s" % (name, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if self.device >= 0 and (not t.is_cuda or t.device.index != self.device):
            raise ValueError("%s must be on cuda:%d, got %s" % (name, self.device, t.device))
        need = ext.get(kind)
        if need is not None and t.numel() < need:
            raise ValueError("%s holds %d elements, the descriptors address %d" % (name, t.numel(), need))
        return t.data_ptr()

    # the library's defaults (fmm.h), for get_option before any set_option
    _OPTION_DEFAULTS = {FMM_OPT_M2L_KERNEL: 0, FMM_OPT_USE_GRAPH: 1, FMM_OPT_TILE_CONFIG: -1,
                        FMM_OPT_ADJOINT_FORM: 0, FMM_OPT_P2M_WINDOW: 0, FMM_OPT_ROUND_SPLIT: -1,
                        FMM_OPT_SLICES: 7}

    def set_option(self, option, value):
        self._run(self.lib.fmm_set_option(self.handle, option, int(value)))
        self._options[option] = int(value)

    def get_option(self, option):
        """The value last set through this wrapper (the library keeps no getter)."""
        return self._options.get(option, self._OPTION_DEFAULTS.get(option))

    def p2m(self, desc, pos, mass, ppc, M, stream=None):
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc, ppc)
        self._run(self.lib.fmm_p2m(self.handle, pd, n, self._buf(pos, e, "pos", "pos"),
                                   self._buf(mass, e, "mass", "mass"), int(ppc), self._buf(M, e, "M", "M"),
                                   self._s(stream, n)))

    def m2l(self, desc, M, L, precision=FMM_FP64, stream=None):
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc)
        self._run(self.lib.fmm_m2l(self.handle, pd, n, self._buf(M, e, "M", "M"), self._buf(L, e, "L", "L"),
                                   int(precision), self._s(stream, n)))

    def m2l_noalloc(self, desc, M, L, precision=FMM_FP64, stream=None):
        """fmm_m2l_noalloc: M2L with no allocation (static device array, at most
        NOALLOC_MAX_SUBGRIDS sub-grids; overlapping calls on one GPU race)."""
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc)
        self._run(self.lib.fmm_m2l_noalloc(self.handle, pd, n, self._buf(M, e, "M", "M"),
                                           self._buf(L, e, "L", "L"), int(precision), self._s(stream, n)))

    def p2m_m2l(self, desc, pos, mass, ppc, M, L, precision=FMM_FP64, stream=None):
        """P2M over the rows holding the reachable window, then M2L, in one launch."""
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc, ppc)
        self._run(self.lib.fmm_p2m_m2l(self.handle, pd, n, self._buf(pos, e, "pos", "pos"),
                                       self._buf(mass, e, "mass", "mass"), int(ppc), self._buf(M, e, "M", "M"),
                                       self._buf(L, e, "L", "L"), int(precision), self._s(stream, n)))

    def m2l_backward(self, desc, dL, dM, stream=None):
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc)
        self._run(self.lib.fmm_m2l_backward(self.handle, pd, n, self._buf(dL, e, "L", "dL"),
                                            self._buf(dM, e, "M", "dM"), self._s(stream, n)))

    def m2l_p2m_backward(self, desc, pos, ppc, dL, dM, dmass, stream=None):
        """M2L adjoint (dL -> dM) and P2M adjoint (dM -> dmass) in one launch."""
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc, ppc)
        self._run(self.lib.fmm_m2l_p2m_backward(self.handle, pd, n, self._buf(pos, e, "pos", "pos"), int(ppc),
                                                self._buf(dL, e, "L", "dL"), self._buf(dM, e, "M", "dM"),
                                                self._buf(dmass, e, "mass", "dmass"), self._s(stream, n)))

    def p2m_backward(self, desc, pos, ppc, dM, dmass, stream=None):
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc, ppc)
        self._run(self.lib.fmm_p2m_backward(self.handle, pd, n, self._buf(pos, e, "pos", "pos"), int(ppc),
                                            self._buf(dM, e, "M", "dM"), self._buf(dmass, e, "mass", "dmass"),
                                            self._s(stream, n)))

    def evaluate(self, desc, pos, mass, ppc, L, out, stream=None):
        """Near field + L2P: out [nsub, 4, 512, ppc] (phi, grad x, y, z)."""
        pd, n = _desc_ptr(desc)
        e = _desc_extents(desc, ppc)
        self._run(self.lib.fmm_evaluate(self.handle, pd, n, self._buf(pos, e, "pos", "pos"),
                                        self._buf(mass, e, "mass", "mass"), int(ppc), self._buf(L, e, "L", "L"),
                                        self._buf(out, e, "out", "out"), self._s(stream, n)))

    # multi-level iteration on a uniform octree (tree: a Tree)
    def tree_upward(self, tree, pos, mass, M, stream=None):
        e = _tree_extents(tree)
        self._run(self.lib.fmm_tree_upward(self.handle, ctypes.byref(tree), self._buf(pos, e, "pos", "pos"),
                                           self._buf(mass, e, "mass", "mass"), self._buf(M, e, "M", "M"),
                                           self._s(stream, 1)))

    def tree_m2l(self, tree, M, L, stream=None):
        e = _tree_extents(tree)
        self._run(self.lib.fmm_tree_m2l(self.handle, ctypes.byref(tree), self._buf(M, e, "M", "M"),
                                        self._buf(L, e, "L", "L"), self._s(stream, 1)))

    def tree_downward(self, tree, L, stream=None):
        e = _tree_extents(tree)
        self._run(self.lib.fmm_tree_downward(self.handle, ctypes.byref(tree), self._buf(L, e, "L", "L"),
                                             self._s(stream, 1)))

    def tree_evaluate(self, tree, pos, mass, L, out, stream=None):
        e = _tree_extents(tree)
        self._run(self.lib.fmm_tree_evaluate(self.handle, ctypes.byref(tree), self._buf(pos, e, "pos", "pos"),
                                             self._buf(mass, e, "mass", "mass"), self._buf(L, e, "L", "L"),
                                             self._buf(out, e, "out", "out"), self._s(stream, 1)))

    def tree_solve(self, tree, pos, mass, M, L, out, stream=None):
        e = _tree_extents(tree)
        self._run(self.lib.fmm_tree_solve(self.handle, ctypes.byref(tree), self._buf(pos, e, "pos", "pos"),
                                          self._buf(mass, e, "mass", "mass"), self._buf(M, e, "M", "M"),
                                          self._buf(L, e, "L", "L"), self._buf(out, e, "out", "out"),
                                          self._s(stream, 1)))

    def stencil_tables(self, p, out, stream=None):
        e = {"out": NSTENCIL * _ncomp(int(p)) ** 2} if 2 <= int(p) <= 4 else {}
        self._run(self.lib.fmm_stencil_tables(self.handle, int(p), self._buf(out, e, "out", "out"),
                                              self._s(stream, 1)))

    def autotune(self, desc, M, L, precision=FMM_FP64, stream=None):
        pd, n = _desc_ptr(desc)
        chosen = ctypes.c_int32(-1)
        e = _desc_extents(desc)
        self._run(self.lib.fmm_autotune(self.handle, pd, n, self._buf(M, e, "M", "M"), self._buf(L, e, "L", "L"),
                                        int(precision), self._s(stream, n), ctypes.byref(chosen)))
        return chosen.value
