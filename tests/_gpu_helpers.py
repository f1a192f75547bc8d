"""Shared helpers of the GPU tests: device buffers for a workload, the HIP
path through the C ABI, and oracle results for chosen sub-grids."""
import numpy as np

import oracle as O
import synth
from paper_2304_11002_amd import fmm


def ensure_library():
    import os
    if not os.path.exists(fmm.LIB_PATH):
        from paper_2304_11002_amd import build
        build.build()
    return fmm.load_library()


def particles(w, idx=None):
    """Host (pos, mass) stacked for the given sub-grid indices of workload w."""
    idx = range(w.nsub) if idx is None else idx
    P, Mm = [], []
    for b in idx:
        seed, bb = synth.subgrid_seed_args(w, b)
        pos, mass = synth.subgrid_particles(seed, bb, w.h(b), w.ppc)
        P.append(pos)
        Mm.append(mass)
    return np.stack(P), np.stack(Mm)


def descriptors(w, idx=None):
    idx = list(range(w.nsub)) if idx is None else list(idx)
    return fmm.make_descriptors(w.p[idx], w.log2_inv_h[idx], w.mask[idx], w.ppc)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def oracle_subgrid(w, b, pos=None, mass=None, with_abs=True):
    """Oracle M, L (and Labs) of sub-grid b of workload w."""
    if pos is None:
        seed, bb = synth.subgrid_seed_args(w, b)
        pos, mass = synth.subgrid_particles(seed, bb, w.h(b), w.ppc)
    p, h, mask = int(w.p[b]), w.h(b), int(w.mask[b])
    M = O.p2m(pos, mass, p, h, mask)
    L = O.m2l(M, p, h, mask)
    La = O.m2l_abs(M, p, h, mask) if with_abs else None
    return M, L, La


def moment_abs_scale(pos, mass, p, h, mask):
    """sum_i |m_i| |a_i^k| / k!: the rounding scale of P2M, via the oracle on |a|."""
    c = O.cell_centres(h)[:, None, :]
    return O.p2m(c + np.abs(pos - c), np.abs(mass), p, h, mask)


def split_views(flat, desc, kind):
    """Per-sub-grid views of a flat ragged M or L array."""
    out = []
    for d in desc:
        C = fmm.ncomp(int(d["p"]))
        if kind == "M":
            o = int(d["m_off"])
            out.append(flat[o:o + C * fmm.NCELL].reshape(C, 24, 24, 24))
        else:
            o = int(d["l_off"])
            out.append(flat[o:o + C * fmm.NTARGET].reshape(C, 8, 8, 8))
    return out
