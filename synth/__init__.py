"""Seeded synthetic inputs for the sub-grid M2L workloads.

This module is shared by the oracle and by the HIP path's tests and bench,
so it holds none of the method's arithmetic: it only draws random numbers
and lays them out. Everything is reproducible per sub-grid, so any subset of
a large batch can be regenerated for the oracle without the rest.

Per sub-grid b of a batch with seed s: rng = numpy default_rng([s, b])
(the single-sub-grid case uses default_rng(s)); draws, in this order:
    u    = rng.random((24, 24, 24, ppc, 3))        indexed [z][y][x][i][xyz]
    mass = rng.lognormal(0.0, 1.0, (24, 24, 24, ppc))
positions y = (j + u) h with j the cell's (x, y, z) frame index, so every
particle lies inside its cell [j h, (j + 1) h). Per-batch draws (orders,
spacings, masks, loss weights, finite-difference entries) come from
default_rng([s, 2**31 - 1]).

The workloads stand in for the paper's production runs (thousands to
millions of 8^3 sub-grids per step, Sec. IV-B "Kokkos and HPX-Kokkos"), whose inputs are
not available; shapes follow the Octo-Tiger sub-grid layout (Sec. IV-C
"Octo-Tiger").
"""

import os
from dataclasses import dataclass, field
from multiprocessing import get_context, shared_memory

import numpy as np

FRAME = 24
NCELL = FRAME ** 3
FULL_MASK = (1 << 27) - 1
CENTRE_BIT = 13
META_STREAM = 2 ** 31 - 1
NEIGHBOUR_BITS = [b for b in range(27) if b != CENTRE_BIT]


def _rng(seed, b):
    return np.random.default_rng(seed if b is None else [seed, b])


def subgrid_particles(seed, b=None, h=1.0, ppc=8):
    """Positions [13824, ppc, 3] and masses [13824, ppc] of one sub-grid frame."""
    rng = _rng(seed, b)
    u = rng.random((FRAME, FRAME, FRAME, ppc, 3))
    mass = rng.lognormal(0.0, 1.0, (FRAME, FRAME, FRAME, ppc))
    g = np.arange(FRAME, dtype=np.float64)
    j = np.stack(np.meshgrid(g, g, g, indexing="ij")[::-1], axis=-1)   # [z][y][x] -> (x, y, z)
    pos = (j[:, :, :, None, :] + u) * h
    return pos.reshape(NCELL, ppc, 3), mass.reshape(NCELL, ppc)


def grid_particles(seed, n, h=1.0, ppc=8):
    """Positions [n^3, ppc, 3] and masses [n^3, ppc] of a uniform n^3-cell domain
    (cell index x + n y + n^2 z), drawn like subgrid_particles: u uniform in the
    cell, lognormal(0, 1) masses, rng = default_rng([seed, 2**30 + n])."""
    rng = np.random.default_rng([seed, 2 ** 30 + n])
    u = rng.random((n, n, n, ppc, 3))
    mass = rng.lognormal(0.0, 1.0, (n, n, n, ppc))
    g = np.arange(n, dtype=np.float64)
    j = np.stack(np.meshgrid(g, g, g, indexing="ij")[::-1], axis=-1)
    pos = (j[:, :, :, None, :] + u) * h
    return pos.reshape(n ** 3, ppc, 3), mass.reshape(n ** 3, ppc)


@dataclass
class Workload:
    """A batch description: per-sub-grid order, spacing exponent and mask."""
    name: str
    seed: int
    p: np.ndarray            # int32 [B]
    log2_inv_h: np.ndarray   # int32 [B], h = 2^-log2_inv_h
    mask: np.ndarray         # uint32 [B]
    ppc: int = 8
    extra: dict = field(default_factory=dict)

    @property
    def nsub(self):
        return int(self.p.shape[0])

    def h(self, b):
        return 2.0 ** -int(self.log2_inv_h[b])


def uniform_workload(name, seed, nsub, p=3):
    return Workload(name, seed,
                    np.full(nsub, p, np.int32),
                    np.zeros(nsub, np.int32),
                    np.full(nsub, FULL_MASK, np.uint32))


def random_mask(rng):
    """Mask with n_abs ~ U{1..26} neighbour blocks absent, chosen uniformly."""
    n_abs = int(rng.integers(1, 27))
    absent = rng.choice(NEIGHBOUR_BITS, size=n_abs, replace=False)
    m = FULL_MASK
    for bit in absent:
        m &= ~(1 << int(bit))
    return m


def uneven_workload(name, seed, nsub, p_ratio=(1, 2, 1), orders=(2, 3, 4), spacings=(0, 1, 2)):
    """Mixed orders in the given ratio (exact counts, permuted), spacing
    exponents uniform over `spacings`, random boundary masks."""
    meta = np.random.default_rng([seed, META_STREAM])
    tot = sum(p_ratio)
    counts = [nsub * r // tot for r in p_ratio]
    counts[orders.index(3) if 3 in orders else 0] += nsub - sum(counts)
    ps = np.concatenate([np.full(c, o, np.int32) for c, o in zip(counts, orders)])
    ps = meta.permutation(ps).astype(np.int32)
    lh = meta.choice(np.asarray(spacings, np.int32), size=nsub).astype(np.int32)
    masks = np.array([random_mask(meta) for _ in range(nsub)], dtype=np.uint32)
    return Workload(name, seed, ps, lh, masks)


def config(n, nsub=None):
    """The five benchmark workloads (sizes can be reduced with nsub for tests).

    1: one p=3 sub-grid, seed 0, all neighbours present.
    2: 4096 uniform p=3 sub-grids (seed 2).
    3: 6000 sub-grids, p in {2,3,4} as 1:2:1, h in {1, 1/2, 1/4}, random masks (seed 3).
    4: the workload of 2, evaluated in split precision.
    5: 2048 uniform p=3 sub-grids (seed 5) with loss weights and 64 FD entries.
    """
    if n == 1:
        return uniform_workload("single_subgrid_p3", 0, 1)
    if n in (2, 4):
        return uniform_workload("uniform_4096_p3", 2, nsub or 4096)
    if n == 3:
        return uneven_workload("uneven_6000_mixed_p", 3, nsub or 6000)
    if n == 5:
        w = uniform_workload("grad_2048_p3", 5, nsub or 2048)
        return w
    raise ValueError(n)


def subgrid_seed_args(w, b):
    """(seed, b) for default_rng: the single-sub-grid workload uses the bare seed."""
    return (w.seed, None) if w.name == "single_subgrid_p3" else (w.seed, b)


def loss_weights(seed, nsub, C=20):
    """w ~ N(0, 1) of shape [B, C, 512] from the meta stream."""
    meta = np.random.default_rng([seed, META_STREAM])
    return meta.standard_normal((nsub, C, 512))


def fd_entries(seed, nsub, count=64, ppc=8):
    """`count` (b, cell, i) particle entries inside the reachable 20^3 window."""
    meta = np.random.default_rng([seed, META_STREAM, 1])
    b = meta.integers(0, nsub, count)
    jx, jy, jz = (meta.integers(2, 22, count) for _ in range(3))
    i = meta.integers(0, ppc, count)
    return np.stack([b, jx + FRAME * jy + FRAME * FRAME * jz, i], axis=1)


# ---------------------------------------------------------------------------
# parallel batch generation into shared memory
# ---------------------------------------------------------------------------

def _fill(args):
    shm_pos, shm_mass, shape_pos, shape_mass, seed, bare, rows, hs, ppc = args
    sp = shared_memory.SharedMemory(name=shm_pos)
    sm = shared_memory.SharedMemory(name=shm_mass)
    try:
        P = np.ndarray(shape_pos, dtype=np.float64, buffer=sp.buf)
        Mm = np.ndarray(shape_mass, dtype=np.float64, buffer=sm.buf)
        for row, h in zip(rows, hs):
            pos, mass = subgrid_particles(seed, None if bare else row, h, ppc)
            P[row] = pos
            Mm[row] = mass
    finally:
        sp.close()
        sm.close()
    return len(rows)


class SharedBatch:
    """Positions [B, 13824, ppc, 3] and masses [B, 13824, ppc] in shared memory."""

    def __init__(self, w, workers=None):
        B, ppc = w.nsub, w.ppc
        self.shape_pos = (B, NCELL, ppc, 3)
        self.shape_mass = (B, NCELL, ppc)
        self._sp = shared_memory.SharedMemory(create=True, size=max(8, 8 * int(np.prod(self.shape_pos))))
        self._sm = shared_memory.SharedMemory(create=True, size=max(8, 8 * int(np.prod(self.shape_mass))))
        self.pos = np.ndarray(self.shape_pos, dtype=np.float64, buffer=self._sp.buf)
        self.mass = np.ndarray(self.shape_mass, dtype=np.float64, buffer=self._sm.buf)
        bare = w.name == "single_subgrid_p3"
        hs = [w.h(b) for b in range(B)]
        if workers is None:
            workers = min(16, len(os.sched_getaffinity(0)))
        workers = max(1, min(workers, B))
        chunks = [list(range(s, B, workers)) for s in range(workers)]
        jobs = [(self._sp.name, self._sm.name, self.shape_pos, self.shape_mass, w.seed, bare,
                 c, [hs[r] for r in c], ppc) for c in chunks if c]
        if workers == 1:
            for j in jobs:
                _fill(j)
        else:
            with get_context("fork").Pool(workers) as pool:
                pool.map(_fill, jobs)

    def close(self):
        for s in (self._sp, self._sm):
            try:
                s.close()
                s.unlink()
            except FileNotFoundError:
                pass
        self.pos = self.mass = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
