"""Plain CPU oracle for the same-level multipole-to-local (M2L) gravity interaction.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it. It shares no code with the HIP library (no kernels,
headers, tables, helpers or generated constants); the only code both sides use
is the seeded input generator in ``synth/``, which holds none of the method's
arithmetic.

What it computes follows the gravity solver described in the paper's
Octo-Tiger subsection (Sec. IV-C, "Octo-Tiger"): cell moments on N^3 = 8^3
sub-grids co-located with the hydro grid, and the same-level cell-to-cell
interaction step of the three-step gravity iteration (Sec. VII-C, "Usage of
multiple HPX tasks per Kokkos kernel invocation"). The paper gives no
formulas; the definitions written out here are textbook Cartesian FMM, and
each function states the reading it takes where the paper is silent.

``oracle.tree`` extends the same definitions to the whole three-step iteration
on a uniform octree (P2M, M2M, interaction-list M2L on every level, L2L, and
the near field plus L2P at the finest level).

Every floating-point step is plain NumPy float64 (float32 only in the
split-precision emulation, which is an expectation model, not a reference).
The exact-slice model (``m2l_exact_slice``) adds integer slice products,
summed exactly in int64; it, too, is an expectation model of a reduced
precision, pinned against the float64 M2L it approximates.
"""

from .fmm import (  # noqa: F401
    BLOCK,
    FRAME,
    FULL_MASK,
    NCELL,
    CENTRE_BIT,
    double_factorial,
    multi_indices,
    ncomp,
    stencil,
    dtensor,
    dtensor_all,
    cell_centres,
    present_cells,
    p2m,
    stencil_tensors,
    m2l,
    m2l_abs,
    m2l_adjoint,
    near_stencil,
    l2p,
    l2p_abs,
    near_field,
    near_field_abs,
    evaluate,
    harmonic_indices,
    harmonic_fold,
    m2l_harmonic,
    m2l_adjoint_abs,
    p2m_adjoint,
    direct_sum,
    m2l_split32_emulated,
    pair_count,
    SLICE_BITS,
    slice_prescale,
    pow2_exponent,
    slice_int8,
    slice_pairs,
    slice_tables,
    m2l_exact_slice,
)
