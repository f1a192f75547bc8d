"""torch.autograd binding of the forward path (P2M then M2L) and its adjoint.

    L = gravity_local_expansion(ctx, desc, pos, mass)   # differentiable in mass

Forward runs fmm_p2m_m2l (P2M and M2L, in one launch for large batches);
backward runs fmm_m2l_p2m_backward (adjoint M2L, dL -> dM, and adjoint P2M,
dM -> d mass, likewise). Positions are held fixed (no gradient). harmonic=True computes M2L and its adjoint in the
harmonic (traceless) form, equal to the dense form up to rounding. Every
step runs in the library's HIP kernels; torch supplies device memory and
the stream.
"""
import torch

from . import fmm


class FMMGravity(torch.autograd.Function):
    @staticmethod
    def forward(actx, mass, pos, handle, desc, ppc, m_elems, l_elems, harmonic):
        M = torch.empty(m_elems, dtype=torch.float64, device=mass.device)
        L = torch.empty(l_elems, dtype=torch.float64, device=mass.device)
        mass_c = mass.contiguous()
        handle.p2m_m2l(desc, pos, mass_c, ppc, M, L, fmm.FMM_FP64_HARMONIC if harmonic else fmm.FMM_FP64)
        actx.save_for_backward(pos)
        actx.handle, actx.desc, actx.ppc, actx.m_elems = handle, desc, ppc, m_elems
        actx.harmonic = harmonic
        actx.mass_shape = mass.shape
        return L

    @staticmethod
    def backward(actx, gL):
        (pos,) = actx.saved_tensors
        gL = gL.contiguous()
        dM = torch.empty(actx.m_elems, dtype=torch.float64, device=gL.device)
        dmass = torch.empty(actx.mass_shape, dtype=torch.float64, device=gL.device)
        prev = actx.handle.get_option(fmm.FMM_OPT_ADJOINT_FORM)
        actx.handle.set_option(fmm.FMM_OPT_ADJOINT_FORM, 1 if actx.harmonic else 0)
        try:
            actx.handle.m2l_p2m_backward(actx.desc, pos, actx.ppc, gL, dM, dmass)
        finally:
            actx.handle.set_option(fmm.FMM_OPT_ADJOINT_FORM, prev)
        return dmass, None, None, None, None, None, None, None


def gravity_local_expansion(handle, desc, pos, mass, ppc=8, harmonic=False):
    """L of every sub-grid (flat, ragged by order), differentiable in `mass`."""
    if pos.dtype != torch.float64 or mass.dtype != torch.float64:
        raise TypeError("pos and mass must be float64")
    if not (pos.is_cuda and mass.is_cuda):
        raise ValueError("pos and mass must be device tensors")
    p = desc["p"].astype("int64")
    C = (p + 1) * (p + 2) * (p + 3) // 6
    m_elems = int((C * fmm.NCELL).sum())
    l_elems = int((C * fmm.NTARGET).sum())
    return FMMGravity.apply(mass, pos.contiguous(), handle, desc, ppc, m_elems, l_elems, harmonic)
