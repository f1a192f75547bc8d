"""MI355X (gfx950) same-level FMM interaction library: C-ABI HIP kernels
(libfmm.so) and a thin Python binding (`fmm`, `autograd`)."""
