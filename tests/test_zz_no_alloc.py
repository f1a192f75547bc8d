"""fmm_m2l_noalloc (descriptors, work list and counter in a static device array;
no allocation) against fmm_m2l with the same configuration: bit for bit, on
two calls in a row, the second with a smaller batch than the first (the array
keeps the first call's contents beyond the second's)."""
import numpy as np
import pytest

import synth
from paper_2304_11002_amd import fmm

from _gpu_helpers import ensure_library, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _batch(torch, seed, n):
    rng = np.random.default_rng(seed)
    p = rng.integers(2, 5, n)
    masks = [synth.random_mask(rng) if rng.random() < 0.7 else fmm.FULL_MASK for _ in range(n)]
    desc, m_el, l_el = fmm.make_descriptors(p, rng.integers(0, 3, n), masks)
    M = torch.from_numpy(rng.standard_normal(m_el)).to("cuda")
    return desc, M, l_el


@pytest.mark.parametrize("prec", [fmm.FMM_FP64_HARMONIC, fmm.FMM_FP64, fmm.FMM_SPLIT_FP32])
def test_noalloc_equals_m2l_on_two_calls(torch, prec):
    ensure_library()
    first = _batch(torch, 51, 600)     # more sub-grids than compute units
    second = _batch(torch, 52, 37)
    with fmm.Context(0) as ctx:
        for desc, M, l_el in (first, second):
            want = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
            got = torch.full((l_el,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.m2l(desc, M, want, prec)
            ctx.m2l_noalloc(desc, M, got, prec)
            torch.cuda.synchronize()
            assert bool(torch.isfinite(got).all())
            assert torch.equal(got, want), "nsub %d, precision %d" % (len(desc), prec)


def test_noalloc_rejects_what_it_cannot_run(torch):
    ensure_library()
    desc, M, l_el = _batch(torch, 53, 3)
    L = torch.zeros(l_el, dtype=torch.float64, device="cuda")
    with fmm.Context(0) as ctx:
        d3, m3, l3 = fmm.make_descriptors([3], [0], [fmm.FULL_MASK])
        with pytest.raises(fmm.FMMError) as ex:
            ctx.m2l_noalloc(d3, torch.zeros(m3, dtype=torch.float64, device="cuda"),
                            torch.zeros(l3, dtype=torch.float64, device="cuda"), fmm.FMM_EXACT_SLICE)
        assert ex.value.status == fmm.FMM_EUNSUPPORTED
        big = np.zeros(fmm.NOALLOC_MAX_SUBGRIDS + 1, fmm.DESC_DTYPE)
        big["p"], big["mask"] = 3, fmm.FULL_MASK
        with pytest.raises(fmm.FMMError) as ex:
            ctx.m2l_noalloc(big, M.data_ptr(), L.data_ptr())
        assert ex.value.status == fmm.FMM_EINVAL and "16384" in str(ex.value)
