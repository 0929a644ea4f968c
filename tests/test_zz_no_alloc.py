"""disco_set_images_noalloc (static scratch, no device allocation) against disco_set_images.

Both entry points run the same kernels; the no-allocation form keeps the FP16 scale
search's per-block maxima in a static device array instead of a per-call allocation.
The stored gradient volumes, and an objective evaluated from them, must be bitwise equal
to those of disco_set_images on fresh contexts.  Two calls in a row share the array: the
second, on a smaller volume, must not see the first call's contents.  A volume whose
block count exceeds the array is rejected with a limit error before anything runs.
"""
import numpy as np
import pytest
import torch

import synth
from tests.fields import say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

# first call on the larger volume, then the smaller one
SHAPES = [((96, 80, 72), (1.1, 1.3, 1.7), 31), ((32, 24, 20), (1.5, 1.5, 2.0), 32)]


@pytest.fixture(scope="module")
def disco():
    from paper_1807_00467_amd import disco as d
    return d


def _pair(shape, spacing, seed):
    d = synth.small_pair(shape=shape, spacing=spacing, seed=seed, n_tubes=8, n_kp=0, field_max=4.0)
    return d, torch.from_numpy(d["R"]).to(DEV), torch.from_numpy(d["T"]).to(DEV)


def _state(disco, ctx, u):
    bufs = [ctx.copy_buffer(b).cpu() for b in (disco.BUF_GRAD_R, disco.BUF_GRAD_T)]
    J = ctx.ngf_eval(u, 10.0).cpu()
    torch.cuda.synchronize()
    return bufs, J


def _bits(t):
    t = t.contiguous()
    return t.view(torch.int16) if t.element_size() == 2 else t.view(torch.int32)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_noalloc_matches_set_images(disco, storage):
    shared = []
    for shape, spacing, seed in SHAPES:
        say(f"[noalloc] storage={storage} shape={shape} seed={seed}")
        d, R, T = _pair(shape, spacing, seed)
        u = torch.from_numpy(np.ascontiguousarray(0.5 * d["u_true"], dtype=np.float32)).to(DEV)
        ref_ctx = disco.Disco(d["shape"], d["spacing"], storage=storage, device=DEV)
        new_ctx = disco.Disco(d["shape"], d["spacing"], storage=storage, device=DEV)
        try:
            ref_ctx.set_images(R, T)
            new_ctx.set_images_noalloc(R, T)
            (rb, rJ), (nb, nJ) = _state(disco, ref_ctx, u), _state(disco, new_ctx, u)
            for name, a, b in zip(("grad R", "grad T"), rb, nb):
                assert a.dtype == b.dtype and a.shape == b.shape, name
                ndiff = int((_bits(a) != _bits(b)).sum())
                say(f"  {name}: {a.numel()} stored values, {ndiff} differ")
                assert ndiff == 0, f"{name}: {ndiff} values differ from disco_set_images"
            say(f"  NGF distance {float(nJ):.17g} vs {float(rJ):.17g}")
            assert float(nJ) == float(rJ)
            shared.append(float(nJ))
        finally:
            ref_ctx.close()
            new_ctx.close()
    assert len(shared) == 2


def test_noalloc_rejects_oversize_fp16(disco):
    # 4 x 4 x 262160 voxels: 16385 tiles of 64 x 16 x 16 > the 2^14 held by the static
    # array (a thin volume, so the test needs little memory)
    shape = (4, 4, 16 * 16384 + 16)
    say(f"[noalloc] oversize fp16 shape={shape}")
    ctx = disco.Disco(shape, (1.0, 1.0, 1.0), storage="fp16", device=DEV)
    try:
        R = torch.zeros(shape[::-1], dtype=torch.float32, device=DEV)
        with pytest.raises(disco.DiscoError) as ei:
            ctx.set_images_noalloc(R, R)
        assert ei.value.code == disco.ERR_LIMIT
        say(f"  rejected: {ei.value}")
        # nothing was queued: the allocating form still works on the same context
        ctx.set_images(R, R)
    finally:
        ctx.close()
