"""The allocation-free entry point (moco_align_noalloc) against moco_align, on
the GPU, through the C ABI: the same kernels on the library's fixed per-device
scratch instead of the context's must give the same results bit for bit.  Two
calls in a row, the second with a smaller input, so the second runs on the
contents the first left in the shared array; forms int8, FFT and FP64; a stack
larger than one chunk of the fixed scratch; a frame too large for it is
refused."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

KEYS = ("shifts", "fmin", "frefine", "coarse", "gaps", "recomputed")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host(r, surface):
    keys = KEYS + (("fsurf",) if surface else ())
    return {k: getattr(r, k).cpu().numpy() for k in keys}


def _same(a, b, label):
    for k in a:
        x, y = a[k], b[k]
        if x.dtype == np.float64:
            x, y = x.view(np.int64), y.view(np.int64)
        assert np.array_equal(x, y), (label, k)


def _pair(moco, ctx, frames, tp, form, surface):
    T = frames.shape[0]
    ref = moco.moco_align(ctx, frames, tp, form=form, surface=surface)
    out = moco._new_result(T, 2 * tp.w - 1, frames.device, surface)
    for v in vars(out).values():      # stale values must not leak into the results
        if v is not None:
            v.fill_(-7)
    got = moco.moco_align_noalloc(ctx, frames, tp, out, form=form)
    torch.cuda.synchronize()
    return _host(ref, surface), _host(got, surface)


CASES = [
    # (label, scene factory, w, ds, form, first T, second T)
    ("poisson512_int8", lambda: synth.poisson512_u16(T=64), 32, True, "int8", 40, 3),
    # 2w - 1 = 15: the int8 correlation's half tile (two 16x16 shift tiles per product)
    ("poisson256_int8_w8", lambda: synth.PoissonScene(256, 256, 41, seed=5), 8, False, "int8",
     40, 3),
    ("poisson512_fft_cert", lambda: synth.poisson512_u16(T=64), 32, True, "fft_cert", 60, 5),
    ("poisson512_fft32_cert", lambda: synth.poisson512_u16(T=64), 32, True, "fft32_cert", 30, 4),
    ("blobs128_fft", lambda: synth.blobs128_f32(), 10, False, "fft", 100, 7),
    ("blobs128_fp64", lambda: synth.blobs128_f32(), 10, False, "fp64", 20, 2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_noalloc_equals_align_two_calls(gpu_lib, case):
    label, make, w, ds, form, T1, T2 = case
    moco = gpu_lib
    sc = make()
    fr = sc.frames(0, T1)
    ctx = moco.Context(0)
    tp = moco.Template(ctx, torch.from_numpy(np.ascontiguousarray(sc.template)).cuda(), w, ds)
    for T in (T1, T2):
        _say("case noalloc %s T=%d" % (label, T))
        frames = torch.from_numpy(np.ascontiguousarray(fr[:T])).cuda()
        ref, got = _pair(moco, ctx, frames, tp, form, surface=True)
        _same(ref, got, "%s T=%d" % (label, T))
    tp.close()
    ctx.close()


def test_noalloc_stack_larger_than_fixed_scratch(gpu_lib):
    # the FFT form at 512x512 needs over 1 MB of scratch per frame: 200 frames
    # take several chunks of the 64 MiB array, then a short stack reuses it
    moco = gpu_lib
    sc = synth.poisson512_u16(T=200)
    fr = sc.frames(0, 200)
    ctx = moco.Context(0)
    tp = moco.Template(ctx, torch.from_numpy(sc.template).cuda(), 32, True)
    for T in (200, 9):
        _say("case noalloc chunked fft_cert T=%d" % T)
        frames = torch.from_numpy(np.ascontiguousarray(fr[:T])).cuda()
        ref, got = _pair(moco, ctx, frames, tp, "fft_cert", surface=False)
        _same(ref, got, "chunked T=%d" % T)
    tp.close()
    ctx.close()


def test_noalloc_refuses_a_frame_beyond_the_fixed_scratch(gpu_lib):
    # a 4096x4096 frame searched at full resolution needs a 128 MiB FP64 grid
    moco = gpu_lib
    ctx = moco.Context(0, scratch_budget=1 << 30)
    tmpl = torch.zeros((4096, 4096), dtype=torch.uint16, device="cuda")
    tp = moco.Template(ctx, tmpl, 2, False)
    frames = torch.zeros((1, 4096, 4096), dtype=torch.uint16, device="cuda")
    out = moco._new_result(1, 3, frames.device, False)
    _say("case noalloc refusal 4096x4096")
    with pytest.raises(moco.MocoError) as ei:
        moco.moco_align_noalloc(ctx, frames, tp, out, form="fp64")
    assert ei.value.code == moco.MOCO_ENOMEM
    tp.close()
    ctx.close()
