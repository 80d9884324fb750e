"""Parity of the FFT form (FP64 complex transforms of the zero-padded grids,
sec. 2) with the FP64 oracle, on the GPU, through the C ABI.

The FFT form is a floating-point form: f is held to the 1e-5 relative rule of
``tests/_parity.py`` (in practice it lands near 1e-13), shifts to bit equality
on frames with clear gaps.  On uint16 data its f is also compared with the
int8 form's exact f.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._parity import check, check_surface

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(moco, frames, tmpl, w, ds, form="fft", surface=False, ctx=None):
    own = ctx is None
    if own:
        ctx = moco.Context(0)
    tp = moco.Template(ctx, _to_dev(tmpl), w, ds)
    r = moco.moco_align(ctx, _to_dev(frames), tp, form=form, surface=surface)
    torch.cuda.synchronize()
    out = {k: getattr(r, k).cpu().numpy() for k in ("shifts", "fmin", "frefine", "coarse", "gaps")}
    if surface:
        out["fsurf"] = r.fsurf.cpu().numpy()
    tp.close()
    if own:
        ctx.close()
    return out


def test_fft_blobs128_f32_all_frames(gpu_lib):
    # 128x128 float32, w = 10, no downsampling: P = Q = 144 (radices 8,2,3,3)
    sc = synth.blobs128_f32()
    fr = sc.frames(0, 100)
    _say("case fft blobs128_f32 T=100 w=10 ds=0")
    res = _run(gpu_lib, fr, sc.template, 10, False, surface=True)
    orc = oracle.align(fr, sc.template, 10, False, want_surface=True)
    st = check(res, orc, False, exact=False, label="fft blobs128")
    err = check_surface(res["fsurf"], orc.surf, label="fft blobs128 surface")
    assert np.array_equal(res["shifts"], sc.shifts(0, 100))
    _say(st, "surface max rel err %.3g" % err)
    assert err < 1e-9


def test_fft_poisson512_u16_ds_against_oracle_and_int8(gpu_lib):
    # 512x512 uint16 -> 256x256 grid, w = 32: P = Q = 288 (radices 8,4,3,3)
    sc = synth.poisson512_u16(T=2000)
    fr = sc.frames(0, 24)
    _say("case fft poisson512_u16 T=24 w=32 ds=1")
    res = _run(gpu_lib, fr, sc.template, 32, True, surface=True)
    orc = oracle.align(fr, sc.template, 32, True, want_surface=True)
    st = check(res, orc, True, exact=False, label="fft poisson512")
    err = check_surface(res["fsurf"], orc.surf, label="fft poisson512 surface")
    _say(st, "surface max rel err %.3g" % err)
    assert err < 1e-9
    ex = _run(gpu_lib, fr, sc.template, 32, True, form="int8", surface=True)
    assert np.array_equal(res["shifts"], ex["shifts"])
    assert np.array_equal(res["coarse"], ex["coarse"])
    # (frame 0 is the template: f(0,0) = 0 there, so no division)
    d = np.abs(res["fsurf"] - ex["fsurf"])
    assert np.all(d <= 1e-9 * np.abs(ex["fsurf"])), d.max()
    # the refine is the same exact integer kernel in both forms
    assert np.array_equal(res["frefine"], ex["frefine"])


def test_fft_lowsnr256_f32_w64(gpu_lib):
    # 256x256 float32, w = 64, low SNR: P = Q = 320 (radices 8,8,5); 16129 shifts
    sc = synth.lowsnr256_f32()
    fr = sc.frames(0, 3)
    _say("case fft lowsnr256_f32 T=3 w=64 ds=0")
    res = _run(gpu_lib, fr, sc.template, 64, False, surface=True)
    orc = oracle.align(fr, sc.template, 64, False, want_surface=True)
    st = check(res, orc, False, exact=False, label="fft lowsnr256")
    err = check_surface(res["fsurf"], orc.surf, label="fft lowsnr256 surface")
    _say(st, "surface max rel err %.3g" % err)


FFT_SHAPES = [
    # (m, n, w, ds, dtype, T): transform lengths P x Q in the comment
    (416, 460, 32, True, "u16", 3),   # grid 208x230: 240 x 270 (radix 5 and three 3s)
    (37, 53, 5, False, "f32", 4),     # 45 x 60, odd grid sides
    (75, 41, 9, True, "u16", 4),      # grid 37x20 (odd m dropped row): 45 x 30
    (9, 9, 1, False, "u16", 3),       # w = 1: P = Q = 9 (odd transform length)
    (2, 2, 1, True, "f32", 3),        # 1x1 grid: P = 2, Q = 2
    (64, 64, 32, True, "u16", 2),     # w = m' = n': 64 x 64
    (300, 17, 8, True, "f32", 3),     # grid 150x8: 160 x 15
    (60, 220, 46, False, "f32", 2),   # 108 x 270 (2*3^3*5)
    (40, 1030, 6, True, "u16", 2),    # grid 20x515: 25 x 540
    (276, 200, 85, False, "f32", 2),  # 384 x 288 (2,3,8,8 and 3,3,4,8): 384 in place of 360
    (512, 796, 48, True, "u16", 2),   # grid 256x398: 320 x 450 (2,3,3,5,5)
    (512, 796, 32, True, "f32", 2),   # grid 256x398: 288 x 432 (2,3,3,3,8)
    (350, 350, 30, False, "u16", 2),  # 384 x 384 (2,3,8,8)
    (380, 140, 16, False, "f32", 2),  # 400 x 160 (5,5,2,8)
    (460, 100, 16, False, "u16", 2),  # 480 x 120 (3,4,5,8)
    (480, 100, 32, False, "u16", 2),  # 512 x 144: the wave-level 512 (8,8,8)
]


@pytest.mark.parametrize("case", FFT_SHAPES, ids=lambda c: "%dx%d_w%d_ds%d_%s" % c[:5])
def test_fft_shapes(gpu_lib, case):
    m, n, w, ds, dt, T = case
    rng = np.random.default_rng(m * 7919 + n)
    base = rng.uniform(0, 1, size=(m, n))
    if dt == "u16":
        tmpl = rng.poisson(300 * base + 50).astype(np.uint16)
        fr = np.stack([rng.poisson(np.roll(300 * base + 50, (k % 3 - 1, 1 - k % 2), (0, 1)))
                       for k in range(T)]).astype(np.uint16)
    else:
        tmpl = base.astype(np.float32)
        fr = np.stack([np.roll(base, (k % 3 - 1, k % 2), (0, 1)) + 0.05 * rng.standard_normal((m, n))
                       for k in range(T)]).astype(np.float32)
    _say("case fft shape", case)
    res = _run(gpu_lib, fr, tmpl, w, ds, surface=True)
    orc = oracle.align(fr, tmpl, w, ds, want_surface=True)
    check(res, orc, ds, exact=False, label=str(case))
    check_surface(res["fsurf"], orc.surf, label=str(case))


def test_fft_chunked_equals_unchunked(gpu_lib):
    # a small scratch budget forces chunks of two frames; results are identical
    sc = synth.poisson512_u16(T=40)
    fr = sc.frames(0, 7)
    big = _run(gpu_lib, fr, sc.template, 32, True, surface=True)
    ctx = gpu_lib.Context(0, scratch_budget=2 * 2 * 1024 * 1024 + 1024)
    small = _run(gpu_lib, fr, sc.template, 32, True, surface=True, ctx=ctx)
    ctx.close()
    for k in big:
        assert np.array_equal(big[k], small[k], equal_nan=True), k


def test_fft_form_resolution(gpu_lib):
    sc = synth.poisson512_u16(T=4)
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _to_dev(sc.template), 32, True)
    assert gpu_lib.resolved_form(ctx, tp, "fft") == "fft"
    assert gpu_lib.resolved_form(ctx, tp, "auto") == "int8"
    tp.close()
    ctx.close()


def test_wide_window_paper_shape_auto_picks_fft(gpu_lib):
    # the paper's 416x460 stack with its window min(m',n')/3 = 69 on the 208x230
    # grid: the FFT form is the faster one there; the int8 form (3x3 groups of
    # 64x64 shift tiles) stays exact
    sc = synth.PoissonScene(416, 460, 3, seed=7)
    fr = sc.frames(0, 3)
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _to_dev(sc.template), 69, True)
    assert gpu_lib.resolved_form(ctx, tp, "auto") == "fft_cert"
    tp.close()
    ctx.close()
    _say("case paper shape 416x460 w=69 ds=1")
    orc = oracle.align(fr, sc.template, 69, True, want_surface=True)
    res = _run(gpu_lib, fr, sc.template, 69, True, form="auto", surface=True)
    check(res, orc, True, exact=False, label="416x460 auto")
    check_surface(res["fsurf"], orc.surf, label="416x460 auto surface")
    ex = _run(gpu_lib, fr, sc.template, 69, True, form="int8", surface=True)
    check(ex, orc, True, exact=True, label="416x460 int8")
    check_surface(ex["fsurf"], orc.surf, exact=True, label="416x460 int8 surface")


# The paper's own setting (sec. 3): downsample once iff a side exceeds 256 and
# a window of a third of the searched grid's side, here w = 85 on 256x256
# grids: transform lengths 384 x 384 (the stack shapes of its timing table;
# a wave-level length in place of the 2,3,5-smooth 360).
PAPER_W85 = [(512, 512, 3, 11), (256, 256, 3, 12)]


@pytest.mark.parametrize("shape", PAPER_W85, ids=lambda c: "%dx%d" % c[:2])
def test_paper_default_window_shapes(gpu_lib, shape):
    m, n, T, seed = shape
    w, ds = gpu_lib.default_params(m, n)
    assert w == 85 and ds == (1 if m > 256 else 0)
    sc = synth.PoissonScene(m, n, T + 1, seed=seed)
    fr = sc.frames(0, T + 1)
    tm = fr[0].copy()
    fr = fr[1:]
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _to_dev(tm), w, ds)
    assert gpu_lib.resolved_form(ctx, tp, "auto") == "fft_cert"
    tp.close()
    ctx.close()
    _say("case paper shape %dx%d w=%d ds=%d" % (m, n, w, ds))
    orc = oracle.align(fr, tm, w, ds, want_surface=True)
    for form in ("auto", "fft"):
        res = _run(gpu_lib, fr, tm, w, ds, form=form, surface=True)
        st = check(res, orc, bool(ds), exact=False, label="paper %dx%d %s" % (m, n, form))
        err = check_surface(res["fsurf"], orc.surf, label="paper %dx%d %s surface" % (m, n, form))
        _say(form, st, "surface max rel err %.3g" % err)
    ex = _run(gpu_lib, fr, tm, w, ds, form="int8", surface=True)
    check(ex, orc, bool(ds), exact=True, label="paper %dx%d int8" % (m, n))
    check_surface(ex["fsurf"], orc.surf, exact=True, label="paper %dx%d int8 surface" % (m, n))
