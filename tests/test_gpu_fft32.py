"""Parity of the plain single-precision form (MOCO_FORM_FFT32: FP32 complex
transforms of the grids less a common offset, sec. 2's FFT construction of h,
with FP64 overlap energies and combine) with the FP64 oracle, on the GPU,
through the C ABI.

This form is not certified: its f error is that of FP32 transforms, which the
common offset keeps near 1e-6 relative at the minimum of the 512x512 uint16
stack and near 1e-5 on the high-SNR 128x128 float32 stack (kappa ~ 350 before
centring).  It is held here to F32_RTOL = 2e-5 relative (twice the search's
1e-5 bar, which the form misses on that stack by a few per cent; the
benchmark reports each config's error), and to bit-exact shifts on every
frame whose oracle gaps are clear.  The cases include grids whose width is not
a multiple of the prep kernel's 128-column strips (padding columns must stay
out of the centred energies) and a two-level search (energies of the centred
FP64 grid).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._parity import check, check_surface

pytestmark = pytest.mark.gpu

F32_RTOL = 2e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(moco, frames, tmpl, w, ds, form="fft32", surface=True, ctx=None):
    own = ctx is None
    if own:
        ctx = moco.Context(0)
    tp = moco.Template(ctx, _to_dev(tmpl), w, ds)
    r = moco.moco_align(ctx, _to_dev(frames), tp, form=form, surface=surface)
    torch.cuda.synchronize()
    out = {k: getattr(r, k).cpu().numpy()
           for k in ("shifts", "fmin", "frefine", "coarse", "gaps", "recomputed")}
    if surface:
        out["fsurf"] = r.fsurf.cpu().numpy()
    tp.close()
    if own:
        ctx.close()
    return out


def _against_oracle(moco, fr, tm, w, ds, label):
    _say("case fft32", label, fr.shape, "w=%d ds=%d" % (w, ds))
    res = _run(moco, fr, tm, w, ds)
    orc = oracle.align(fr, tm, w, ds, want_surface=True)
    st = check(res, orc, bool(ds), exact=False, rtol=F32_RTOL, label=label)
    err = check_surface(res["fsurf"], orc.surf, rtol=F32_RTOL, label=label + " surface")
    assert not res["recomputed"].any()
    _say(st, "surface max rel err %.3g" % err)
    return res, err


def test_fft32_blobs128_f32(gpu_lib):
    sc = synth.blobs128_f32()
    fr = sc.frames(0, 100)
    res, _ = _against_oracle(gpu_lib, fr, sc.template, 10, 0, "blobs128")
    assert np.array_equal(res["shifts"], sc.shifts(0, 100))


# (Frame 0 of the Poisson stacks is the template itself, f = 0 at its shift:
# single precision cannot meet the rule's floor there, 1e-9 of the energies,
# so these cases start at frame 1.)


def test_fft32_poisson512_u16_ds(gpu_lib):
    sc = synth.poisson512_u16(T=2000)
    fr = sc.frames(1, 25)
    res, err = _against_oracle(gpu_lib, fr, sc.template, 32, 1, "poisson512")
    assert err < 1e-5
    ex = _run(gpu_lib, fr, sc.template, 32, 1, form="int8", surface=False)
    assert np.array_equal(res["shifts"], ex["shifts"])
    # the refine is the exact integer kernel in every form
    assert np.array_equal(res["frefine"][np.all(res["coarse"] == ex["coarse"], axis=1)],
                          ex["frefine"][np.all(res["coarse"] == ex["coarse"], axis=1)])


def test_fft32_lowsnr256_f32_w64(gpu_lib):
    sc = synth.lowsnr256_f32()
    _against_oracle(gpu_lib, sc.frames(0, 4), sc.template, 64, 0, "lowsnr256")


def test_fft32_paper_416x460_w69(gpu_lib):
    # grid 208x230: 230 columns pad to two 128-column strips in the prep kernel
    sc = synth.PoissonScene(416, 460, 4, seed=7)
    fr = sc.frames(0, 4)
    _against_oracle(gpu_lib, fr[1:], fr[0], 69, 1, "416x460")


def test_fft32_two_levels(gpu_lib):
    # two 2x2 levels: the FP64 grid of level 2, energies of the centred grid
    sc = synth.poisson512_u16(T=40)
    fr = sc.frames(1, 7)
    _against_oracle(gpu_lib, fr, sc.template, 16, 2, "poisson512 L2")


FFT32_SHAPES = [
    # (m, n, w, ds, dtype, T)
    (37, 53, 5, 0, "f32", 4),       # odd sides, float32
    (75, 41, 9, 1, "u16", 4),       # grid 37x20, odd m dropped
    (130, 262, 40, 0, "u16", 2),    # 262 columns: one partial prep strip, no downsampling
    (300, 17, 8, 1, "f32", 3),      # tall and narrow
    (9, 9, 1, 0, "u16", 3),         # w = 1
]


@pytest.mark.parametrize("case", FFT32_SHAPES, ids=lambda c: "%dx%d_w%d_ds%d_%s" % c[:5])
def test_fft32_shapes(gpu_lib, case):
    m, n, w, ds, dt, T = case
    rng = np.random.default_rng(m * 7919 + n + 3)
    base = rng.uniform(0, 1, size=(m, n))
    if dt == "u16":
        tmpl = rng.poisson(300 * base + 50).astype(np.uint16)
        fr = np.stack([rng.poisson(np.roll(300 * base + 50, (k % 3 - 1, 1 - k % 2), (0, 1)))
                       for k in range(T)]).astype(np.uint16)
    else:
        tmpl = base.astype(np.float32)
        fr = np.stack([np.roll(base, (k % 3 - 1, k % 2), (0, 1)) + 0.05 * rng.standard_normal((m, n))
                       for k in range(T)]).astype(np.float32)
    _against_oracle(gpu_lib, fr, tmpl, w, ds, str(case))


def test_fft32_chunked_equals_unchunked(gpu_lib):
    sc = synth.poisson512_u16(T=40)
    fr = sc.frames(0, 7)
    big = _run(gpu_lib, fr, sc.template, 32, 1)
    ctx = gpu_lib.Context(0, scratch_budget=2 * 1024 * 1024 + 1024)
    small = _run(gpu_lib, fr, sc.template, 32, 1, ctx=ctx)
    ctx.close()
    for k in big:
        assert np.array_equal(big[k], small[k], equal_nan=True), k


def test_fft32_never_chosen_by_auto(gpu_lib):
    for args in ((synth.poisson512_u16(T=2).template, 32, 1),
                 (synth.lowsnr256_f32().template, 64, 0)):
        ctx = gpu_lib.Context(0)
        tp = gpu_lib.Template(ctx, _to_dev(args[0]), args[1], args[2])
        assert gpu_lib.resolved_form(ctx, tp, "fft32") == "fft32"
        assert gpu_lib.resolved_form(ctx, tp, "auto") != "fft32"
        tp.close()
        ctx.close()
