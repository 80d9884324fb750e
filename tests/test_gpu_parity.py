"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Inputs come from the seeded generators in ``synth``; expected values come from
``oracle`` on the same inputs.  See ``tests/_parity.py`` for the rule.
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


def _run(moco, frames, tmpl, w, ds, form="auto", surface=False, ctx=None):
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


def test_blobs128_f32_all_frames(gpu_lib):
    sc = synth.blobs128_f32()
    fr = sc.frames(0, 100)
    _say("case blobs128_f32 T=100 w=10 ds=0 form=fp64")
    res = _run(gpu_lib, fr, sc.template, 10, False, "fp64", surface=True)
    orc = oracle.align(fr, sc.template, 10, False, want_surface=True)
    st = check(res, orc, False, exact=False, label="blobs128")
    check_surface(res["fsurf"], orc.surf, label="blobs128 surface")
    # planted shifts are recovered (high SNR)
    assert np.array_equal(res["shifts"], sc.shifts(0, 100))
    _say(st)


def test_poisson512_u16_ds_first_frames_bit_exact(gpu_lib):
    sc = synth.poisson512_u16(T=2000)
    T = 24
    fr = sc.frames(0, T)
    _say("case poisson512_u16 T=%d w=32 ds=1 form=fp64" % T)
    res = _run(gpu_lib, fr, sc.template, 32, True, "fp64", surface=True)
    orc = oracle.align(fr, sc.template, 32, True, want_surface=True)
    st = check(res, orc, True, exact=True, label="poisson512")
    check_surface(res["fsurf"], orc.surf, exact=True, label="poisson512 surface")
    _say(st)


RAGGED = [
    # (m, n, w, ds, dtype, T)
    (37, 53, 5, False, "f32", 5),
    (75, 41, 9, True, "u16", 5),
    (64, 64, 32, True, "u16", 3),     # largest window: w = m' = n'
    (9, 9, 1, False, "u16", 4),       # single shift: plain mean squared error
    (300, 17, 8, True, "f32", 3),     # tall, odd n, n' = 8 = w
    (130, 262, 40, False, "u16", 2),  # several LDS row tiles, ragged tail
    (2, 2, 1, True, "f32", 3),        # smallest downsampled image
]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: "%dx%d_w%d_ds%d_%s" % c[:5])
def test_ragged_shapes(gpu_lib, case):
    m, n, w, ds, dt, T = case
    rng = np.random.default_rng(m * 1000 + n)
    base = rng.uniform(0, 1, size=(m, n))
    if dt == "u16":
        tmpl = rng.poisson(300 * base + 50).astype(np.uint16)
        fr = np.stack([rng.poisson(np.roll(300 * base + 50, (k % 3 - 1, 1 - k % 2), (0, 1)))
                       for k in range(T)]).astype(np.uint16)
    else:
        tmpl = base.astype(np.float32)
        fr = np.stack([np.roll(base, (k % 3 - 1, k % 2), (0, 1)) + 0.05 * rng.standard_normal((m, n))
                       for k in range(T)]).astype(np.float32)
    _say("case ragged", case)
    res = _run(gpu_lib, fr, tmpl, w, ds, "fp64", surface=True)
    orc = oracle.align(fr, tmpl, w, ds, want_surface=True)
    check(res, orc, ds, exact=(dt == "u16"), label=str(case))
    check_surface(res["fsurf"], orc.surf, exact=(dt == "u16"), label=str(case))


def test_empty_stack_is_noop(gpu_lib):
    ctx = gpu_lib.Context(0)
    tmpl = _to_dev(np.ones((16, 16), np.float32))
    tp = gpu_lib.Template(ctx, tmpl, 4, False)
    fr = torch.empty((0, 16, 16), dtype=torch.float32, device="cuda")
    r = gpu_lib.moco_align(ctx, fr, tp)
    torch.cuda.synchronize()
    assert r.shifts.shape == (0, 2)


def test_validation_errors(gpu_lib):
    ctx = gpu_lib.Context(0)
    t16 = _to_dev(np.ones((16, 16), np.uint16))
    for w, ds in [(0, False), (17, False), (9, True)]:
        with pytest.raises(gpu_lib.MocoError) as ei:
            gpu_lib.Template(ctx, t16, w, ds)
        assert ei.value.code == gpu_lib.MOCO_EINVAL
    tp = gpu_lib.Template(ctx, t16, 4, True)
    fr = _to_dev(np.ones((2, 16, 16), np.float32))
    with pytest.raises(gpu_lib.MocoError) as ei:   # dtype differs from the template's
        gpu_lib.moco_align(ctx, fr, tp)
    assert ei.value.code == gpu_lib.MOCO_EINVAL
    fr = _to_dev(np.ones((2, 18, 16), np.uint16))
    with pytest.raises(gpu_lib.MocoError):         # size differs from the template's
        gpu_lib.moco_align(ctx, fr, tp)


def test_scratch_budget_too_small(gpu_lib):
    ctx = gpu_lib.Context(0, scratch_budget=4096)
    tp = gpu_lib.Template(ctx, _to_dev(np.ones((64, 64), np.uint16)), 8, False)
    with pytest.raises(gpu_lib.MocoError) as ei:
        gpu_lib.moco_align(ctx, _to_dev(np.ones((3, 64, 64), np.uint16)), tp)
    assert ei.value.code == gpu_lib.MOCO_ENOMEM


def test_chunked_equals_unchunked(gpu_lib):
    # a small scratch budget forces several chunks; results must be identical
    sc = synth.poisson512_u16(T=40)
    fr = sc.frames(0, 12)
    big = _run(gpu_lib, fr, sc.template, 32, True, "fp64")
    ctx = gpu_lib.Context(0, scratch_budget=3 * 1200 * 1024)
    small = _run(gpu_lib, fr, sc.template, 32, True, "fp64", ctx=ctx)
    for k in big:
        assert np.array_equal(big[k], small[k], equal_nan=True), k


def test_deterministic_repeat(gpu_lib):
    sc = synth.blobs128_f32(seed=3)
    fr = sc.frames(0, 16)
    a = _run(gpu_lib, fr, sc.template, 10, False, "fp64", surface=True)
    b = _run(gpu_lib, fr, sc.template, 10, False, "fp64", surface=True)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
