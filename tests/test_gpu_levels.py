"""Several levels of downsampling on the GPU (sec. 2, last paragraph: the
argmin multiplied by two multiple times, nine evaluations per level) against
the oracle, through the C ABI."""
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(moco, frames, tmpl, w, ds, form="auto", surface=False):
    ctx = moco.Context(0)
    tp = moco.Template(ctx, _dev(tmpl), w, ds)
    r = moco.moco_align(ctx, _dev(frames), tp, form=form, surface=surface)
    torch.cuda.synchronize()
    out = {k: getattr(r, k).cpu().numpy() for k in ("shifts", "fmin", "frefine", "coarse", "gaps")}
    if surface:
        out["fsurf"] = r.fsurf.cpu().numpy()
    resolved = moco.resolved_form(ctx, tp, form)
    tp.close()
    ctx.close()
    return out, resolved


@pytest.mark.parametrize("form", ["fp64", "fft"])
def test_two_levels_poisson512(gpu_lib, form):
    # 512x512 uint16 -> 128x128 searched grid, w = 16; the FP64 form stays exact
    # (every level's values are multiples of 4^-l)
    sc = synth.poisson512_u16(T=2000)
    fr = sc.frames(0, 8)
    _say("case two levels poisson512 T=8 w=16 form=%s" % form)
    res, used = _run(gpu_lib, fr, sc.template, 16, 2, form=form, surface=True)
    assert used == form
    orc = oracle.align(fr, sc.template, 16, 2, want_surface=True)
    exact = form == "fp64"
    st = check(res, orc, True, exact=exact, label="2 levels %s" % form)
    check_surface(res["fsurf"], orc.surf, exact=exact, label="2 levels %s surface" % form)
    _say(st)


def test_auto_with_two_levels_is_not_int8(gpu_lib):
    sc = synth.poisson512_u16(T=4)
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _dev(sc.template), 16, 2)
    assert gpu_lib.resolved_form(ctx, tp, "auto") == "fft_cert"
    with pytest.raises(gpu_lib.MocoError) as ei:
        gpu_lib.moco_align(ctx, _dev(sc.frames(0, 2)), tp, form="int8")
    assert ei.value.code == gpu_lib.MOCO_EINVAL
    tp.close()
    ctx.close()


@pytest.mark.parametrize("levels", [3, 4])
def test_planted_shifts_through_three_and_four_levels(gpu_lib, levels):
    rng = np.random.default_rng(40 + levels)
    m = n = 256
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    b = np.full((m, n), 20.0)
    for _ in range(40):
        ci, cj, sg = rng.uniform(0, m), rng.uniform(0, n), rng.uniform(4, 9)
        b += rng.uniform(50, 200) * np.exp(-((i - ci) ** 2 + (j - cj) ** 2) / (2 * sg * sg))
    b = np.rint(b).astype(np.uint16)
    shifts = [(0, 0), (13, -21), (-17, 9), (22, 15), (-9, -30)]
    fr = np.stack([np.roll(b, s, axis=(0, 1)) for s in shifts])
    w = (m >> levels) // 3 + 1
    _say("case %d levels planted shifts w=%d" % (levels, w))
    res, used = _run(gpu_lib, fr, b, w, levels)
    orc = oracle.align(fr, b, w, levels)
    # frame 0 is the template: f = 0 there, held to the rule's floor
    floor = 1e-9 * 2.0 * float(np.mean(b.astype(np.float64) ** 2))
    check(res, orc, True, exact=False, label="%d levels" % levels, f_floor=floor)
    assert [tuple(x) for x in res["shifts"]] == shifts


@pytest.mark.parametrize("case", [(70, 90, 4, 2, "f32", 3), (131, 67, 3, 2, "u16", 4),
                                  (200, 160, 6, 3, "u16", 2)],
                         ids=lambda c: "%dx%d_w%d_L%d_%s" % c[:5])
def test_levels_ragged(gpu_lib, case):
    m, n, w, L, dt, T = case
    rng = np.random.default_rng(m * 13 + n)
    base = rng.uniform(0, 1, size=(m, n))
    if dt == "u16":
        tmpl = rng.poisson(300 * base + 50).astype(np.uint16)
        fr = np.stack([rng.poisson(np.roll(300 * base + 50, (2 * k - 3, 5 - k), (0, 1)))
                       for k in range(T)]).astype(np.uint16)
    else:
        tmpl = base.astype(np.float32)
        fr = np.stack([np.roll(base, (k - 1, 2 * k), (0, 1)) + 0.05 * rng.standard_normal((m, n))
                       for k in range(T)]).astype(np.float32)
    _say("case levels ragged", case)
    for form in ("fp64", "fft"):
        res, _ = _run(gpu_lib, fr, tmpl, w, L, form=form, surface=True)
        orc = oracle.align(fr, tmpl, w, L, want_surface=True)
        exact = form == "fp64" and dt == "u16"
        check(res, orc, True, exact=exact, label="%s %s" % (case, form))
        check_surface(res["fsurf"], orc.surf, exact=exact, label="%s %s surface" % (case, form))


def test_default_params_binding(gpu_lib):
    assert gpu_lib.default_params(512, 512) == (85, 1)
    assert gpu_lib.default_params(256, 256) == (85, 0)
