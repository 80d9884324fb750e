"""Form choice by measurement (moco_tune) and by a recorded table
(moco_tune_set): AUTO follows the recorded form for a search key, and its
results are those of that form called explicitly.  Every test leaves the
process table empty."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _out(r):
    return {k: getattr(r, k).cpu().numpy() for k in ("shifts", "fmin", "frefine", "coarse", "gaps")}


def _same(a, b):
    for k in a:
        x, y = a[k], b[k]
        if x.dtype == np.float64:
            x, y = x.view(np.int64), y.view(np.int64)
        assert np.array_equal(x, y), k


def test_tune_picks_a_form_and_auto_follows(gpu_lib):
    sc = synth.poisson512_u16(T=2000)
    fr = torch.from_numpy(sc.frames(0, 16)).cuda()
    _say("case tune 512x512 uint16 w=32 ds=1")
    gpu_lib.tune_clear()
    ctx = gpu_lib.Context(0)
    try:
        tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), 32, True)
        chosen, times = gpu_lib.tune(ctx, tp, frames=32)
        _say("tuned", chosen, {k: "%.3g us" % (v * 1e6) for k, v in times.items()})
        assert set(times) == {"int8", "fft_cert"}
        assert all(v > 0 for v in times.values())
        assert chosen == min(times, key=times.get)
        assert gpu_lib.tune_get(512, 512, 32, 1, "u16") == chosen
        assert gpu_lib.resolved_form(ctx, tp, "auto") == chosen
        # another template of the same key follows the table too
        tp2 = gpu_lib.Template(ctx, fr[3].contiguous(), 32, True)
        assert gpu_lib.resolved_form(ctx, tp2, "auto") == chosen
        a = _out(gpu_lib.moco_align(ctx, fr, tp, form="auto"))
        b = _out(gpu_lib.moco_align(ctx, fr, tp, form=chosen))
        torch.cuda.synchronize()
        _same(a, b)
        tp2.close()
        tp.close()
    finally:
        gpu_lib.tune_clear()
        ctx.close()


def test_recorded_form_overrides_the_model(gpu_lib):
    sc = synth.poisson512_u16(T=2000)
    fr = torch.from_numpy(sc.frames(0, 8)).cuda()
    gpu_lib.tune_clear()
    ctx = gpu_lib.Context(0)
    try:
        tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), 32, True)
        assert gpu_lib.resolved_form(ctx, tp, "auto") == "int8"    # the model's choice
        gpu_lib.tune_set(512, 512, 32, 1, "u16", "fp64")
        assert gpu_lib.resolved_form(ctx, tp, "auto") == "fp64"
        a = _out(gpu_lib.moco_align(ctx, fr, tp, form="auto"))
        b = _out(gpu_lib.moco_align(ctx, fr, tp, form="fp64"))
        torch.cuda.synchronize()
        _same(a, b)
        # a recorded form that does not apply is ignored (float32: no int8 form)
        t32 = gpu_lib.Template(ctx, torch.from_numpy(sc.template.astype(np.float32)).cuda(), 32, True)
        gpu_lib.tune_set(512, 512, 32, 1, "f32", "int8")
        assert gpu_lib.resolved_form(ctx, t32, "auto") == "fft32_cert"
        gpu_lib.tune_clear()
        assert gpu_lib.resolved_form(ctx, tp, "auto") == "int8"
        t32.close()
        tp.close()
    finally:
        gpu_lib.tune_clear()
        ctx.close()


# the int8 form's two tile shapes give the same exact results: shift windows
# of one, two and five tile groups, a frame of several chunks of digits
TILE_CASES = [
    # (m, n, w, ds, T): 2w-1 = W
    (256, 256, 33, 0, 4),    # W = 65: 3x3 tiles of 32 against 2x2 groups of 2x2
    (256, 256, 64, 0, 3),    # W = 127: 4x4 against 2x2 groups
    (416, 460, 69, 1, 3),    # W = 137, grid 208x230: 5x5 against 3x3 groups
    (200, 136, 20, 0, 5),    # W = 39
]


@pytest.mark.parametrize("case", TILE_CASES, ids=lambda c: "%dx%d_w%d_ds%d" % c[:4])
def test_int8_tile_shapes_agree_with_the_oracle(gpu_lib, case):
    import oracle
    from tests._parity import check, check_surface
    m, n, w, ds, T = case
    sc = synth.PoissonScene(m, n, T + 1, seed=m + w)
    fr = sc.frames(1, T + 1)
    gpu_lib.tune_clear()
    ctx = gpu_lib.Context(0)
    try:
        tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), w, ds)
        model = gpu_lib.int8_tile(tp)
        res = {}
        for tile in (32, 64):
            gpu_lib.tune_set_tile(m, n, w, ds, "u16", tile)
            assert gpu_lib.int8_tile(tp) == tile
            r = gpu_lib.moco_align(ctx, torch.from_numpy(fr).cuda(), tp, form="int8", surface=True)
            torch.cuda.synchronize()
            res[tile] = {k: getattr(r, k).cpu().numpy() for k in
                         ("shifts", "coarse", "fmin", "frefine", "gaps", "fsurf")}
        _say("case int8 tiles", case, "model tile", model)
        for k in res[32]:
            assert np.array_equal(res[32][k], res[64][k], equal_nan=True), k
        orc = oracle.align(fr, sc.template, w, bool(ds), want_surface=True)
        check(res[32], orc, bool(ds), exact=True, label="int8 tile 32 %s" % (case,))
        check_surface(res[32]["fsurf"], orc.surf, exact=True, label="int8 tile 32 surface")
        tp.close()
    finally:
        gpu_lib.tune_clear()
        ctx.close()


HALF_CASES = [
    # (m, n, w, ds, T): 2w-1 <= 16, two 16x16 tiles on the diagonal of one MFMA
    # product against one 32x32 tile
    (256, 256, 8, 0, 5),     # W = 15
    (512, 796, 8, 1, 3),     # W = 15, grid 256x398
    (130, 262, 1, 0, 4),     # W = 1
    (200, 136, 6, 1, 70),    # W = 11, 70 frames (more than the small-launch class)
]


@pytest.mark.parametrize("case", HALF_CASES, ids=lambda c: "%dx%d_w%d_ds%d" % c[:4])
def test_int8_half_tile_agrees_with_the_single_tile_and_the_oracle(gpu_lib, case):
    import oracle
    from tests._parity import check, check_surface
    m, n, w, ds, T = case
    sc = synth.PoissonScene(m, n, T + 1, seed=m + 3 * w)
    fr = sc.frames(1, T + 1)
    gpu_lib.tune_clear()
    ctx = gpu_lib.Context(0)
    try:
        tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), w, ds)
        # the model's half tile goes with three digit products
        assert gpu_lib.int8_tile(tp) == (16 if gpu_lib.int8_products(tp) == 3 else 32)
        res = {}
        for tile in (16, 32):
            gpu_lib.tune_set_tile(m, n, w, ds, "u16", tile)
            r = gpu_lib.moco_align(ctx, torch.from_numpy(fr).cuda(), tp, form="int8", surface=True)
            torch.cuda.synchronize()
            res[tile] = {k: getattr(r, k).cpu().numpy() for k in
                         ("shifts", "coarse", "fmin", "frefine", "gaps", "fsurf")}
        _say("case int8 half tile", case)
        for k in res[16]:
            assert np.array_equal(res[16][k], res[32][k], equal_nan=True), k
        nchk = min(T, 6)
        orc = oracle.align(fr[:nchk], sc.template, w, bool(ds), want_surface=True)
        sub = {k: v[:nchk] for k, v in res[16].items()}
        check(sub, orc, bool(ds), exact=True, label="int8 half tile %s" % (case,))
        check_surface(sub["fsurf"], orc.surf, exact=True, label="int8 half tile surface")
        with pytest.raises(gpu_lib.MocoError):
            gpu_lib.tune_set_tile(256, 256, 9, 0, "u16", 16)   # 2w-1 = 17
        tp.close()
    finally:
        gpu_lib.tune_clear()
        ctx.close()


def test_tune_records_the_faster_tile(gpu_lib):
    sc = synth.PoissonScene(256, 256, 4, seed=31)
    gpu_lib.tune_clear()
    ctx = gpu_lib.Context(0)
    try:
        tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), 40, False)
        # 79 shifts a side: the model's 2x2 groups of 2x2 tiles (16 tiles)
        # against 3x3 single tiles (9), timed by the tuner
        assert gpu_lib.int8_tile(tp) == 64
        form, times = gpu_lib.tune(ctx, tp, frames=256)
        tile = gpu_lib.int8_tile(tp)
        _say("tuned", form, times, "int8 tile", tile)
        assert tile in (32, 64) and "int8" in times
        gpu_lib.tune_clear()
        assert gpu_lib.int8_tile(tp) == 64
        with pytest.raises(gpu_lib.MocoError):
            gpu_lib.tune_set_tile(256, 256, 8, 0, "u16", 64)      # 2w-1 = 15: one tile
        with pytest.raises(gpu_lib.MocoError):
            gpu_lib.tune_set_tile(256, 256, 40, 0, "u16", 16)
        with pytest.raises(gpu_lib.MocoError):
            gpu_lib.tune_set_tile(256, 256, 40, 0, "f32", 32)
        tp.close()
    finally:
        gpu_lib.tune_clear()
        ctx.close()
