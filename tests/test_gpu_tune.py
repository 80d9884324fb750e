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
