"""Parity at the workloads' full sizes, in the launch configuration the benchmark
times (whole stacks per call, the benchmark's scratch budget, AUTO form), on
sampled frames the oracle computes one by one.

* 2000 frames of 512x512 uint16 (2x downsample, w = 32): the int8 form; sampled
  frames bit-identical to the oracle (shifts, f, the nine refine values, gaps).
* 10000 frames of 256x256 float32 at low SNR (w = 64): the certified FFT form;
  64 sampled frames: shifts equal to the oracle's where the certificate held
  (and to the FP64 form's where it did not), f within the 1e-5 bar.
* the 64-stack mixed batch (128x128 .. 512x796, 50-3000 frames, w from
  {8, 16, 32, 48}), each stack's first frames repeated to its length as in the
  benchmark: one moco_align_batch call; every frame's results equal those of
  the frame it repeats, and the first two frames of every stack agree with the
  oracle.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._parity import check

pytestmark = pytest.mark.gpu

BUDGET = 16 << 30


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host(r, idx=None):
    out = {k: getattr(r, k).cpu().numpy() for k in ("shifts", "fmin", "frefine", "coarse", "gaps")}
    if r.recomputed is not None:
        out["recomputed"] = r.recomputed.cpu().numpy()
    if idx is not None:
        out = {k: v[idx] for k, v in out.items()}
    return out


def test_full_stack_512_uint16_sampled(gpu_lib):
    T = 2000
    sc = synth.poisson512_u16(T=T)
    fr = sc.frames(0, T, workers=synth.default_workers())
    _say("case full stack 2000 x 512x512 uint16 w=32 ds=1 (AUTO)")
    ctx = gpu_lib.Context(0, scratch_budget=BUDGET)
    tp = gpu_lib.Template(ctx, torch.from_numpy(fr[0].copy()).cuda(), 32, True)
    assert gpu_lib.resolved_form(ctx, tp, "auto") == "int8"
    r = gpu_lib.moco_align(ctx, torch.from_numpy(fr).cuda(), tp)
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([np.linspace(0, T - 1, 14).astype(int), [1, 999, 1000]]))
    got = _host(r, idx)
    orc = oracle.align(fr[idx], fr[0], 32, True)
    st = check(got, orc, True, exact=True, label="full 2000x512^2")
    # f bit-identical on every sampled frame, the shifts too
    assert np.array_equal(got["shifts"], orc.shifts)
    assert np.array_equal(got["fmin"], orc.fmin)
    assert np.array_equal(got["frefine"], orc.frefine)
    _say("sampled frames", idx.tolist(), st)
    tp.close()
    ctx.close()


def test_full_stack_256_float32_w64_sampled(gpu_lib):
    T = 10000
    sc = synth.lowsnr256_f32()
    fr = sc.frames(0, T)
    _say("case full stack 10000 x 256x256 float32 w=64 (AUTO)")
    ctx = gpu_lib.Context(0, scratch_budget=BUDGET)
    tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), 64, False)
    assert gpu_lib.resolved_form(ctx, tp, "auto") == "fft32_cert"
    r = gpu_lib.moco_align(ctx, torch.from_numpy(fr).cuda(), tp)
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([np.linspace(0, T - 1, 62).astype(int), [1, 5000]]))
    assert idx.size >= 64
    got = _host(r, idx)
    orc = oracle.align(fr[idx], sc.template, 64, False)
    st = check(got, orc, False, exact=False, label="full 10000x256^2 f32")
    # certified by the FP32 bound (0) or the FP64 one (1): the exact shift;
    # direct sums (2): the FP64 form's
    rec = got["recomputed"] == 2
    assert np.array_equal(got["shifts"][~rec], orc.shifts[~rec])
    if rec.any():
        direct = _host(gpu_lib.moco_align(ctx, torch.from_numpy(fr[idx]).cuda(), tp, form="fp64"))
        assert np.array_equal(got["shifts"][rec], direct["shifts"][rec])
    rel = np.abs(got["fmin"] - orc.fmin) / np.abs(orc.fmin)
    assert rel.max() <= 1e-5
    _say("sampled frames", idx.tolist(), st, "recomputed", int(rec.sum()),
         "max f rel err %.3g" % rel.max())
    tp.close()
    ctx.close()


def test_full_mixed_batch_repeated_frames(gpu_lib):
    unique = 8
    specs = synth.mixed_stacks(64)
    ctx = gpu_lib.Context(0, scratch_budget=BUDGET)
    items, data, total = [], [], 0
    for sp in specs:
        sc, T = sp["scene"], sp["T"]
        u = min(unique, T)
        uniq = sc.frames(0, u)
        dev = torch.from_numpy(uniq).cuda()
        fr = torch.empty((T, sp["m"], sp["n"]), dtype=dev.dtype, device=dev.device)
        for k in range(0, T, u):
            fr[k:k + u] = dev[:min(u, T - k)]
        tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), sp["w"], sp["downsample"])
        items.append((fr, tp))
        data.append((uniq, sc.template, sp))
        total += T
    _say("case full mixed batch: 64 stacks, %d frames" % total)
    res = gpu_lib.moco_align_batch(ctx, items, form="auto")
    torch.cuda.synchronize()
    for (fr, tp), r, (uniq, tm, sp) in zip(items, res, data):
        T, u = sp["T"], uniq.shape[0]
        got = _host(r)
        src = np.arange(T) % u
        for k in ("shifts", "coarse", "fmin", "frefine", "gaps"):
            a = got[k]
            b = a[src]
            if a.dtype == np.float64:
                a, b = a.view(np.int64), b.view(np.int64)
            assert np.array_equal(a, b), (k, sp["m"], sp["n"], sp["w"], T)
        orc = oracle.align(uniq[:2], tm, sp["w"], sp["downsample"])
        form = gpu_lib.resolved_form(ctx, tp, "auto")
        # frame 0 is the template (f = 0 at its shift): the rule's floor
        # 1e-9 (A+B)/Area, with (A+B)/Area about twice the grid's mean square
        g = tm.astype(np.float64)
        if sp["downsample"]:
            g = g[:g.shape[0] // 2 * 2, :g.shape[1] // 2 * 2]
            g = (g[0::2, 0::2] + g[0::2, 1::2] + g[1::2, 0::2] + g[1::2, 1::2]) / 4
        check({k: v[:2] for k, v in got.items()}, orc, sp["downsample"],
              exact=form not in ("fft", "fft_cert", "fft32_cert"), f_floor=1e-9 * 2 * float(np.mean(g * g)),
              label="batch %dx%d w%d T=%d %s" % (sp["m"], sp["n"], sp["w"], T, form))
    for _, tp in items:
        tp.close()
    del items
    torch.cuda.empty_cache()
    ctx.close()
