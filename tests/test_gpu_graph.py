"""A moco_align call captured as a HIP graph (moco_graph_*): every replay,
with the frame buffer refilled and unrelated eager work (including a call that
grows the context's scratch) between replays, equals an eager moco_align on
the same frames bit for bit."""
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


def _host(r):
    return {k: getattr(r, k).cpu().numpy().copy() for k in KEYS}


@pytest.mark.parametrize("form,T", [("int8", 1), ("int8", 24), ("fft_cert", 5), ("fp64", 3),
                                    ("fft32_cert", 6), ("auto", 2)])
def test_graph_replays_equal_eager_calls(gpu_lib, form, T):
    sc = synth.poisson512_u16(T=2000)
    pool = torch.from_numpy(sc.frames(0, 4 * T)).cuda()
    other = torch.from_numpy(sc.frames(100, 164)).cuda()
    _say("case graph form=%s T=%d 512x512 uint16 w=32 ds=1" % (form, T))
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, torch.from_numpy(sc.template).cuda(), 32, True)
    buf = torch.empty((T, 512, 512), dtype=torch.uint16, device="cuda")
    buf.copy_(pool[:T])
    g = gpu_lib.Graph(ctx, buf, tp, form=form)
    try:
        for rep in range(4):
            buf.copy_(pool[rep * T:(rep + 1) * T])
            torch.cuda.synchronize()
            got = _host(g.launch())
            torch.cuda.synchronize()
            got = _host(g.out)
            eager = _host(gpu_lib.moco_align(ctx, buf, tp, form=form))
            torch.cuda.synchronize()
            for k in KEYS:
                a, b = got[k], eager[k]
                if a.dtype == np.float64:
                    a, b = a.view(np.int64), b.view(np.int64)
                assert np.array_equal(a, b), (rep, k)
            # eager work between replays; a larger stack grows the context's scratch
            gpu_lib.moco_align(ctx, other[: 16 * (rep + 1)], tp)
            torch.cuda.synchronize()
    finally:
        g.close()
        tp.close()
        ctx.close()


def test_graph_rejects_an_empty_stack(gpu_lib):
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, torch.ones((32, 32), dtype=torch.uint16).cuda(), 4, False)
    with pytest.raises(gpu_lib.MocoError) as ei:
        gpu_lib.Graph(ctx, torch.ones((0, 32, 32), dtype=torch.uint16).cuda(), tp)
    assert ei.value.code == gpu_lib.MOCO_EINVAL
    tp.close()
    ctx.close()


def test_batch_graph_replays_equal_eager_batches(gpu_lib):
    # uneven stacks through four forms (int8 with both tile shapes, the
    # certified FP32 and FP64 FFT forms) captured as one graph
    specs = [(synth.poisson512_u16(T=40), 32, True, 6),
             (synth.PoissonScene(256, 256, 40, seed=3), 16, False, 5),
             (synth.blobs128_f32(seed=4), 10, False, 4),
             (synth.PoissonScene(416, 460, 40, seed=5), 69, True, 3)]
    ctx = gpu_lib.Context(0)
    items, pools, tps = [], [], []
    for sc, w, ds, T in specs:
        pool = torch.from_numpy(sc.frames(0, 4 * T)).cuda()
        tp = gpu_lib.Template(ctx, torch.from_numpy(np.ascontiguousarray(sc.template)).cuda(), w, ds)
        buf = torch.empty_like(pool[:T])
        buf.copy_(pool[:T])
        items.append((buf, tp))
        pools.append(pool)
        tps.append(tp)
    forms = [gpu_lib.resolved_form(ctx, tp, "auto") for tp in tps]
    _say("case batch graph, forms", forms)
    assert "fft32_cert" in forms and "int8" in forms
    other = torch.from_numpy(synth.poisson512_u16(T=300).frames(100, 164)).cuda()
    g = gpu_lib.BatchGraph(ctx, items)
    try:
        for rep in range(4):
            for (buf, _), pool in zip(items, pools):
                T = buf.shape[0]
                buf.copy_(pool[rep * T:(rep + 1) * T])
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            got = [_host(r) for r in g.results]
            eager = [_host(r) for r in gpu_lib.moco_align_batch(ctx, items)]
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(got, eager)):
                for key in KEYS:
                    x, y = a[key], b[key]
                    if x.dtype == np.float64:
                        x, y = x.view(np.int64), y.view(np.int64)
                    assert np.array_equal(x, y), (rep, k, key)
            # eager work between replays; a larger stack grows the context's scratch
            gpu_lib.moco_align(ctx, other[: 16 * (rep + 1)], tps[0])
            torch.cuda.synchronize()
    finally:
        g.close()
        for tp in tps:
            tp.close()
        ctx.close()


def test_batch_graph_rejects_a_batch_without_frames(gpu_lib):
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, torch.ones((32, 32), dtype=torch.uint16).cuda(), 4, False)
    with pytest.raises(gpu_lib.MocoError) as ei:
        gpu_lib.BatchGraph(ctx, [(torch.ones((0, 32, 32), dtype=torch.uint16).cuda(), tp)])
    assert ei.value.code == gpu_lib.MOCO_EINVAL
    tp.close()
    ctx.close()
