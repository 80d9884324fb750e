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
