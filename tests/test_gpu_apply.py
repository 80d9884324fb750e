"""The corrected stack and its mean image on the GPU (moco_apply, through the
C ABI) against the oracle's, on the same frames and shifts."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_apply_poisson512_with_found_shifts_bit_exact(gpu_lib):
    # the shifts the search finds, applied; uint16 values and exact integer sums
    sc = synth.poisson512_u16(T=2000)
    fr = sc.frames(0, 24)
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _dev(sc.template), 32, True)
    frd = _dev(fr)
    r = gpu_lib.moco_align(ctx, frd, tp)
    out, mean = gpu_lib.moco_apply(ctx, frd, r.shifts)
    torch.cuda.synchronize()
    sh = r.shifts.cpu().numpy()
    _say("case apply poisson512 T=24, shifts", sh[:4].tolist())
    o_out, o_mean = oracle.apply(fr, sh)
    assert out.dtype == torch.uint16
    assert np.array_equal(out.cpu().numpy().astype(np.float64), o_out)
    assert np.array_equal(mean.cpu().numpy(), o_mean)
    tp.close()
    ctx.close()


def test_apply_float32_planted_shifts(gpu_lib):
    sc = synth.blobs128_f32()
    fr = sc.frames(0, 100)
    sh = sc.shifts(0, 100).astype(np.int32)
    ctx = gpu_lib.Context(0)
    out, mean = gpu_lib.moco_apply(ctx, _dev(fr), _dev(sh))
    torch.cuda.synchronize()
    o_out, o_mean = oracle.apply(fr, sh)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), o_out)
    g = mean.cpu().numpy()
    assert np.all(np.abs(g - o_mean) <= 1e-13 * np.maximum(np.abs(o_mean), 1e-30) + 1e-300)
    ctx.close()


@pytest.mark.parametrize("m,n,T", [(37, 53, 5), (9, 6, 70), (1, 1, 3), (130, 257, 40),
                                   (40, 64, 30), (33, 72, 9), (7, 8, 50)])
def test_apply_ragged_shapes_and_far_shifts(gpu_lib, m, n, T):
    # rows of a multiple of 8 pixels take the 16-byte path, the others the
    # per-pixel one; shifts reach past every edge
    rng = np.random.default_rng(m * 31 + n)
    fr = rng.integers(0, 65536, size=(T, m, n)).astype(np.uint16)
    sh = np.stack([rng.integers(-m - 2, m + 3, size=T), rng.integers(-n - 2, n + 3, size=T)],
                  axis=1).astype(np.int32)
    sh[0] = (0, 0)
    _say("case apply ragged", m, n, T)
    ctx = gpu_lib.Context(0)
    out, mean = gpu_lib.moco_apply(ctx, _dev(fr), _dev(sh))
    only_mean = gpu_lib.moco_apply(ctx, _dev(fr), _dev(sh), frames_out=False)[1]
    only_out = gpu_lib.moco_apply(ctx, _dev(fr), _dev(sh), mean=False)[0]
    torch.cuda.synchronize()
    o_out, o_mean = oracle.apply(fr, sh)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), o_out)
    assert np.array_equal(only_out.cpu().numpy().astype(np.float64), o_out)
    assert np.array_equal(mean.cpu().numpy(), o_mean)
    assert np.array_equal(only_mean.cpu().numpy(), o_mean)
    ctx.close()


def test_apply_mean_chunks_bounded_by_budget(gpu_lib):
    # a budget of two planes of partial sums: the mean comes out identical
    T, m, n = 300, 64, 48
    rng = np.random.default_rng(3)
    fr = rng.integers(0, 65536, size=(T, m, n)).astype(np.uint16)
    sh = rng.integers(-5, 6, size=(T, 2)).astype(np.int32)
    ctx = gpu_lib.Context(0, scratch_budget=2 * m * n * 8)
    _, mean = gpu_lib.moco_apply(ctx, _dev(fr), _dev(sh), frames_out=False)
    torch.cuda.synchronize()
    _, o_mean = oracle.apply(fr, sh, want_frames=False)
    assert np.array_equal(mean.cpu().numpy(), o_mean)
    small = gpu_lib.Context(0, scratch_budget=m * n * 8 - 8)
    with pytest.raises(gpu_lib.MocoError) as ei:
        gpu_lib.moco_apply(small, _dev(fr), _dev(sh), frames_out=False)
    assert ei.value.code == gpu_lib.MOCO_ENOMEM
    # the corrected frames alone need no scratch
    out, _ = gpu_lib.moco_apply(small, _dev(fr), _dev(sh), mean=False)
    torch.cuda.synchronize()
    o_out, _ = oracle.apply(fr, sh)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), o_out)
    ctx.close()
    small.close()


def test_apply_validation(gpu_lib):
    ctx = gpu_lib.Context(0)
    fr = _dev(np.ones((2, 8, 8), np.uint16))
    sh = _dev(np.zeros((2, 2), np.int32))
    with pytest.raises(ValueError):
        gpu_lib.moco_apply(ctx, fr, _dev(np.zeros((3, 2), np.int32)))
    with pytest.raises(gpu_lib.MocoError) as ei:
        gpu_lib.moco_apply(ctx, fr, sh, frames_out=False, mean=False)
    assert ei.value.code == gpu_lib.MOCO_EINVAL
    # T = 0 is a no-op
    out, mean = gpu_lib.moco_apply(ctx, _dev(np.ones((0, 8, 8), np.uint16)),
                                   _dev(np.zeros((0, 2), np.int32)))
    assert out.shape == (0, 8, 8)
    ctx.close()
