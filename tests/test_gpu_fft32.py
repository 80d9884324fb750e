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
    (512, 796, 48, 1, "u16", 2),    # 320 x 450
    (350, 350, 30, 0, "f32", 2),    # 384 x 384
    (460, 100, 16, 0, "f32", 2),    # 480 x 120
    (470, 80, 16, 0, "f32", 2),     # 512 (in place of the smooth 486) x 96
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
    # the plain form never; the certified one for float32 data
    for args, auto in (((synth.poisson512_u16(T=2).template, 32, 1), "int8"),
                       ((synth.lowsnr256_f32().template, 64, 0), "fft32_cert")):
        ctx = gpu_lib.Context(0)
        tp = gpu_lib.Template(ctx, _to_dev(args[0]), args[1], args[2])
        assert gpu_lib.resolved_form(ctx, tp, "fft32") == "fft32"
        assert gpu_lib.resolved_form(ctx, tp, "auto") == auto
        tp.close()
        ctx.close()


# ---- the certified single-precision form ----------------------------------
# An argmin certified by the FP32 bound is exact, and its f is then evaluated
# by its definition in FP64 (bit-exact on uint16); on uint16 frames with at
# most one 2x2 level, an uncertified frame whose open shifts all neighbour the
# computed argmin is settled by exact sums over those nine shifts
# (recomputed 3); the other frames left uncertified go through the certified
# FP64 form and equal its results.  So f at the argmin meets the search's
# 1e-5 bar on every frame; the rest of the surface keeps the FP32 correlation
# (held to F32_RTOL).


def _cert32(moco, fr, tm, w, ds, label, aba=None):
    """aba: (A+B)/Area scale for the rule's floor on noise-free frames."""
    f_floor = 1e-12 if aba is None else 1e-9 * aba
    res = _run(moco, fr, tm, w, ds, form="fft32_cert")
    ref = _run(moco, fr, tm, w, ds, form="fft_cert")
    orc = oracle.align(fr, tm, w, ds, want_surface=True)
    rec = res["recomputed"]
    assert set(np.unique(rec).tolist()) <= {0, 1, 2, 3}, label
    st = check(res, orc, bool(ds), exact=False, label=label, f_floor=f_floor)
    # an argmin certified by either bound, or settled from its candidates, is
    # the exact argmin of the grid
    cert = rec != 2
    assert np.array_equal(res["coarse"][cert], orc.coarse[cert]), label
    # frames the FP32 bound left to the FP64 form: its results, bit for bit
    re = (rec == 1) | (rec == 2)
    for k in ("shifts", "coarse", "fmin", "frefine", "gaps", "fsurf"):
        assert np.array_equal(res[k][re], ref[k][re], equal_nan=True), (label, k)
    assert np.array_equal(ref["recomputed"][re], (rec[re] == 2).astype(np.int32)), label
    # frames settled from their candidates (uint16 only): exact f at the
    # exact argmin, and the same refine as the FP64 form
    r3 = rec == 3
    if r3.any():
        assert not np.issubdtype(fr.dtype, np.floating), label
        assert np.array_equal(res["fmin"][r3], orc.fmin[r3]), label
        for k in ("shifts", "coarse", "fmin", "frefine"):
            assert np.array_equal(res[k][r3], ref[k][r3], equal_nan=True), (label, k)
    # the FP32 surfaces (the others were compared with the FP64 form's above)
    ok = (rec == 0) | r3
    err = check_surface(res["fsurf"][ok], orc.surf[ok], A_plus_B_over_area=aba, rtol=F32_RTOL,
                        label=label + " surface") if ok.any() else 0.0
    _say(label, st, "recomputed", np.bincount(rec, minlength=4).tolist(),
         "surface max rel err %.3g" % err)
    return res, orc


def test_fft32_cert_lowsnr256_f32_w64(gpu_lib):
    sc = synth.lowsnr256_f32()
    res, orc = _cert32(gpu_lib, sc.frames(0, 8), sc.template, 64, 0, "cert32 lowsnr256")
    assert (res["recomputed"] == 0).mean() >= 0.75


def test_fft32_cert_blobs128_meets_the_bar(gpu_lib):
    # the high-SNR stack where the plain FP32 form's f misses 1e-5 (kappa ~350)
    sc = synth.blobs128_f32()
    fr = sc.frames(0, 100)
    res, orc = _cert32(gpu_lib, fr, sc.template, 10, 0, "cert32 blobs128")
    assert np.array_equal(res["shifts"], sc.shifts(0, 100))
    ok = res["recomputed"] == 0
    assert ok.mean() >= 0.75
    rel = np.abs(res["fmin"][ok] - orc.fmin[ok]) / orc.fmin[ok]
    assert rel.max() < 1e-12, rel.max()


def test_fft32_cert_poisson512_u16_ds(gpu_lib):
    # gaps of a few per cent of f: some frames certified, the others settled
    # from the candidates the bound leaves (all neighbours of the argmin here)
    sc = synth.poisson512_u16(T=2000)
    fr = sc.frames(1, 25)
    res, orc = _cert32(gpu_lib, fr, sc.template, 32, 1, "cert32 poisson512")
    rec = res["recomputed"]
    assert (rec == 3).any() and not ((rec == 1) | (rec == 2)).any()
    ok = (rec == 0) | (rec == 3)
    # the definition's f is exact on uint16 grids (multiples of 1/16)
    assert np.array_equal(res["fmin"][ok], orc.fmin[ok])
    ex = _run(gpu_lib, fr, sc.template, 32, 1, form="int8", surface=False)
    assert np.array_equal(res["shifts"], ex["shifts"])


def test_fft32_cert_exact_ties_are_recomputed(gpu_lib):
    # rows of period two and exact rolls: many shifts tie exactly
    tmpl, fr, _ = synth.row_periodic(96, 100, 12, "f32", max_shift=4, noisy_every=3, seed=3)
    # noise-free frames have f = 0 at their shift: the rule's floor, 1e-9 of
    # (A+B)/Area, about twice the grid's mean square
    aba = 2 * float(np.mean(tmpl.astype(np.float64) ** 2))
    res, orc = _cert32(gpu_lib, fr, tmpl, 6, 0, "cert32 ties", aba=aba)
    tie = orc.gap_c == 0
    assert tie.any()
    assert np.all(res["recomputed"][tie] == 2)


def test_fft32_cert_chunked_equals_unchunked(gpu_lib):
    sc = synth.poisson512_u16(T=40)
    fr = sc.frames(1, 9)
    big = _run(gpu_lib, fr, sc.template, 32, 1, form="fft32_cert")
    ctx = gpu_lib.Context(0, scratch_budget=3 * 1024 * 1024)
    small = _run(gpu_lib, fr, sc.template, 32, 1, form="fft32_cert", ctx=ctx)
    ctx.close()
    for k in big:
        assert np.array_equal(big[k], small[k], equal_nan=True), k


def _centred_bound_terms(fr_grid, t_grid, c, P, Q):
    """Norms of the centred grids and the largest magnitudes of their
    zero-padded spectra (numpy FFT in FP64)."""
    x, y = fr_grid - c, t_grid - c
    X = np.abs(np.fft.rfft2(x, (P, Q))).max()
    Y = np.abs(np.fft.rfft2(y, (P, Q))).max()
    return np.sqrt((x * x).sum()), np.sqrt((y * y).sum()), X, Y


def _plan_eps(n, u):
    c = {2: 1, 4: 2, 8: 6, 3: 10, 5: 18}
    e = 0.0
    for r in (8, 4, 2, 3, 5):
        while n % r == 0:
            n //= r
            e += (5 + c[r]) * u
    assert n == 1
    return e


def test_fft32_error_within_the_certificate_bound(gpu_lib):
    # the plain FP32 surface against the oracle: on every shift, the observed
    # error of Area*f is within 2 hb, the certificate's bound on 2|h^ - h|
    u = 2.0 ** -24
    for sc, w, T in ((synth.blobs128_f32(), 10, 6), (synth.lowsnr256_f32(), 64, 3)):
        fr = sc.frames(0, T)
        tm = sc.template.astype(np.float64)
        m, n = tm.shape
        P = next(k for k in range(m + w - 1, 4 * m) if _smooth(k))
        Q = next(k for k in range(n + w - 1, 4 * n) if _smooth(k))
        eps = _plan_eps(P, u) + _plan_eps(Q, u) + 2 * u
        e1, e2 = eps + u, eps + 7 * u
        res = _run(gpu_lib, fr, sc.template, w, 0, form="fft32")
        orc = oracle.align(fr, sc.template, w, False, want_surface=True)
        c = tm.mean()
        W = 2 * w - 1
        s = np.arange(W) - (w - 1)
        area = np.outer(m - np.abs(s), n - np.abs(s)).astype(np.float64)
        worst = 0.0
        for k in range(T):
            na, nb, X, Y = _centred_bound_terms(fr[k].astype(np.float64), tm, c, P, Q)
            hb = 2 * (e1 * na * Y + e2 * (X + e1 * np.sqrt(P * Q) * na) * nb)
            obs = np.max(np.abs(res["fsurf"][k] - orc.surf[k]) * area)
            assert obs <= 2 * hb, (k, obs, hb)
            worst = max(worst, obs / (2 * hb))
        _say("observed error / bound, worst frame: %.3g" % worst)


def _smooth(k):
    for p in (2, 3, 5):
        while k % p == 0:
            k //= p
    return k == 1
