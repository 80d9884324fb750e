"""The certified FFT form: an argmin certificate against the transforms' error
bound, with direct FP64 sums for the frames it does not certify (the exact
argmin of eq. (f) over the searched grid, sec. 2), on the GPU through the C ABI.

* The bound itself (moco_template_fft_bound) is checked against observed
  errors: the FFT form's f on every shift, against the oracle (uint16: exact)
  or the FP64 direct form (float32), stays inside Delta/Area + u|f|.
* Exact ties (a template whose rows repeat with period two and frames that are
  exact rolls of it: many shifts score alike) are never certified, so they are
  recomputed by the FP64 direct form; on uint16 data the shifts then equal the
  oracle's on every frame, with bit-exact f.  (On float32 data the direct
  form's own rounding of the energy split decides exact ties, so recomputed
  frames are compared with that form.)
* Frames with clear gaps are certified and come out bit-identical to the plain
  FFT form.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(moco, ctx, tp, frames, form, surface=False):
    r = moco.moco_align(ctx, _dev(frames), tp, form=form, surface=surface)
    torch.cuda.synchronize()
    out = {k: getattr(r, k).cpu().numpy()
           for k in ("shifts", "fmin", "frefine", "coarse", "gaps", "recomputed")}
    if surface:
        out["fsurf"] = r.fsurf.cpu().numpy()
    return out


def _grid(x, levels):
    """The searched grid: 2x2 box means, `levels` times (odd trailing row/column dropped)."""
    g = np.asarray(x, np.float64)
    for _ in range(int(levels)):
        m2, n2 = g.shape[-2] // 2, g.shape[-1] // 2
        g = g[..., :2 * m2, :2 * n2]
        g = (g[..., 0::2, 0::2] + g[..., 0::2, 1::2] + g[..., 1::2, 0::2] + g[..., 1::2, 1::2]) / 4
    return g


def _delta(kf, ke, sa, sb, mg, ng):
    sab = np.sqrt(sa) * np.sqrt(sb)
    return 1.01 * (ke * (sa + sb) + 2 * U * sab + 2 * kf * np.sqrt(mg * ng) * sab)


def _areas(mg, ng, w):
    s = np.arange(-(w - 1), w)
    return np.outer(mg - np.abs(s), ng - np.abs(s)).astype(np.float64)


CASES = {
    # name: (maker, w, levels, frames)
    "blobs128_f32_w10": (lambda: (synth.blobs128_f32().template,
                                  synth.blobs128_f32().frames(0, 16)), 10, 0),
    "poisson512_u16_w32_ds1": (lambda: (synth.poisson512_u16(T=2000).template,
                                        synth.poisson512_u16(T=2000).frames(0, 6)), 32, 1),
    "lowsnr256_f32_w64": (lambda: (synth.lowsnr256_f32().template,
                                   synth.lowsnr256_f32().frames(0, 3)), 64, 0),
    "ties_u16_61x77_w9": (lambda: synth.row_periodic(61, 77, 8, "u16", 3, 3)[:2], 9, 0),
    "ties_f32_130x98_w7_ds1": (lambda: synth.row_periodic(130, 98, 8, "f32", 6, 2)[:2], 7, 1),
    "poisson_u16_200x230_w20_ds2": (lambda: (synth.PoissonScene(200, 230, 4, seed=5).template,
                                             synth.PoissonScene(200, 230, 4, seed=5).frames(0, 4)),
                                    20, 2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fft_error_bound_holds_and_certificate_follows_it(gpu_lib, name):
    make, w, levels = CASES[name]
    tmpl, fr = make()
    _say("case bound %s T=%d" % (name, len(fr)))
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _dev(tmpl), w, levels)
    kf, ke = gpu_lib.fft_bound(tp)
    assert 0 < kf < 1e-11 and 0 < ke < 1e-11
    fft = _run(gpu_lib, ctx, tp, fr, "fft", surface=True)
    if tmpl.dtype == np.uint16:
        # the oracle's f is exact on uint16 grids
        ref = oracle.align(fr, tmpl, w, levels, want_surface=True).surf
        slack = 0.0
    else:
        ref = _run(gpu_lib, ctx, tp, fr, "fp64", surface=True)["fsurf"]
        slack = None
    ga, gb = _grid(fr, levels), _grid(tmpl, levels)
    mg, ng = gb.shape
    sa = (ga ** 2).sum(axis=(1, 2))
    sb = float((gb ** 2).sum())
    area = _areas(mg, ng, w)
    worst = 0.0
    for k in range(len(fr)):
        d = _delta(kf, ke, sa[k], sb, mg, ng)
        if slack is None:
            # the direct FP64 sums' own rounding: at most m'n'+4 roundings of terms
            # no larger than the overlap energies
            sl = (mg * ng + 4) * U * (sa[k] + sb) / area
        else:
            sl = slack
        bound = d / area + 1.01 * U * np.abs(ref[k]) + sl
        err = np.abs(fft["fsurf"][k] - ref[k])
        assert np.all(err <= bound), (k, float((err / bound).max()))
        worst = max(worst, float((err / bound).max()))
    # the certificate of the certified form is the rule stated with this bound
    cert = _run(gpu_lib, ctx, tp, fr, "fft_cert")
    amin = float((mg - (w - 1)) * (ng - (w - 1)))
    f1, gap = fft["fmin"], fft["gaps"][:, 0]
    f2 = f1 + gap
    with np.errstate(invalid="ignore"):
        margin = gap - 1.01 * U * (np.abs(f1) + np.abs(f2))
        ok = np.where(np.isinf(f2), True, margin > 2 * _delta(kf, ke, sa, sb, mg, ng) / amin)
    assert np.array_equal(cert["recomputed"], (~ok).astype(np.int32))
    _say("%s: observed error / bound <= %.3g; %d of %d frames recomputed"
         % (name, worst, int(cert["recomputed"].sum()), len(fr)))
    tp.close()
    ctx.close()


@pytest.mark.parametrize("dtype,m,n,w,levels", [("u16", 64, 72, 8, 0), ("u16", 128, 128, 8, 1),
                                                ("u16", 97, 110, 12, 0), ("f32", 96, 96, 10, 0),
                                                ("u16", 160, 176, 6, 2)])
def test_exact_ties_are_recomputed_and_match_the_oracle(gpu_lib, dtype, m, n, w, levels):
    tmpl, fr, _ = synth.row_periodic(m, n, 12, dtype, max_shift=min(4, w - 1), noisy_every=3,
                                     seed=m + n)
    _say("case ties %s %dx%d w=%d levels=%d T=12" % (dtype, m, n, w, levels))
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _dev(tmpl), w, levels)
    cert = _run(gpu_lib, ctx, tp, fr, "fft_cert")
    plain = _run(gpu_lib, ctx, tp, fr, "fft")
    direct = _run(gpu_lib, ctx, tp, fr, "fp64")
    orc = oracle.align(fr, tmpl, w, levels)
    noise_free = np.arange(len(fr)) % 3 != 2
    # exact ties (gap 0 on the searched grid) cannot be certified
    tied = noise_free & (orc.gap_c == 0)
    assert tied.sum() >= 4
    assert np.all(cert["recomputed"][tied] == 1)
    rec = cert["recomputed"] == 1
    # recomputed frames are the FP64 direct form's, bit for bit
    for k in ("shifts", "coarse", "fmin", "gaps", "frefine"):
        assert np.array_equal(cert[k][rec].view(np.int64) if cert[k].dtype == np.float64
                              else cert[k][rec],
                              direct[k][rec].view(np.int64) if direct[k].dtype == np.float64
                              else direct[k][rec]), k
    # certified frames: the exact argmin
    assert np.array_equal(cert["coarse"][~rec], orc.coarse[~rec])
    assert np.array_equal(cert["shifts"][~rec], orc.shifts[~rec])
    if dtype == "u16":
        # on uint16 grids the direct sums are exact too: every frame, whatever
        # its gap, has the exact shift, and recomputed frames the exact f
        assert np.array_equal(cert["coarse"], orc.coarse)
        assert np.array_equal(cert["shifts"], orc.shifts)
        assert np.array_equal(cert["fmin"][rec], orc.fmin[rec])
        if levels:
            assert np.array_equal(cert["frefine"], orc.frefine)
    # frames the certificate passed keep the plain FFT form's results bit for bit
    for k in ("shifts", "coarse", "fmin", "gaps"):
        assert np.array_equal(cert[k][~rec].view(np.int64) if cert[k].dtype == np.float64
                              else cert[k][~rec],
                              plain[k][~rec].view(np.int64) if plain[k].dtype == np.float64
                              else plain[k][~rec]), k
    assert np.all(plain["recomputed"] == 0)
    differ = int((plain["coarse"] != orc.coarse).any(axis=1).sum())
    _say("ties %s %dx%d: %d of %d recomputed; the plain FFT form's argmin differs from the "
         "exact one on %d frames" % (dtype, m, n, int(rec.sum()), len(fr), differ))
    tp.close()
    ctx.close()


def test_clear_gaps_are_certified_poisson512(gpu_lib):
    sc = synth.poisson512_u16(T=2000)
    fr = sc.frames(0, 24)
    _say("case certified poisson512 T=24 w=32 ds=1")
    ctx = gpu_lib.Context(0)
    tp = gpu_lib.Template(ctx, _dev(sc.template), 32, True)
    cert = _run(gpu_lib, ctx, tp, fr, "fft_cert", surface=True)
    plain = _run(gpu_lib, ctx, tp, fr, "fft", surface=True)
    assert np.all(cert["recomputed"] == 0)
    for k in ("shifts", "coarse", "fmin", "gaps", "frefine", "fsurf"):
        a, b = cert[k], plain[k]
        if a.dtype == np.float64:
            a, b = a.view(np.int64), b.view(np.int64)
        assert np.array_equal(a, b), k
    orc = oracle.align(fr, sc.template, 32, True)
    assert np.array_equal(cert["shifts"], orc.shifts)
    # the exact forms recompute nothing and say so
    ex = _run(gpu_lib, ctx, tp, fr, "int8")
    assert np.all(ex["recomputed"] == 0)
    tp.close()
    ctx.close()


def test_certified_chunks_and_batch(gpu_lib):
    tmpl, fr, _ = synth.row_periodic(128, 140, 40, "u16", max_shift=5, noisy_every=4, seed=11)
    w = 8
    _say("case certified chunks T=40 128x140 w=8")
    big = gpu_lib.Context(0)
    tb = gpu_lib.Template(big, _dev(tmpl), w, 0)
    whole = _run(gpu_lib, big, tb, fr, "fft_cert")
    # a budget of a few frames' scratch: several chunks
    small = gpu_lib.Context(0, scratch_budget=3 << 20)
    ts = gpu_lib.Template(small, _dev(tmpl), w, 0)
    parts = _run(gpu_lib, small, ts, fr, "fft_cert")
    for k in whole:
        assert np.array_equal(whole[k].view(np.int64) if whole[k].dtype == np.float64 else whole[k],
                              parts[k].view(np.int64) if parts[k].dtype == np.float64 else parts[k]), k
    orc = oracle.align(fr, tmpl, w, 0)
    assert np.array_equal(whole["shifts"], orc.shifts)
    assert whole["recomputed"].sum() >= 10
    # a batch under AUTO: float32 data resolve to the certified FP32 FFT form
    f32 = fr.astype(np.float32)
    t32 = gpu_lib.Template(big, _dev(tmpl.astype(np.float32)), w, 0)
    assert gpu_lib.resolved_form(big, t32, "auto") == "fft32_cert"
    res = gpu_lib.moco_align_batch(big, [(_dev(f32), t32), (_dev(fr), tb)], form="auto")
    torch.cuda.synchronize()
    one = _run(gpu_lib, big, t32, f32, "fft32_cert")
    assert np.array_equal(res[0].shifts.cpu().numpy(), one["shifts"])
    assert np.array_equal(res[0].recomputed.cpu().numpy(), one["recomputed"])
    # certified by the FP32 or the FP64 bound: the exact shift
    direct = one["recomputed"] == 2
    assert np.array_equal(one["shifts"][~direct], orc.shifts[~direct])
    # the uint16 stack: whichever form AUTO ranks faster, the exact shifts
    used = gpu_lib.resolved_form(big, tb, "auto")
    alone = _run(gpu_lib, big, tb, fr, used)
    assert np.array_equal(res[1].shifts.cpu().numpy(), orc.shifts)
    assert np.array_equal(res[1].recomputed.cpu().numpy(), alone["recomputed"])
    for t in (t32, ts, tb):
        t.close()
    small.close()
    big.close()
