"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage of section 2 ("Mathematical Development") or
section 3 ("Results") it follows.  None of them retypes the oracle: they use
a literal 1-based enumeration with exact rationals, the paper's own DP
recurrence and FFT construction run through numpy, closed forms, planted
shifts, statistics of the noise, and a hand-worked fixture.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests._exact import f_exact, overlap_set

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ints(rng, m, n, lo=0, hi=50):
    return rng.integers(lo, hi, size=(m, n)).astype(np.int64)


# --- overlap set and its area (sec. 2, definition of D) -------------------

def test_area_equals_literal_enumeration():
    for m in range(1, 8):
        for n in range(1, 8):
            for s in range(-(m - 1), m):
                for t in range(-(n - 1), n):
                    lit = len(overlap_set(m, n, s, t))
                    assert lit == (m - abs(s)) * (n - abs(t))
                    assert oracle.area(m, n, s, t) == lit


# --- the objective itself (sec. 2, objective f) ----------------------------

@pytest.mark.parametrize("seed", range(6))
def test_f_matches_exact_rationals_all_windows(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 8)), int(rng.integers(1, 8))
    a, b = _ints(rng, m, n, -20, 60), _ints(rng, m, n, -20, 60)
    al, bl = a.tolist(), b.tolist()
    for w in range(1, min(m, n) + 1):
        surf = oracle.surface(a, b, w)
        for s in range(-(w - 1), w):
            for t in range(-(w - 1), w):
                ex = f_exact(al, bl, s, t)
                # integer data: oracle sums exactly, one rounding at the division
                assert surf[s + w - 1, t + w - 1] == float(ex), (m, n, w, s, t)


def test_hand_worked_fixture():
    rows = {}
    shifts = []
    with open(os.path.join(GOLDEN, "hand_2x3_w2.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            k, *v = line.split()
            if k in ("m", "n", "w"):
                rows[k] = int(v[0])
            elif k in ("a", "b"):
                rows[k] = [float(x) for x in v]
            elif k == "argmin":
                rows["argmin"] = tuple(int(x) for x in v)
            elif k == "gap":
                rows["gap"] = int(v[0]) / int(v[1])
            else:
                shifts.append((int(k), int(v[0]), int(v[1]), int(v[2])))
    m, n, w = rows["m"], rows["n"], rows["w"]
    a = np.array(rows["a"]).reshape(m, n)
    b = np.array(rows["b"]).reshape(m, n)
    surf = oracle.surface(a, b, w)
    assert len(shifts) == (2 * w - 1) ** 2
    for s, t, tot, ar in shifts:
        assert oracle.area(m, n, s, t) == ar
        assert surf[s + w - 1, t + w - 1] == tot / ar
    r = oracle.align(a[None], b, w, False)
    assert tuple(r.shifts[0]) == rows["argmin"]
    assert r.fmin[0] == 2.0
    assert r.gap_c[0] == rows["gap"]


def _read_search_fixture(name):
    rec = {"coarse": {}, "nine": {}}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            k, *v = line.split()
            if k in ("m", "n", "w", "ds"):
                rec[k] = int(v[0])
            elif k in ("a", "b"):
                rec[k] = [int(x) for x in v]
            elif k in ("coarse", "nine"):
                rec[k][(int(v[0]), int(v[1]))] = Fraction(int(v[2]), int(v[3]))
            elif k in ("coarse_argmin", "shift"):
                rec[k] = (int(v[0]), int(v[1]))
            else:   # gap_c, gap_r, kappa: numerator denominator
                rec[k] = Fraction(int(v[0]), int(v[1]))
    return rec


def test_hand_worked_search_with_refine_fixture():
    """Whole search on a 4x4 pair, one 2x2 level, w = 2 (sec. 2: the window on
    the downsampled images, the argmin doubled and the nine evaluations at full
    resolution): every coarse value, the coarse gap, kappa at the argmin, the
    nine values, the final shift and the refine gap, each worked by hand."""
    rec = _read_search_fixture("hand_4x4_ds1_w2.txt")
    m, n, w, ds = rec["m"], rec["n"], rec["w"], rec["ds"]
    a = np.array(rec["a"], np.float64).reshape(m, n)
    b = np.array(rec["b"], np.float64).reshape(m, n)
    W = 2 * w - 1
    assert len(rec["coarse"]) == W * W and len(rec["nine"]) == 9
    # the hand values agree with the literal 1-based enumeration
    al, bl = a.astype(int).tolist(), b.astype(int).tolist()
    for (S, T), v in rec["nine"].items():
        assert f_exact(al, bl, S, T) == v
    r = oracle.align(a[None], b, w, bool(ds), want_surface=True)
    for (s, t), v in rec["coarse"].items():
        assert r.surf[0, s + w - 1, t + w - 1] == float(v), (s, t)
    assert tuple(r.coarse[0]) == rec["coarse_argmin"]
    assert r.fmin[0] == float(rec["coarse"][rec["coarse_argmin"]])
    # gaps are differences of two rounded f values (second best minus best)
    best = min(rec["coarse"].values())
    assert r.gap_c[0] == float(best + rec["gap_c"]) - float(best)
    assert r.kappa[0] == float(rec["kappa"])
    cs, ct = rec["coarse_argmin"]
    for u in (-1, 0, 1):
        for v in (-1, 0, 1):
            assert r.frefine[0, (u + 1) * 3 + (v + 1)] == float(rec["nine"][(2 * cs + u, 2 * ct + v)])
    assert tuple(r.shifts[0]) == rec["shift"]
    fb = rec["nine"][rec["shift"]]
    assert r.gap_r[0] == float(fb + rec["gap_r"]) - float(fb)
    assert abs(r.gap_r[0] - float(rec["gap_r"])) < 1e-15


def _tie_key(f, s, t):
    # the tie order read for the argmin: f, then max(|s|,|t|), |s|+|t|, s, t
    return (f, max(abs(s), abs(t)), abs(s) + abs(t), s, t)


def _box_exact(x):
    m, n = len(x) // 2, len(x[0]) // 2
    return [[Fraction(x[2 * i][2 * j] + x[2 * i][2 * j + 1] + x[2 * i + 1][2 * j]
                      + x[2 * i + 1][2 * j + 1], 4) for j in range(n)] for i in range(m)]


def _search_exact(al, bl, w, ds):
    """The search of sec. 2 in exact rationals on the literal overlap set:
    (coarse argmin, f1, gap_c, kappa, final shift, gap_r, best of the nine;
    the last two None without downsampling)."""
    ga, gb = (_box_exact(al), _box_exact(bl)) if ds else (al, bl)
    vals = []
    for s in range(-(w - 1), w):
        for t in range(-(w - 1), w):
            vals.append((_tie_key(f_exact(ga, gb, s, t), s, t), s, t))
    vals.sort()
    (k1, s1, t1) = vals[0]
    f1 = k1[0]
    gap_c = vals[1][0][0] - f1 if len(vals) > 1 else None
    D = overlap_set(len(ga), len(ga[0]), s1, t1)
    A = sum(Fraction(ga[i + s1 - 1][j + t1 - 1]) ** 2 for (i, j) in D)
    B = sum(Fraction(gb[i - 1][j - 1]) ** 2 for (i, j) in D)
    kappa = (A + B) / (len(D) * f1) if f1 != 0 else None
    if not ds:
        return (s1, t1), f1, gap_c, kappa, (s1, t1), None, None
    nine = sorted((_tie_key(f_exact(al, bl, 2 * s1 + u, 2 * t1 + v), 2 * s1 + u, 2 * t1 + v),
                   2 * s1 + u, 2 * t1 + v) for u in (-1, 0, 1) for v in (-1, 0, 1))
    fb = nine[0][0][0]
    return (s1, t1), f1, gap_c, kappa, (nine[0][1], nine[0][2]), nine[1][0][0] - fb, fb


@pytest.mark.parametrize("seed", range(8))
def test_gaps_and_kappa_match_exact_rationals(seed):
    """gap_c, gap_r (second best minus best, sec. 2 argmin and nine-point step)
    and kappa = (A+B)/(Area f1) at the argmin (the energy split of sec. 2) on
    random integer images, against exact rationals with the tie order written
    out independently."""
    rng = np.random.default_rng(500 + seed)
    ds = seed % 2
    m, n = (int(rng.integers(4, 9)), int(rng.integers(4, 9)))
    w = int(rng.integers(1, min(m >> ds, n >> ds) + 1))
    b = _ints(rng, m, n, 0, 40)
    a = np.roll(b, (int(rng.integers(-2, 3)), int(rng.integers(-2, 3))), axis=(0, 1)) \
        + _ints(rng, m, n, 0, 9)
    al, bl = a.tolist(), b.tolist()
    (cs, ct), f1, gap_c, kappa, shift, gap_r, fb = _search_exact(al, bl, w, ds)
    r = oracle.align(a[None], b, w, bool(ds))
    assert tuple(r.coarse[0]) == (cs, ct)
    assert r.fmin[0] == float(f1)
    u = 2.0 ** -53
    if gap_c is None:
        assert r.gap_c[0] == math.inf
    else:
        # a difference of two correctly rounded values
        assert abs(r.gap_c[0] - float(gap_c)) <= 2 * u * (2 * float(f1) + float(gap_c)) + 1e-300
    if kappa is None:
        assert not np.isfinite(r.kappa[0]) or np.isnan(r.kappa[0])
    else:
        assert abs(r.kappa[0] - float(kappa)) <= 8 * u * float(kappa)
    assert tuple(r.shifts[0]) == shift
    if gap_r is None:
        assert r.gap_r[0] == math.inf
    else:
        assert abs(r.gap_r[0] - float(gap_r)) <= 2 * u * (2 * float(fb) + float(gap_r)) + 1e-300


def test_kappa_of_the_search_is_one_over_relative_contrast():
    """kappa = (A+B)/(Area f) at the argmin: a frame that is the template plus a
    constant c at the zero shift has f = c^2 and A + B = sum (b+c)^2 + sum b^2,
    a closed form independent of the oracle's arithmetic."""
    rng = np.random.default_rng(77)
    b = _ints(rng, 10, 12, 5, 60)
    for c in (1, 3, 7):
        a = b + c
        r = oracle.align(a[None], b, 1, False)
        N = b.size
        AB = int(((b + c) ** 2).sum() + (b ** 2).sum())
        assert r.fmin[0] == float(c * c)
        assert r.kappa[0] == pytest.approx(AB / (N * c * c), rel=1e-15)


# --- the energy split (sec. 2, Area*f = sum a^2 + sum b^2 - 2 sum ab) -------

@pytest.mark.parametrize("seed", range(4))
def test_energy_split_identity_in_integers(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = 9, 7
    a, b = _ints(rng, m, n, 0, 1000), _ints(rng, m, n, 0, 1000)
    for s in range(-3, 4):
        for t in range(-3, 4):
            A, B, h, ar = oracle.terms(a, b, s, t)
            ex = f_exact(a.tolist(), b.tolist(), s, t)
            assert ar == (m - abs(s)) * (n - abs(t))
            assert int(A) + int(B) - 2 * int(h) == ex * int(ar)


# --- the DP recurrence for the overlap energies (sec. 2, recurrence for g) --

def _g_by_recurrence(a):
    """g_{s,t} for s,t <= 0 from g_{s,t} = g_{s-1,t} + g_{s,t-1} - g_{s-1,t-1} + a_{m+s,n+t}^2,
    with g = 0 when m+s = 0 or n+t = 0 (empty overlap); 1-based a as printed."""
    m, n = a.shape
    g = {}
    for s in range(-m, 1):
        for t in range(-n, 1):
            if m + s == 0 or n + t == 0:
                g[(s, t)] = 0
            else:
                g[(s, t)] = (g[(s - 1, t)] + g[(s, t - 1)] - g[(s - 1, t - 1)]
                             + int(a[m + s - 1, n + t - 1]) ** 2)
    return g


@pytest.mark.parametrize("shape", [(6, 5), (4, 7), (8, 8)])
def test_overlap_energy_matches_paper_recurrence(shape):
    rng = np.random.default_rng(7)
    a = _ints(rng, *shape, 0, 300)
    b = _ints(rng, *shape, 0, 300)
    m, n = shape
    g = _g_by_recurrence(a)
    for s in range(-(m - 1), 1):
        for t in range(-(n - 1), 1):
            A, _, _, _ = oracle.terms(a, b, s, t)
            assert int(A) == g[(s, t)]
    # other quadrants: the same recurrence on the mirrored image (s -> -s and/or t -> -t)
    for fi, fj in ((True, False), (False, True), (True, True)):
        am = a[::-1] if fi else a
        am = am[:, ::-1] if fj else am
        gm = _g_by_recurrence(np.ascontiguousarray(am))
        for s in range(-(m - 1), 1):
            for t in range(-(n - 1), 1):
                ss, tt = (-s if fi else s), (-t if fj else t)
                A, _, _, _ = oracle.terms(a, b, ss, tt)
                assert int(A) == gm[(s, t)]


# --- the FFT construction of h (sec. 2, padded transforms and ifft2) -------

@pytest.mark.parametrize("shape,w", [((5, 7), 4), ((12, 9), 5), ((16, 16), 8)])
def test_correlation_matches_paper_fft_construction(shape, w):
    rng = np.random.default_rng(11)
    m, n = shape
    a = _ints(rng, m, n, 0, 500)
    b = _ints(rng, m, n, 0, 500)
    # paper's construction: rotate b by 180 degrees, pad both with w zero
    # columns on the right and w zero rows below, multiply the transforms
    bhat = b[::-1, ::-1]
    pa = np.zeros((m + w, n + w)); pa[:m, :n] = a
    pb = np.zeros((m + w, n + w)); pb[:m, :n] = bhat
    c = np.real(np.fft.ifft2(np.fft.fft2(pa) * np.fft.fft2(pb)))
    # the minimal-padding correlation form: any P >= m+w-1, Q >= n+w-1
    P, Q = m + w - 1, n + w - 1
    qa = np.zeros((P, Q)); qa[:m, :n] = a
    qb = np.zeros((P, Q)); qb[:m, :n] = b
    cc = np.real(np.fft.ifft2(np.fft.fft2(qa) * np.conj(np.fft.fft2(qb))))
    for s in range(-(w - 1), w):
        for t in range(-(w - 1), w):
            _, _, h, _ = oracle.terms(a, b, s, t)
            assert round(c[s + m - 1, t + n - 1]) == int(h)
            assert round(cc[s % P, t % Q]) == int(h)


# --- the search: argmin and sign (sec. 2), refine convention (sec. 2, last paragraph)

def _blob_image(rng, m, n, k=12):
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    img = 1.0 + 0.3 * np.cos(2 * np.pi * i / m + 0.4) * np.cos(2 * np.pi * j / n + 1.1)
    for _ in range(k):
        ci, cj = rng.uniform(0, m), rng.uniform(0, n)
        sg = rng.uniform(1.5, 3.5)
        img = img + rng.uniform(0.5, 2.0) * np.exp(-((i - ci) ** 2 + (j - cj) ** 2) / (2 * sg * sg))
    return img


def test_planted_shifts_recovered_without_downsampling():
    rng = np.random.default_rng(3)
    m, n, w = 40, 36, 9
    b = _blob_image(rng, m, n)
    truth = [(0, 0), (3, -5), (-8, 8), (7, 1), (-2, -6), (8, -8)]
    frames = np.stack([np.roll(b, st, axis=(0, 1)) + 1e-4 * rng.standard_normal((m, n))
                       for st in truth])
    r = oracle.align(frames, b, w, False)
    assert [tuple(x) for x in r.shifts] == truth
    assert [tuple(x) for x in r.coarse] == truth


def test_planted_odd_and_even_shifts_refined_at_full_resolution():
    rng = np.random.default_rng(5)
    m, n, w = 64, 60, 8
    b = _blob_image(rng, m, n, 20)
    truth = [(7, -13), (6, 4), (-5, -1), (0, 0), (-14, 9), (1, 1), (13, -14)]
    frames = np.stack([np.roll(b, st, axis=(0, 1)) for st in truth])
    r = oracle.align(frames, b, w, True)
    for k, (S, T) in enumerate(truth):
        assert tuple(r.shifts[k]) == (S, T)
        cs, ct = r.coarse[k]
        assert S - 2 * cs in (-1, 0, 1) and T - 2 * ct in (-1, 0, 1)
        # rolled, noise-free: wrapped pixels lie outside D, so f(S,T) is exactly 0
        u, v = S - 2 * cs, T - 2 * ct
        assert r.frefine[k, (u + 1) * 3 + (v + 1)] == 0.0


def test_rolled_seam_gives_exact_zero():
    rng = np.random.default_rng(9)
    b = _blob_image(rng, 23, 29)
    for S, T in [(4, -7), (-9, 2), (0, 11)]:
        a = np.roll(b, (S, T), axis=(0, 1))
        assert oracle.f(a, b, S, T) == 0.0
        assert oracle.f(a, b, S + 1, T) > 0.0


def test_zero_shift_normalisation_two_noisy_copies():
    # f(0,0) of two independent noisy copies of one image estimates 2 sigma^2
    rng = np.random.default_rng(21)
    m = n = 128
    base = _blob_image(rng, m, n, 40)
    sig = 0.3
    a = base + sig * rng.standard_normal((m, n))
    b = base + sig * rng.standard_normal((m, n))
    N = m * n
    ratio = oracle.f(a, b, 0, 0) / (2 * sig * sig)
    assert abs(ratio - 1.0) < 5 * math.sqrt(2.0 / N)


def test_window_one_is_plain_mse():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((31, 17))
    b = rng.standard_normal((31, 17))
    r = oracle.align(a[None], b, 1, False)
    mse = math.fsum(((a - b) ** 2).ravel()) / a.size
    assert tuple(r.shifts[0]) == (0, 0)
    assert r.fmin[0] == pytest.approx(mse, rel=1e-14, abs=0)


def test_swap_symmetry():
    rng = np.random.default_rng(8)
    a, b = _ints(rng, 11, 13, 0, 99), _ints(rng, 11, 13, 0, 99)
    sab = oracle.surface(a, b, 5)
    sba = oracle.surface(b, a, 5)
    assert np.array_equal(sab, sba[::-1, ::-1])


def test_downsample_is_box_mean():
    rng = np.random.default_rng(12)
    for m, n in [(8, 8), (9, 7), (5, 12)]:
        x = rng.integers(0, 65536, size=(m, n)).astype(np.float64)
        mc, nc = m // 2, n // 2
        ref = x[:2 * mc, :2 * nc].reshape(mc, 2, nc, 2).mean((1, 3))
        assert np.array_equal(oracle.downsample(x), ref)


def test_tie_order_prefers_smallest_displacement():
    # constant images: f == 0 at every shift, so the tie order alone decides
    a = np.full((9, 9), 3.0)
    r = oracle.align(a[None], a, 4, False)
    assert tuple(r.shifts[0]) == (0, 0) and r.gap_c[0] == 0.0
    # period-3 image: zero at every multiple of 3; the smallest is (0,0)
    i = np.arange(12)[:, None]
    j = np.arange(12)[None, :]
    p = ((i % 3) * 7 + (j % 3) * 2).astype(float)
    r = oracle.align(np.roll(p, (3, 0), axis=(0, 1))[None], p, 5, False)
    assert tuple(r.shifts[0]) == (0, 0)
    # two equal minima at the same ring: (-1, 0) wins over (0, -1)? ring 1, |s|+|t| 1, s smaller
    a = np.zeros((5, 5))
    b = np.zeros((5, 5))
    r = oracle.align(a[None], b, 2, False)
    assert tuple(r.shifts[0]) == (0, 0)


def test_tie_order_lexicographic_within_ring():
    # a and b both symmetric under transposition make f(s,t) == f(t,s) exactly
    # (integer data); a = roll(b,(1,0)) + roll(b,(0,1)) against 2b puts the
    # minimum on the pair (1,0)/(0,1), which the order (ring, |s|+|t|, s, t)
    # resolves to (0,1)
    i = np.arange(24)[:, None]
    j = np.arange(24)[None, :]
    b = np.zeros((24, 24))
    for ci, cj, amp in [(6, 15, 40), (15, 6, 40), (12, 12, 70), (4, 4, 25), (19, 19, 25)]:
        b += np.rint(amp * np.exp(-((i - ci) ** 2 + (j - cj) ** 2) / 8.0))
        b += np.rint(amp * np.exp(-((i - cj) ** 2 + (j - ci) ** 2) / 8.0))
    assert np.array_equal(b, b.T)
    a = np.roll(b, (1, 0), axis=(0, 1)) + np.roll(b, (0, 1), axis=(0, 1))
    surf = oracle.surface(a, 2 * b, 3)
    assert surf[3, 2] == surf[2, 3]                   # f(1,0) == f(0,1)
    assert surf[3, 2] == surf.min()
    r = oracle.align(a[None], 2 * b, 3, False)
    assert tuple(r.shifts[0]) == (0, 1)
    assert r.gap_c[0] == 0.0


def test_validation_rules():
    assert oracle.validate(1, 8, 8, 8, 0)
    assert not oracle.validate(1, 8, 8, 9, 0)       # w > m'
    assert not oracle.validate(1, 8, 8, 5, 1)       # w > m/2
    assert oracle.validate(0, 8, 8, 4, 1)           # T = 0 is valid
    assert not oracle.validate(1, 1, 8, 1, 1)       # m' = 0
    assert not oracle.validate(1, 8, 8, 0, 0)       # w < 1
    assert oracle.validate(1, 8, 8, 2, 2)           # two levels: 2x2 grid, w = 2
    assert not oracle.validate(1, 8, 8, 2, -1)      # levels >= 0
    assert not oracle.validate(-1, 8, 8, 2, 0)


# --- the corrected stack and its mean image (sec. 2, the motion-corrected
# video; sec. 3, fig. 1 and fig. 2) ------------------------------------------

def test_correction_of_a_rolled_frame_is_the_template_except_where_black():
    # fig. 1's caption: a corrected frame matches the template except where it
    # is black.  A noise-free frame roll(b,(S,T)) moved back by (S,T) is b on
    # the overlap set D_{S,T} (taken literally, 1-based) and 0 on the rest.
    rng = np.random.default_rng(11)
    m, n = 9, 13
    b = _ints(rng, m, n, 1, 200).astype(np.float64)
    for S, T in [(0, 0), (3, -5), (-4, 2), (8, 12), (-8, -12)]:
        a = np.roll(b, (S, T), axis=(0, 1))
        out, mean = oracle.apply(a[None], [[S, T]])
        D = overlap_set(m, n, S, T)          # 1-based (i', j') with (i'+S, j'+T) inside
        want = np.zeros((m, n))
        for (ip, jp) in D:
            want[ip - 1, jp - 1] = b[ip - 1, jp - 1]
        assert np.array_equal(out[0], want), (S, T)
        assert np.array_equal(mean, want)


def test_correction_composes_and_beyond_the_frame_is_black():
    # moving by s1 then s2 equals moving by s1+s2, except where the second move
    # reads outside the frame; a shift of a whole side or more leaves nothing
    rng = np.random.default_rng(12)
    m, n = 11, 7
    a = _ints(rng, m, n, 1, 99).astype(np.float64)
    for s1, s2 in [((2, 1), (3, -2)), ((-4, 3), (1, 1)), ((5, -6), (-7, 2))]:
        c1, _ = oracle.apply(a[None], [s1])
        c2, _ = oracle.apply(c1, [s2])
        c12, _ = oracle.apply(a[None], [(s1[0] + s2[0], s1[1] + s2[1])])
        i = np.arange(m)[:, None] + s2[0]
        j = np.arange(n)[None, :] + s2[1]
        inside = (i >= 0) & (i < m) & (j >= 0) & (j < n)
        assert np.array_equal(c2[0], np.where(inside, c12[0], 0.0)), (s1, s2)
    for S, T in [(m, 0), (0, -n), (-m - 3, 2 * n)]:
        c, mean = oracle.apply(a[None], [(S, T)])
        assert not c.any() and not mean.any()


def test_mean_image_of_the_corrected_stack():
    # fig. 2: the mean of the corrected video.  Integer data keep every sum
    # exact, so the mean equals the exact rational mean; zero shifts give the
    # plain mean of the frames.
    rng = np.random.default_rng(13)
    T, m, n = 7, 6, 5
    fr = rng.integers(0, 1000, size=(T, m, n)).astype(np.float64)
    sh = np.zeros((T, 2), np.int32)
    _, mean = oracle.apply(fr, sh)
    from fractions import Fraction
    for i in range(m):
        for j in range(n):
            exact = Fraction(int(fr[:, i, j].sum()), T)
            assert mean[i, j] == float(exact)
    sh = rng.integers(-3, 4, size=(T, 2)).astype(np.int32)
    out, mean = oracle.apply(fr, sh)
    for i in range(m):
        for j in range(n):
            assert mean[i, j] == float(Fraction(int(out[:, i, j].sum()), T))


# --- more than one level of downsampling (sec. 2, last paragraph: the argmin
# is multiplied by two "multiple times", nine evaluations each time) --------

def _smooth_scene(rng, m, n, k=12):
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    img = np.zeros((m, n))
    for _ in range(k):
        ci, cj = rng.uniform(0, m), rng.uniform(0, n)
        sg = rng.uniform(3, 6)
        img += rng.uniform(50, 200) * np.exp(-((i - ci) ** 2 + (j - cj) ** 2) / (2 * sg * sg))
    return np.rint(img + 20)


def test_multilevel_coarse_surface_is_the_search_on_twice_downsampled_images():
    rng = np.random.default_rng(21)
    m, n = 64, 48
    b = _smooth_scene(rng, m, n)
    fr = np.stack([np.roll(b, (5, -7), axis=(0, 1)), np.roll(b, (-9, 3), axis=(0, 1))])
    box = lambda x: x[..., : x.shape[-2] // 2 * 2, : x.shape[-1] // 2 * 2].reshape(
        x.shape[:-2] + (x.shape[-2] // 2, 2, x.shape[-1] // 2, 2)).mean(axis=(-3, -1))
    r2 = oracle.align(fr, b, 5, 2, want_surface=True)
    r0 = oracle.align(box(box(fr)), box(box(b)), 5, 0, want_surface=True)
    assert np.array_equal(r2.surf, r0.surf)
    assert np.array_equal(r2.coarse, r0.coarse)


@pytest.mark.parametrize("levels", [2, 3])
def test_multilevel_recovers_planted_shifts_of_every_parity(levels):
    rng = np.random.default_rng(22 + levels)
    m = n = 128
    b = _smooth_scene(rng, m, n, k=20)
    shifts = [(0, 0), (5, -7), (-6, 9), (11, 3), (-13, -2), (8, 10)]
    fr = np.stack([np.roll(b, s, axis=(0, 1)) for s in shifts])
    w = (m >> levels) // 3
    r = oracle.align(fr, b, w, levels)
    assert [tuple(x) for x in r.shifts] == shifts
    # the coarse argmin is the planted shift divided by 2^levels, to within a
    # step of each level's refinement
    for (S, T), (cs, ct) in zip(shifts, r.coarse):
        assert abs(cs * (1 << levels) - S) < (1 << levels) and abs(ct * (1 << levels) - T) < (1 << levels)


def test_multilevel_validation():
    assert oracle.validate(1, 64, 64, 8, 3)          # 8x8 coarse grid, w = 8
    assert not oracle.validate(1, 64, 64, 9, 3)      # w > m'
    assert not oracle.validate(1, 64, 64, 1, 5)      # at most 4 levels
    assert not oracle.validate(1, 15, 64, 1, 4)      # m >> 4 = 0
