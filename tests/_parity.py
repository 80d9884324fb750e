"""Parity rule between the HIP path and the FP64 oracle.

Shifts: bit-exact on every frame whose oracle gaps are clear, i.e. second-best
minus best f on the searched grid above 1e-4*f_min, and (when downsampling)
the same for the nine full-resolution values.  Frames inside the gap band are
counted and reported, not hidden.

f values: |f_gpu - f_oracle| <= rtol * max(|f_oracle|, 1e-9*(A+B)/Area); the
floor only matters for noise-free tests where f_oracle is 0.  rtol is 1e-5
for every form; the FP64 exact form on uint16 data is held to bit equality.

Gaps (second best minus best f, on the searched grid and among the nine):
bit-equal where f is held to bit equality; otherwise within the error the f
rule allows for two values, rtol * (|f_best| + |f_second|) (+ the floor).  The
nine-point gap is compared only where both sides took the same coarse argmin;
both sides write +inf where there is no second value.
"""
import numpy as np

GAP_REL = 1e-4
F_RTOL = 1e-5


def clear_frames(orc, ds: bool) -> np.ndarray:
    ok = orc.gap_c > GAP_REL * np.abs(orc.fmin)
    ok |= (orc.fmin == 0) & (orc.gap_c > 0)
    if ds:
        fr = np.nanmin(orc.frefine, axis=1)
        okr = (orc.gap_r > GAP_REL * np.abs(fr)) | ((fr == 0) & (orc.gap_r > 0))
        ok &= okr
    return ok


def check(res, orc, ds: bool, exact: bool, rtol: float = F_RTOL, label: str = "",
          f_floor: float = 1e-12):
    """Compare a GPU result (numpy dict) with an oracle AlignResult; returns stats.
    f_floor: the rule's floor 1e-9*(A+B)/Area for f values near 0 (noise-free
    frames), as an absolute scale."""
    T = orc.shifts.shape[0]
    ok = clear_frames(orc, ds)
    shifts = res["shifts"]
    coarse = res["coarse"]
    mism = np.where(ok & np.any(shifts != orc.shifts, axis=1))[0]
    assert mism.size == 0, "%s: shift mismatch on clear frames %s: gpu %s oracle %s" % (
        label, mism[:8], shifts[mism[:8]], orc.shifts[mism[:8]])
    # f at the coarse argmin: compare where both sides picked the same coarse shift
    same = np.all(coarse == orc.coarse, axis=1)
    assert np.all(same[ok]), label
    fg, fo = res["fmin"][same], orc.fmin[same]
    if exact:
        assert np.array_equal(fg, fo), "%s: fmin differs (max |d| %g)" % (
            label, np.max(np.abs(fg - fo)) if fg.size else 0)
    else:
        err = np.abs(fg - fo) / np.maximum(np.abs(fo), 1e-300)
        assert np.all(np.abs(fg - fo) <= rtol * np.maximum(np.abs(fo), f_floor)), \
            "%s: fmin rel err max %g" % (label, err.max())
    stats = {"frames": T, "clear": int(ok.sum()), "near_ties": int((~ok).sum())}
    if ds:
        rg, ro = res["frefine"][same], orc.frefine[same]
        if exact:
            assert np.array_equal(rg, ro), "%s: frefine differs" % label
        else:
            assert np.all(np.abs(rg - ro) <= rtol * np.maximum(np.abs(ro), f_floor)), label
    if "gaps" in res:
        gg, go = res["gaps"], np.stack([orc.gap_c, orc.gap_r], axis=1)
        _check_gaps(gg[:, 0], go[:, 0], orc.fmin, exact, rtol, f_floor, label + " gap_c")
        if ds:
            fb = np.nanmin(orc.frefine, axis=1)
            _check_gaps(gg[same, 1], go[same, 1], fb[same], exact, rtol, f_floor,
                        label + " gap_r")
        else:
            assert np.all(np.isinf(gg[:, 1])), "%s: refine gap without downsampling" % label
        fin = np.isfinite(go[:, 0]) & (go[:, 0] > 0)
        if fin.any():
            stats["gap_c_max_abs_err"] = float(np.max(np.abs(gg[fin, 0] - go[fin, 0])))
    if fo.size:
        stats["fmin_max_rel_err"] = float(np.max(np.abs(fg - fo) / np.maximum(np.abs(fo), 1e-300)))
    return stats


def _check_gaps(gg, go, fbest, exact, rtol, f_floor, label):
    inf_o = np.isinf(go)
    assert np.array_equal(np.isinf(gg), inf_o), "%s: +inf where the oracle has a value" % label
    fin = ~inf_o
    if exact:
        assert np.array_equal(gg[fin], go[fin]), "%s: differs, max |d| %g" % (
            label, np.max(np.abs(gg[fin] - go[fin])) if fin.any() else 0)
        return
    fb = np.abs(fbest[fin])
    tol = rtol * (np.maximum(fb, f_floor) + np.maximum(fb + np.abs(go[fin]), f_floor))
    d = np.abs(gg[fin] - go[fin])
    assert np.all(d <= tol), "%s: max |d| %g beyond %g" % (
        label, d.max(), tol[np.argmax(d - tol)])


def check_surface(sg, so, A_plus_B_over_area=None, exact=False, rtol=F_RTOL, label=""):
    if exact:
        assert np.array_equal(sg, so), "%s: surface differs, max |d| %g" % (
            label, np.nanmax(np.abs(sg - so)))
        return 0.0
    floor = 0.0 if A_plus_B_over_area is None else 1e-9 * A_plus_B_over_area
    tol = rtol * np.maximum(np.abs(so), floor)
    d = np.abs(sg - so)
    assert np.all(d <= tol), "%s: surface rel err max %g" % (label, np.max(d / np.maximum(np.abs(so), 1e-300)))
    return float(np.max(d / np.maximum(np.abs(so), 1e-300)))
