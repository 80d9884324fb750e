"""moco oracle: a plain FP64 CPU brute force of the translation search.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP path (``paper_1506_06039_amd``) and never imports it.

The arithmetic lives in ``moco_oracle.c`` (plain C, FP64, no fast-math, OpenMP
over frames only); this module only builds it with gcc and marshals numpy
arrays.  Every function follows section 2 of the paper ("Mathematical
Development"): the objective f over the overlap set D, the window
max(|s|,|t|) < w, the argmin, and the x2 step with nine evaluations.  The
downsampling filter (a 2x2 box mean) and the tie order are readings of a
paper that names neither; they are listed with the other readings in the
design notes.

Functions with no independent pin: none.  Absolute f values are pinned by
closed forms, statistics and brute force (see ``tests/test_oracle_pins.py``);
the paper itself prints no worked example.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "moco_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile moco_oracle.c into oracle/liboracle.so with gcc (-O2 -fopenmp)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    c_int = ctypes.c_int
    lib.oracle_downsample.argtypes = [dp, c_int, c_int, dp]
    lib.oracle_downsample.restype = None
    lib.oracle_area.argtypes = [c_int, c_int, c_int, c_int]
    lib.oracle_area.restype = ctypes.c_double
    lib.oracle_f.argtypes = [dp, dp, c_int, c_int, c_int, c_int]
    lib.oracle_f.restype = ctypes.c_double
    lib.oracle_terms.argtypes = [dp, dp, c_int, c_int, c_int, c_int, dp]
    lib.oracle_terms.restype = None
    lib.oracle_surface.argtypes = [dp, dp, c_int, c_int, c_int, dp]
    lib.oracle_surface.restype = None
    lib.oracle_validate.argtypes = [c_int] * 5
    lib.oracle_validate.restype = c_int
    lib.oracle_align.argtypes = [dp, dp, c_int, c_int, c_int, c_int, c_int,
                                 ip, ip, dp, dp, dp, dp, dp, dp, c_int]
    lib.oracle_align.restype = c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = c_int
    lib.oracle_apply.argtypes = [dp, ip, c_int, c_int, c_int, dp, dp]
    lib.oracle_apply.restype = None
    _lib = lib
    return lib


def _dp(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.float64)


def downsample(x) -> np.ndarray:
    """2x2 box mean with floor dimensions (odd trailing row/column dropped)."""
    x = _f64(x)
    m, n = x.shape
    y = np.empty((m // 2, n // 2), np.float64)
    _load().oracle_downsample(_dp(x), m, n, _dp(y))
    return y


def area(m: int, n: int, s: int, t: int) -> float:
    """Area(D_{s,t}) by counting the overlap set."""
    return _load().oracle_area(m, n, s, t)


def f(a, b, s: int, t: int) -> float:
    """f_{s,t}: mean of (a[i+s][j+t]-b[i][j])^2 over D_{s,t}."""
    a, b = _f64(a), _f64(b)
    m, n = a.shape
    return _load().oracle_f(_dp(a), _dp(b), m, n, s, t)


def terms(a, b, s: int, t: int):
    """(sum a^2, sum b^2, sum a*b, Area) over D_{s,t}, each by its own sum."""
    a, b = _f64(a), _f64(b)
    m, n = a.shape
    out = np.empty(4, np.float64)
    _load().oracle_terms(_dp(a), _dp(b), m, n, s, t, _dp(out))
    return tuple(float(v) for v in out)


def surface(a, b, w: int) -> np.ndarray:
    """All f_{s,t} with max(|s|,|t|) < w as a (2w-1, 2w-1) array [s+w-1, t+w-1]."""
    a, b = _f64(a), _f64(b)
    m, n = a.shape
    W = 2 * w - 1
    out = np.empty((W, W), np.float64)
    _load().oracle_surface(_dp(a), _dp(b), m, n, w, _dp(out))
    return out


def validate(T: int, m: int, n: int, w: int, ds: int) -> bool:
    return _load().oracle_validate(T, m, n, w, ds) == 0


def threads() -> int:
    return _load().oracle_threads()


@dataclass
class AlignResult:
    coarse: np.ndarray    # (T, 2) int32 argmin on the searched grid
    shifts: np.ndarray    # (T, 2) int32 final (S, T)
    fmin: np.ndarray      # (T,) f at the coarse argmin
    gap_c: np.ndarray     # (T,) second-best minus best on the coarse surface
    frefine: np.ndarray   # (T, 9) f at (2s*+u, 2t*+v), [u+1][v+1]; NaN if not ds
    gap_r: np.ndarray     # (T,) second-best minus best of the nine
    kappa: np.ndarray     # (T,) (A+B)/(Area*fmin) at the coarse argmin
    surf: np.ndarray | None  # (T, 2w-1, 2w-1) or None


def align(frames, template, w: int, downsample: bool, want_surface: bool = False,
          nthreads: int = 0, chunk: int = 64) -> AlignResult:
    """Align every frame of ``frames`` (T, m, n) against ``template`` (m, n).

    Inputs of any real dtype are converted to FP64 (exact for uint16 and
    float32).  Frames are converted in chunks so that a long stack never needs
    an FP64 copy in memory at once.
    """
    frames = np.asarray(frames)
    T, m, n = frames.shape
    ds = int(downsample)   # levels of 2x2 downsampling (True = 1)
    if not validate(T, m, n, w, ds):
        raise ValueError("invalid search: T=%d m=%d n=%d w=%d ds=%d" % (T, m, n, w, ds))
    tm = _f64(template)
    if tm.shape != (m, n):
        raise ValueError("template shape %s != frame shape %s" % (tm.shape, (m, n)))
    W = 2 * w - 1
    coarse = np.zeros((T, 2), np.int32)
    shifts = np.zeros((T, 2), np.int32)
    fmin = np.zeros(T, np.float64)
    gap_c = np.zeros(T, np.float64)
    frefine = np.zeros((T, 9), np.float64)
    gap_r = np.zeros(T, np.float64)
    kappa = np.zeros(T, np.float64)
    surf = np.zeros((T, W, W), np.float64) if want_surface else None
    lib = _load()
    for k0 in range(0, T, chunk):
        k1 = min(T, k0 + chunk)
        fr = _f64(frames[k0:k1])
        c = np.zeros((k1 - k0, 2), np.int32)
        sh = np.zeros((k1 - k0, 2), np.int32)
        fm = np.zeros(k1 - k0)
        gc = np.zeros(k1 - k0)
        fr9 = np.zeros((k1 - k0, 9))
        gr = np.zeros(k1 - k0)
        kp = np.zeros(k1 - k0)
        sf = np.zeros((k1 - k0, W, W)) if want_surface else None
        rc = lib.oracle_align(_dp(fr), _dp(tm), k1 - k0, m, n, w, ds, _ip(c), _ip(sh),
                              _dp(fm), _dp(gc), _dp(fr9), _dp(gr), _dp(kp),
                              _dp(sf) if sf is not None else None, nthreads)
        if rc != 0:
            raise RuntimeError("oracle_align failed")
        coarse[k0:k1] = c
        shifts[k0:k1] = sh
        fmin[k0:k1] = fm
        gap_c[k0:k1] = gc
        frefine[k0:k1] = fr9
        gap_r[k0:k1] = gr
        kappa[k0:k1] = kp
        if want_surface:
            surf[k0:k1] = sf
    return AlignResult(coarse, shifts, fmin, gap_c, frefine, gap_r, kappa, surf)


def apply(frames, shifts, want_frames: bool = True):
    """The corrected stack and its mean image: frame k moved by its (S,T),
    black (0) outside the overlap with the template, and the FP64 mean of the
    corrected frames (summed in frame order).  Returns (corrected or None, mean)."""
    fr = _f64(frames)
    T, m, n = fr.shape
    sh = np.ascontiguousarray(np.asarray(shifts), dtype=np.int32).reshape(T, 2)
    out = np.empty((T, m, n), np.float64) if want_frames else None
    mean = np.empty((m, n), np.float64)
    _load().oracle_apply(_dp(fr), _ip(sh), T, m, n, _dp(out) if out is not None else None,
                         _dp(mean))
    return out, mean
