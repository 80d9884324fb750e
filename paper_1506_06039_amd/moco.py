"""Python binding of libmoco.so (argument marshalling only).

Every step of the search runs in the HIP kernels behind the C ABI declared in
``include/moco.h``; this module only turns torch device tensors into pointers
and the current torch stream into a ``hipStream_t``.  There is no CPU path:
if the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmoco.so")

MOCO_OK, MOCO_EINVAL, MOCO_ENOMEM, MOCO_EDEVICE, MOCO_EBUSY, MOCO_ECANCELED = 0, -1, -2, -3, -4, -5
MOCO_U16, MOCO_F32 = 1, 2
FORMS = {"auto": 0, "fft": 1, "fft_cert": 2, "fp64": 3, "int8": 4, "fft32": 5,
         "fft32_cert": 6}
FORM_COUNT = 7


class MocoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("moco error %d: %s" % (code, msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("libmoco.so is not built (%s); run python -m paper_1506_06039_amd.build"
                      % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)


class _Outputs(ctypes.Structure):
    _fields_ = [("shifts", ctypes.c_void_p), ("fmin", ctypes.c_void_p),
                ("fsurf", ctypes.c_void_p), ("frefine", ctypes.c_void_p),
                ("coarse", ctypes.c_void_p), ("gaps", ctypes.c_void_p),
                ("recomputed", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_lib.moco_create.argtypes = [_i, ctypes.c_size_t, ctypes.POINTER(_vp)]
_lib.moco_create.restype = _i
_lib.moco_destroy.argtypes = [_vp]
_lib.moco_destroy.restype = None
_lib.moco_template_create.argtypes = [_vp, _vp, _i, _i, _i, _i, _i, _vp, ctypes.POINTER(_vp)]
_lib.moco_template_create.restype = _i
_lib.moco_template_destroy.argtypes = [_vp]
_lib.moco_template_destroy.restype = None
_lib.moco_align.argtypes = [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i,
                            ctypes.POINTER(_Outputs), _vp]
_lib.moco_align.restype = _i
_lib.moco_align_noalloc.argtypes = [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i,
                                    ctypes.POINTER(_Outputs), _vp]
_lib.moco_align_noalloc.restype = _i
_lib.moco_profile_enable.argtypes = [_vp, _i]
_lib.moco_profile_enable.restype = _i
_lib.moco_profile_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
_lib.moco_profile_read.restype = _i
class _Stack(ctypes.Structure):
    _fields_ = [("d_frames", ctypes.c_void_p), ("tmpl", ctypes.c_void_p),
                ("T", ctypes.c_int), ("m", ctypes.c_int), ("n", ctypes.c_int),
                ("w", ctypes.c_int), ("downsample", ctypes.c_int), ("dtype", ctypes.c_int),
                ("out", _Outputs)]


_lib.moco_align_batch.argtypes = [_vp, ctypes.POINTER(_Stack), _i, _i, _i, _vp]
_lib.moco_align_batch.restype = _i
_lib.moco_graph_create_batch.argtypes = [_vp, ctypes.POINTER(_Stack), _i, _i, _i,
                                         ctypes.POINTER(_vp)]
_lib.moco_graph_create_batch.restype = _i
class ServerResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("source", ctypes.c_int), ("status", ctypes.c_int),
                ("shift", ctypes.c_int32 * 2), ("coarse", ctypes.c_int32 * 2),
                ("fmin", ctypes.c_double), ("frefine", ctypes.c_double * 9),
                ("gaps", ctypes.c_double * 2), ("latency_us", ctypes.c_double)]


_lib.moco_server_create.argtypes = [_vp, ctypes.c_size_t, _i, ctypes.POINTER(_vp)]
_lib.moco_server_create.restype = _i
_lib.moco_server_add_source.argtypes = [_vp, _i, _vp, _i, _i, _i, _i, _i]
_lib.moco_server_add_source.restype = _i
_lib.moco_server_submit.argtypes = [_vp, _i, _vp, ctypes.c_uint64]
_lib.moco_server_submit.restype = _i
_lib.moco_server_poll.argtypes = [_vp, ctypes.POINTER(ServerResult), _i, _i]
_lib.moco_server_poll.restype = _i
_lib.moco_server_pending.argtypes = [_vp]
_lib.moco_server_pending.restype = _i
_lib.moco_server_destroy.argtypes = [_vp]
_lib.moco_server_destroy.restype = _i
_lib.moco_template_form.argtypes = [_vp, _i, ctypes.POINTER(_i)]
_lib.moco_template_form.restype = _i
_lib.moco_template_fft_bound.argtypes = [_vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
_lib.moco_template_fft_bound.restype = _i
_lib.moco_template_int8_products.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
_lib.moco_template_int8_products.restype = _i
_lib.moco_template_int8_tile.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
_lib.moco_template_int8_tile.restype = _i
_lib.moco_tune_set_tile.argtypes = [_i, _i, _i, _i, _i, _i]
_lib.moco_tune_set_tile.restype = _i
_lib.moco_graph_create.argtypes = [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i,
                                   ctypes.POINTER(_Outputs), ctypes.POINTER(_vp)]
_lib.moco_graph_create.restype = _i
_lib.moco_graph_launch.argtypes = [_vp, _vp]
_lib.moco_graph_launch.restype = _i
_lib.moco_graph_destroy.argtypes = [_vp]
_lib.moco_graph_destroy.restype = None
_lib.moco_tune.argtypes = [_vp, _vp, _i, _vp, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double)]
_lib.moco_tune.restype = _i
_lib.moco_tune_set.argtypes = [_i, _i, _i, _i, _i, _i]
_lib.moco_tune_set.restype = _i
_lib.moco_tune_get.argtypes = [_i, _i, _i, _i, _i, ctypes.POINTER(_i)]
_lib.moco_tune_get.restype = _i
_lib.moco_tune_clear.argtypes = []
_lib.moco_tune_clear.restype = None
_lib.moco_last_error.argtypes = []
_lib.moco_last_error.restype = ctypes.c_char_p
_lib.moco_version.argtypes = []
_lib.moco_version.restype = ctypes.c_char_p
_lib.moco_apply.argtypes = [_vp, _vp, _vp, _i, _i, _i, _i, _vp, _vp, _vp]
_lib.moco_apply.restype = _i
_lib.moco_default_params.argtypes = [_i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]
_lib.moco_default_params.restype = _i


def _check(rc: int):
    if rc != MOCO_OK:
        raise MocoError(rc, _lib.moco_last_error().decode())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint16:
        return MOCO_U16
    if t.dtype == torch.float32:
        return MOCO_F32
    raise TypeError("frames must be uint16 or float32, got %s" % t.dtype)


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def version() -> str:
    return _lib.moco_version().decode()


def last_error() -> str:
    return _lib.moco_last_error().decode()


class Context:
    """moco_create / moco_destroy."""

    def __init__(self, device: int = 0, scratch_budget: int = 0):
        h = _vp()
        _check(_lib.moco_create(device, scratch_budget, ctypes.byref(h)))
        self.handle = h
        self.device = torch.device("cuda", device)

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.moco_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Template:
    """moco_template_create / moco_template_destroy."""

    def __init__(self, ctx: Context, template: torch.Tensor, w: int, downsample: int):
        if not template.is_cuda or template.dim() != 2:
            raise ValueError("template must be a 2-D device tensor")
        template = template.contiguous()
        m, n = template.shape
        h = _vp()
        _check(_lib.moco_template_create(ctx.handle, template.data_ptr(), _dtype_code(template),
                                         m, n, w, int(downsample),
                                         _stream_handle(template.device), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.m, self.n, self.w, self.downsample = m, n, w, int(downsample)
        self.dtype = template.dtype

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.ctx.device)
            _lib.moco_template_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Result:
    shifts: torch.Tensor            # (T, 2) int32
    fmin: torch.Tensor              # (T,) float64
    frefine: torch.Tensor           # (T, 9) float64
    coarse: torch.Tensor            # (T, 2) int32
    gaps: torch.Tensor              # (T, 2) float64
    fsurf: torch.Tensor | None      # (T, W, W) float64
    recomputed: torch.Tensor | None = None  # (T,) int32


def moco_align(ctx: Context, frames: torch.Tensor, tmpl: Template, form: str = "auto",
               surface: bool = False, out: Result | None = None) -> Result:
    """Align frames (T, m, n) against a prepared template; enqueued on the current stream."""
    if not frames.is_cuda or frames.dim() != 3:
        raise ValueError("frames must be a 3-D device tensor")
    if not frames.is_contiguous():
        raise ValueError("frames must be contiguous")
    T, m, n = frames.shape
    W = 2 * tmpl.w - 1
    dev = frames.device
    if out is None:
        out = Result(
            shifts=torch.empty((T, 2), dtype=torch.int32, device=dev),
            fmin=torch.empty(T, dtype=torch.float64, device=dev),
            frefine=torch.empty((T, 9), dtype=torch.float64, device=dev),
            coarse=torch.empty((T, 2), dtype=torch.int32, device=dev),
            gaps=torch.empty((T, 2), dtype=torch.float64, device=dev),
            fsurf=torch.empty((T, W, W), dtype=torch.float64, device=dev) if surface else None,
            recomputed=torch.empty(T, dtype=torch.int32, device=dev))
    o = _outputs(out, T, W, dev)
    _check(_lib.moco_align(ctx.handle, frames.data_ptr(), tmpl.handle, T, m, n, tmpl.w,
                           int(tmpl.downsample), _dtype_code(frames), FORMS[form],
                           ctypes.byref(o), _stream_handle(dev)))
    return out


def moco_align_noalloc(ctx: Context, frames: torch.Tensor, tmpl: Template, out: Result,
                       form: str = "auto") -> Result:
    """moco_align through the allocation-free entry point: the library's fixed
    per-device scratch instead of the context's; the caller brings every
    output (out), so nothing is allocated here either."""
    if not frames.is_cuda or frames.dim() != 3 or not frames.is_contiguous():
        raise ValueError("frames must be a contiguous 3-D device tensor")
    T, m, n = frames.shape
    o = _outputs(out, T, 2 * tmpl.w - 1, frames.device)
    _check(_lib.moco_align_noalloc(ctx.handle, frames.data_ptr(), tmpl.handle, T, m, n, tmpl.w,
                                   int(tmpl.downsample), _dtype_code(frames), FORMS[form],
                                   ctypes.byref(o), _stream_handle(frames.device)))
    return out


class Graph:
    """moco_graph_*: a moco_align call on `frames` captured once; launch()
    realigns whatever `frames` holds then, into `out` (kept alive here)."""

    def __init__(self, ctx: Context, frames: torch.Tensor, tmpl: Template, form: str = "auto",
                 surface: bool = False, out: Result | None = None):
        if not frames.is_cuda or frames.dim() != 3 or not frames.is_contiguous():
            raise ValueError("frames must be a contiguous 3-D device tensor")
        T, m, n = frames.shape
        self.frames, self.tmpl, self.ctx = frames, tmpl, ctx
        self.out = out if out is not None else \
            _new_result(T, 2 * tmpl.w - 1, frames.device, surface)
        o = _outputs(self.out, T, 2 * tmpl.w - 1, frames.device)
        h = _vp()
        _check(_lib.moco_graph_create(ctx.handle, frames.data_ptr(), tmpl.handle, T, m, n, tmpl.w,
                                      int(tmpl.downsample), _dtype_code(frames), FORMS[form],
                                      ctypes.byref(o), ctypes.byref(h)))
        self.handle = h

    def launch(self) -> Result:
        """Enqueue a replay on the current stream; returns the output record."""
        _check(_lib.moco_graph_launch(self.handle, _stream_handle(self.frames.device)))
        return self.out

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.frames.device)
            _lib.moco_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def moco_apply(ctx: Context, frames: torch.Tensor, shifts: torch.Tensor, frames_out: bool = True,
               mean: bool = True, out: torch.Tensor | None = None,
               mean_out: torch.Tensor | None = None):
    """The corrected stack (T, m, n), same dtype, black outside each frame's
    overlap with the template, and its FP64 mean image (m, n); enqueued on the
    current stream.  Returns (corrected or None, mean or None)."""
    if not frames.is_cuda or frames.dim() != 3 or not frames.is_contiguous():
        raise ValueError("frames must be a contiguous 3-D device tensor")
    T, m, n = frames.shape
    if shifts.dtype != torch.int32 or tuple(shifts.shape) != (T, 2) or not shifts.is_contiguous():
        raise ValueError("shifts must be a contiguous (T, 2) int32 tensor")
    dev = frames.device
    if shifts.device != dev:
        raise ValueError("shifts are on %s, frames on %s" % (shifts.device, dev))
    if frames_out and out is None:
        out = torch.empty_like(frames)
    if mean and mean_out is None:
        mean_out = torch.empty((m, n), dtype=torch.float64, device=dev)
    if frames_out:
        _check_tensor("out", out, (T, m, n), frames.dtype, dev)
        nb = frames.numel() * frames.element_size()
        if out.data_ptr() < frames.data_ptr() + nb and frames.data_ptr() < out.data_ptr() + nb:
            raise ValueError("out must not overlap the frames")
    if mean:
        _check_tensor("mean_out", mean_out, (m, n), torch.float64, dev)
    _check(_lib.moco_apply(ctx.handle, frames.data_ptr(), shifts.data_ptr(), T, m, n,
                           _dtype_code(frames), out.data_ptr() if frames_out else None,
                           mean_out.data_ptr() if mean else None, _stream_handle(dev)))
    return (out if frames_out else None), (mean_out if mean else None)


def default_params(m: int, n: int):
    """The paper's defaults for an m x n stack: (w, downsample levels)."""
    w, ds = _i(), _i()
    _check(_lib.moco_default_params(m, n, ctypes.byref(w), ctypes.byref(ds)))
    return w.value, ds.value


def _new_result(T: int, W: int, dev, surface: bool) -> Result:
    return Result(
        shifts=torch.empty((T, 2), dtype=torch.int32, device=dev),
        fmin=torch.empty(T, dtype=torch.float64, device=dev),
        frefine=torch.empty((T, 9), dtype=torch.float64, device=dev),
        coarse=torch.empty((T, 2), dtype=torch.int32, device=dev),
        gaps=torch.empty((T, 2), dtype=torch.float64, device=dev),
        fsurf=torch.empty((T, W, W), dtype=torch.float64, device=dev) if surface else None,
        recomputed=torch.empty(T, dtype=torch.int32, device=dev))


_OUT_SPEC = (  # field, trailing shape (after T) as a function of W, dtype, required
    ("shifts", lambda W: (2,), torch.int32, True),
    ("fmin", lambda W: (), torch.float64, True),
    ("frefine", lambda W: (9,), torch.float64, True),
    ("coarse", lambda W: (2,), torch.int32, True),
    ("gaps", lambda W: (2,), torch.float64, True),
    ("fsurf", lambda W: (W, W), torch.float64, False),
    ("recomputed", lambda W: (), torch.int32, False),
)


def _check_tensor(name: str, t: torch.Tensor, shape, dtype, dev):
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch.Tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.dtype != dtype:
        raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    if t.device != dev:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, dev))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _validate_result(r: Result, T: int, W: int, dev):
    """Every output the kernels write must have exactly the shape, dtype and
    device they assume: a wrong one would be written past its end."""
    if not isinstance(r, Result):
        raise ValueError("out must be a Result")
    for name, shp, dt, required in _OUT_SPEC:
        t = getattr(r, name)
        if t is None:
            if required:
                raise ValueError("out.%s is required" % name)
            continue
        _check_tensor("out." + name, t, (T,) + shp(W), dt, dev)


def _outputs(r: Result, T: int, W: int, dev) -> "_Outputs":
    _validate_result(r, T, W, dev)
    return _Outputs(r.shifts.data_ptr(), r.fmin.data_ptr(),
                    r.fsurf.data_ptr() if r.fsurf is not None else None,
                    r.frefine.data_ptr(), r.coarse.data_ptr(), r.gaps.data_ptr(),
                    r.recomputed.data_ptr() if r.recomputed is not None else None)


def _stack_records(items, surface: bool):
    """The moco_stack records of (frames, Template[, Result]) items, their
    Results (new where not given) and the device."""
    stacks = (_Stack * max(1, len(items)))()
    results = []
    dev = None
    for k, it in enumerate(items):
        frames, tmpl = it[0], it[1]
        if not frames.is_cuda or frames.dim() != 3 or not frames.is_contiguous():
            raise ValueError("stack %d: frames must be a contiguous 3-D device tensor" % k)
        T, m, n = frames.shape
        dev = frames.device
        res = it[2] if len(it) > 2 and it[2] is not None else \
            _new_result(T, 2 * tmpl.w - 1, dev, surface)
        results.append(res)
        o = _outputs(res, T, 2 * tmpl.w - 1, dev)
        stacks[k] = _Stack(frames.data_ptr(), tmpl.handle.value, T, m, n, tmpl.w,
                           int(tmpl.downsample), _dtype_code(frames), o)
    return stacks, results, dev


def moco_align_batch(ctx: Context, items, form: str = "auto", lanes: int = 0,
                     surface: bool = False):
    """Align several stacks in one call.  items: list of (frames, Template) or
    (frames, Template, Result).  Returns the list of Results (enqueued on the
    current stream)."""
    stacks, results, dev = _stack_records(items, surface)
    stream = _stream_handle(dev if dev is not None else ctx.device)
    _check(_lib.moco_align_batch(ctx.handle, stacks, len(items), FORMS[form], lanes, stream))
    return results


class BatchGraph:
    """moco_graph_create_batch: a moco_align_batch call captured once;
    launch() realigns whatever the stacks' frame buffers hold then, into
    `results` (the buffers and templates are kept alive here)."""

    def __init__(self, ctx: Context, items, form: str = "auto", lanes: int = 0,
                 surface: bool = False):
        self.items = list(items)
        stacks, self.results, dev = _stack_records(self.items, surface)
        self.device = dev if dev is not None else torch.device("cuda", ctx.device)
        h = _vp()
        _check(_lib.moco_graph_create_batch(ctx.handle, stacks, len(self.items), FORMS[form],
                                            lanes, ctypes.byref(h)))
        self.handle = h

    def launch(self):
        """Enqueue a replay on the current stream; returns the Results."""
        _check(_lib.moco_graph_launch(self.handle, _stream_handle(self.device)))
        return self.results

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.moco_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def align(frames: torch.Tensor, template: torch.Tensor, w: int, downsample: bool,
          form: str = "auto", surface: bool = False) -> Result:
    """One-shot convenience: context + template + align on the current stream."""
    ctx = Context(frames.device.index or 0)
    tp = Template(ctx, template, w, downsample)
    r = moco_align(ctx, frames, tp, form=form, surface=surface)
    torch.cuda.synchronize(frames.device)
    tp.close()
    ctx.close()
    return r


STAGE_COUNT = 7


def profile_enable(ctx: Context, on: bool = True):
    """moco_profile_enable: bracket every stage launch with HIP events."""
    _check(_lib.moco_profile_enable(ctx.handle, int(bool(on))))


def profile_read(ctx: Context):
    """moco_profile_read: (milliseconds, launches) per stage since the last read."""
    ms = (ctypes.c_double * STAGE_COUNT)()
    n = (ctypes.c_int64 * STAGE_COUNT)()
    _check(_lib.moco_profile_read(ctx.handle, ms, n))
    return list(ms), list(n)


def resolved_form(ctx: Context, tmpl: Template, form: str) -> str:
    """moco_template_form: the correlation form a call with ``form`` runs for this template."""
    r = _i()
    _check(_lib.moco_template_form(tmpl.handle, FORMS[form], ctypes.byref(r)))
    return {v: k for k, v in FORMS.items()}[r.value]


_FORM_NAMES = {v: k for k, v in FORMS.items()}
_DTYPES = {"u16": 1, "f32": 2}


def tune(ctx: Context, tmpl: Template, frames: int = 0):
    """moco_tune: time the forms that apply to this template on `frames` copies
    of it (0: 1024) and record the fastest for its key; AUTO then picks it.
    Returns (form, {form: s/frame})."""
    chosen = _i()
    sec = (ctypes.c_double * FORM_COUNT)()
    _check(_lib.moco_tune(ctx.handle, tmpl.handle, frames, _stream_handle(ctx.device),
                          ctypes.byref(chosen), sec))
    times = {_FORM_NAMES[k]: sec[k] for k in range(FORM_COUNT) if k in _FORM_NAMES and sec[k] >= 0}
    return _FORM_NAMES[chosen.value], times


def tune_set(m: int, n: int, w: int, downsample: int, dtype: str, form: str):
    """moco_tune_set (dtype "u16" or "f32")."""
    _check(_lib.moco_tune_set(m, n, w, int(downsample), _DTYPES[dtype], FORMS[form]))


def tune_get(m: int, n: int, w: int, downsample: int, dtype: str):
    """moco_tune_get: the recorded form name, or None."""
    f = _i()
    rc = _lib.moco_tune_get(m, n, w, int(downsample), _DTYPES[dtype], ctypes.byref(f))
    return _FORM_NAMES[f.value] if rc == 0 else None


def tune_clear():
    _lib.moco_tune_clear()


def tune_save(path: str, keys):
    """Write the recorded forms of `keys` ((m, n, w, downsample, dtype) tuples)
    as a JSON list."""
    import json
    rows = []
    for m, n, w, ds, dt in keys:
        f = tune_get(m, n, w, ds, dt)
        if f is not None:
            rows.append({"m": m, "n": n, "w": w, "downsample": int(ds), "dtype": dt, "form": f})
    with open(path, "w") as fh:
        json.dump(rows, fh, indent=1)


def tune_load(path: str) -> int:
    """Record every form of a JSON list written by tune_save; returns how many."""
    import json
    rows = json.load(open(path))
    for r in rows:
        tune_set(r["m"], r["n"], r["w"], r["downsample"], r["dtype"], r["form"])
    return len(rows)


def fft_bound(tmpl: Template):
    """moco_template_fft_bound: (kf, ke) with |h^ - h| <= kf sqrt(m'n' Sa Sb)
    and energy errors <= ke Sa (Sa, Sb: the grids' sums of squares)."""
    kf, ke = ctypes.c_double(), ctypes.c_double()
    _check(_lib.moco_template_fft_bound(tmpl.handle, ctypes.byref(kf), ctypes.byref(ke)))
    return kf.value, ke.value


def int8_tile(tmpl: Template) -> int:
    """moco_template_int8_tile: the int8 form's shift tile (16, 32 or 64) for the
    template's key now, in launches of more than 64 frames (recorded by tune
    or tune_set_tile, else the model's)."""
    n = ctypes.c_int()
    _check(_lib.moco_template_int8_tile(tmpl.handle, ctypes.byref(n)))
    return n.value


def tune_set_tile(m: int, n: int, w: int, downsample: int, dtype: str, tile: int):
    """moco_tune_set_tile (dtype "u16")."""
    _check(_lib.moco_tune_set_tile(m, n, w, int(downsample), _DTYPES[dtype], tile))


def int8_products(tmpl: Template) -> int:
    """moco_template_int8_products: digit products per correlation term in the
    int8 form's main pass (3: base-128 digits and their sums; 4: base-256)."""
    n = ctypes.c_int()
    _check(_lib.moco_template_int8_products(tmpl.handle, ctypes.byref(n)))
    return n.value


class Server:
    """moco_server_*: single host frames from many sources, continuous batching."""

    def __init__(self, ctx: Context, device_budget: int = 0, max_slots: int = 64):
        h = _vp()
        _check(_lib.moco_server_create(ctx.handle, device_budget, max_slots, ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def add_source(self, source: int, template, w: int, downsample: bool):
        """template: host numpy array (uint16 or float32), m x n."""
        import numpy as np
        t = np.ascontiguousarray(template)
        code = MOCO_U16 if t.dtype == np.uint16 else MOCO_F32 if t.dtype == np.float32 else None
        if code is None:
            raise TypeError("template must be uint16 or float32")
        m, n = t.shape
        _check(_lib.moco_server_add_source(self.handle, source, t.ctypes.data, code, m, n, w,
                                           int(downsample)))
        self._keep[source] = ((m, n), t.dtype)

    def submit(self, source: int, frame, tag: int) -> bool:
        """True when admitted, False on back-pressure (no free slot)."""
        import numpy as np
        f = np.ascontiguousarray(frame)
        spec = self._keep.get(source)
        if spec is not None and (f.shape != spec[0] or f.dtype != spec[1]):
            # the library copies the source's frame size from this pointer
            raise ValueError("source %d takes %s %s frames, got %s %s"
                             % (source, spec[0], spec[1], f.shape, f.dtype))
        rc = _lib.moco_server_submit(self.handle, source, f.ctypes.data, tag)
        if rc == MOCO_EBUSY:
            return False
        _check(rc)
        return True

    def poll(self, max_results: int = 256, timeout_us: int = 0):
        buf = (ServerResult * max_results)()
        k = _lib.moco_server_poll(self.handle, buf, max_results, timeout_us)
        if k < 0:
            _check(k)
        return [buf[i] for i in range(k)]

    def pending(self) -> int:
        return _lib.moco_server_pending(self.handle)

    def close(self) -> int:
        if getattr(self, "handle", None):
            n = _lib.moco_server_destroy(self.handle)
            self.handle = None
            return n
        return 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
