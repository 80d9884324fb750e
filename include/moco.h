/*
 * moco.h -- C ABI of the MI355X (gfx950) translation-search library.
 *
 * The library computes, for every frame a of a stack and one template b, the
 * integer translation (S,T) chosen by the search of Dubbs, Guevara, Peterka
 * and Yuste, "moco: Fast Motion Correction for Calcium Imaging"
 * (arXiv:1506.06039), section 2:
 *
 *   f_{s,t} = (1/Area(D_{s,t})) * sum over (i,j) in D_{s,t} of (a[i+s][j+t] - b[i][j])^2
 *
 * where D_{s,t} is the set of pixels (i,j) such that both (i,j) and
 * (i+s,j+t) lie inside the m x n image (sec. 2, objective and overlap set).
 * Every shift with max(|s|,|t|) < w is scored (sec. 2, first paragraph), on
 * the frame box-downsampled by 2x2 `downsample` times (0: the frame itself;
 * 1: once, the paper's setting for frames larger than 256x256); the argmin is
 * then multiplied by two and f_{2s+u,2t+v}, u,v in {-1,0,1}, evaluated on the
 * next finer level with the minimum kept, once per level down to full
 * resolution (sec. 2, last paragraph).
 *
 * Indices are 0-based.  Row shift s runs along m, column shift t along n.
 * A frame made as np.roll(template, (S,T), axis=(0,1)) returns (S,T); the
 * frame is corrected by shifting it by (-S,-T).
 *
 * Conventions for every entry point:
 *   - Return value: MOCO_OK (0) or a negative moco_status.  Nothing throws,
 *     aborts or exits across this boundary.  moco_last_error() returns a
 *     thread-local message describing the last failure of the calling thread.
 *   - Device pointers ("d_" prefix) are HIP device addresses on the context's
 *     device, owned by the caller; the library never frees them.
 *   - Work is ordered on the caller's HIP stream (`hip_stream`, a hipStream_t
 *     passed as void*; NULL is the legacy default stream).  Outputs are valid
 *     once that stream has synchronised.  Entry points return as soon as the
 *     work is enqueued.
 *   - A context is used by one host thread at a time.  Calls on one context
 *     share its scratch memory: enqueue them on one stream, or synchronise
 *     between calls made on different streams.
 *   - Layouts are row-major and contiguous.
 */
#ifndef MOCO_H
#define MOCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MOCO_OK = 0,
    MOCO_EINVAL = -1,    /* an argument is out of range, null or inconsistent */
    MOCO_ENOMEM = -2,    /* device scratch beyond the context's budget, or allocation failure */
    MOCO_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed */
    MOCO_EBUSY = -4,     /* serving: no free slot or memory right now (back-pressure) */
    MOCO_ECANCELED = -5  /* serving: request cancelled by server destruction */
} moco_status;

typedef enum {
    MOCO_U16 = 1,   /* uint16 pixels (photon counts) */
    MOCO_F32 = 2    /* float32 pixels (must be finite) */
} moco_dtype;

/* How the correlation sum of a[i+s][j+t]*b[i][j] (the third term of the
 * energy split of sec. 2) is computed.  Every form computes the same f. */
typedef enum {
    MOCO_FORM_AUTO = 0,       /* library choice: a form recorded for the search key
                                 (moco_tune, moco_tune_set) where it applies; for uint16
                                 data, of MOCO_FORM_INT8_MFMA and MOCO_FORM_FFT_CERTIFIED
                                 the one a per-frame time model of the template's
                                 geometry ranks faster among those that apply (int8 for
                                 small windows, the FFT for wide ones); for float32 data
                                 MOCO_FORM_FFT32_CERTIFIED; else MOCO_FORM_FP64_EXACT */
    MOCO_FORM_FFT = 1,        /* h from FP64 complex transforms of the zero-padded grids
                                 (sec. 2, the FFT construction of h), transform lengths
                                 5-smooth and at most 2048; f to about 1e-12 relative */
    MOCO_FORM_FFT_CERTIFIED = 2, /* MOCO_FORM_FFT with a certified argmin: per frame, if
                                 the gap between the best and second-best f of the searched
                                 grid does not exceed twice the transforms' error bound
                                 (moco_template_fft_bound), the frame's correlation is
                                 recomputed by MOCO_FORM_FP64_EXACT's direct sums and the
                                 frame combined again; otherwise the computed argmin is the
                                 exact argmin of the grid.  Recomputed frames equal
                                 MOCO_FORM_FP64_EXACT's results bit for bit; on uint16 data
                                 that is the exact argmin with bit-exact f, so the searched
                                 grid's shift is the exact one on every frame (on float32
                                 data, the FP64 form's own rounding decides ties closer
                                 than it) */
    MOCO_FORM_FP64_EXACT = 3, /* direct FP64 sums on the vector ALUs; bit-exact f for uint16 */
    MOCO_FORM_INT8_MFMA = 4,  /* uint16 only: exact integer correlation on int8 matrix
                                 cores (balanced base-128 digits and three products per
                                 term when the template allows, else base-256 and four:
                                 moco_template_int8_products); bit-exact f */
    MOCO_FORM_FFT32 = 5,      /* the plain single-precision form: h from FP32 complex
                                 transforms (sec. 2, the FFT construction of h) of the
                                 grids less a common offset c (the template grid's mean,
                                 rounded to an integer for uint16 data), with the overlap
                                 energies of the centred grids and f = (A + B - 2h)/Area
                                 in FP64 (the split holds for any common offset); f to
                                 about 1e-6 relative, not certified: the argmin can
                                 differ from the exact one where the best and second-best
                                 f are closer than that.  Never chosen by AUTO; the
                                 single-precision comparator of the other forms.  Same
                                 applicability as MOCO_FORM_FFT */
    MOCO_FORM_FFT32_CERTIFIED = 6 /* MOCO_FORM_FFT32 with a certified argmin: the
                                 argmin of the searched grid is certified when the gap to
                                 the second-best f exceeds twice an a-posteriori bound of
                                 the FP32 correlation's error (first order in 2^-24, from
                                 the centred grids' 2-norms and the largest magnitudes of
                                 the frame's and the template's spectra); a certified
                                 frame's f at its argmin is then evaluated by its
                                 definition (FP64 sum of squared differences over D; exact
                                 for uint16), and the gap moves with it, while the rest
                                 of the surface keeps its FP32 correlation.  Frames not
                                 certified go through MOCO_FORM_FFT_CERTIFIED (FP64
                                 transforms, then direct sums for what its bound leaves)
                                 and equal its results.  Same applicability as
                                 MOCO_FORM_FFT */
} moco_form;

/* Number of moco_form values (the length of moco_tune's seconds_per_frame). */
#define MOCO_FORM_COUNT 7

typedef struct moco_ctx moco_ctx;
typedef struct moco_tmpl moco_tmpl;

/* Outputs of one stack of T frames.  All are device pointers; only `shifts`
 * is required.  W = 2w-1.
 *   shifts  T x 2 int32   final (S,T) (after the x2 refine when downsampled)
 *   fmin    T     double  f at the argmin of the searched (coarse) grid
 *   fsurf   T x W x W double  every f of the searched grid, [frame][s+w-1][t+w-1]
 *   frefine T x 9 double  f at (2s*+u, 2t*+v), [u+1][v+1]; NaN when not downsampled
 *   coarse  T x 2 int32   argmin (s*,t*) on the searched grid
 *   gaps    T x 2 double  (second-best minus best f on the searched grid,
 *                          second-best minus best of the nine; +inf when n/a)
 *   recomputed T int32    1 where MOCO_FORM_FFT_CERTIFIED recomputed the frame's
 *                          correlation by direct sums (its argmin was not
 *                          certified); for MOCO_FORM_FFT32_CERTIFIED the number
 *                          of passes after the FP32 one: 1 FP64 transforms, 2
 *                          FP64 transforms and direct sums, or 3 where exact
 *                          integer sums over the nine shifts around the
 *                          computed argmin settled it (uint16 frames with at
 *                          most one 2x2 level and w <= 32, when every shift
 *                          the bound leaves open is among those nine); else 0 (every
 *                          other form writes 0)
 * f is in squared intensity units of the searched grid (box-mean units when
 * downsampled). */
typedef struct {
    int32_t *shifts;
    double *fmin;
    double *fsurf;
    double *frefine;
    int32_t *coarse;
    double *gaps;
    int32_t *recomputed;
} moco_outputs;

/* Create a context on HIP device `device`.  `scratch_budget_bytes` caps the
 * device scratch the context may hold (0 = 1 GiB); larger stacks are processed
 * in chunks that fit.  On success *out owns the context.
 * Errors: MOCO_EINVAL (null out, bad device), MOCO_EDEVICE. */
int moco_create(int device, size_t scratch_budget_bytes, moco_ctx **out);

/* Release the context and its scratch.  Safe on NULL.  The caller must have
 * synchronised every stream used with it. */
void moco_destroy(moco_ctx *ctx);

/* Prepare a template for search (sec. 2: b, its overlap energies sum b^2 for
 * every shift of the window, computed once and kept resident).
 * d_template: m x n pixels of `dtype` on the device, read on `hip_stream`
 * during this call's enqueued work only (the library keeps its own copy).
 * Errors: MOCO_EINVAL (validation as for moco_align), MOCO_ENOMEM, MOCO_EDEVICE. */
int moco_template_create(moco_ctx *ctx, const void *d_template, moco_dtype dtype, int m, int n,
                         int w, int downsample, void *hip_stream, moco_tmpl **out);

/* Release a template.  Safe on NULL.  Pending work that uses it must have
 * completed (synchronise its stream first). */
void moco_template_destroy(moco_tmpl *tmpl);

/* Align one stack: T frames of m x n pixels (d_frames, T*m*n elements of
 * `dtype`) against a template prepared with the same (dtype, m, n, w,
 * downsample).  T == 0 is a no-op.  Validation (MOCO_EINVAL): downsample (the
 * number of 2x2 levels) in 0..4; m' = m >> downsample, n' = n >> downsample
 * (each level drops an odd trailing row/column) at least 1; 1 <= w <=
 * min(m',n'); T >= 0; known dtype and form; non-null frames, template and
 * out->shifts; template parameters equal to the call's.  MOCO_FORM_INT8_MFMA on
 * float32 data, or with more than one level, is MOCO_EINVAL.  The nine refine
 * values and the refine gap are those of the full-resolution step; the levels
 * in between keep only their argmin. */
int moco_align(moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m, int n,
               int w, int downsample, moco_dtype dtype, moco_form form, const moco_outputs *out,
               void *hip_stream);

/* moco_align for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, validation, results (bit for bit) and kernels as moco_align, but
 * its scratch is a fixed 64 MiB device array held by the library on each
 * device (from the first moco_create on that device until the process ends)
 * instead of the context's budget: it calls no hipMalloc, hipFree or other
 * allocating routine, and records no stage timing.  Stacks larger than the
 * array run in chunks that fit it.  Every call on one device shares that
 * device's array, whatever the context: calls that overlap in time on one
 * device race (enqueue them on one stream, or synchronise between them).
 * Errors: those of moco_align; MOCO_ENOMEM when one frame needs more than the
 * 64 MiB (moco_align serves such frames). */
int moco_align_noalloc(moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m,
                       int n, int w, int downsample, moco_dtype dtype, moco_form form,
                       const moco_outputs *out, void *hip_stream);

/* A moco_align call captured as a HIP graph, for callers that repeat the same
 * call (a frame buffer refilled between calls: a camera, a serving loop):
 * replaying it aligns whatever d_frames holds when the replay runs into the
 * same outputs, with one launch instead of one per kernel.  The graph has its
 * own scratch (the size moco_align would use, allocated here); it refers to
 * d_frames, the template and the outputs, which must outlive it.  The
 * arguments and errors are moco_align's (T >= 1); the call is captured on a
 * stream of its own, with stage timing off, and nothing runs until a launch. */
typedef struct moco_graph moco_graph;
int moco_graph_create(moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m,
                      int n, int w, int downsample, moco_dtype dtype, moco_form form,
                      const moco_outputs *out, moco_graph **graph);

/* Replay the captured call on hip_stream (ordered after work enqueued there
 * before).  Replays on one graph share its scratch: enqueue them on one stream
 * or synchronise between them.  Errors: MOCO_EINVAL, MOCO_EDEVICE. */
int moco_graph_launch(moco_graph *graph, void *hip_stream);

/* Release a graph.  Safe on NULL.  Its replays must have completed. */
void moco_graph_destroy(moco_graph *graph);

/* One stack of a batch: moco_align's arguments as a record. */
typedef struct {
    const void *d_frames;
    const moco_tmpl *tmpl;
    int T, m, n, w, downsample;
    moco_dtype dtype;
    moco_outputs out;
} moco_stack;

/* Align a batch of stacks of uneven length, size and window (each frame of each
 * stack exactly as moco_align would: the search of sec. 2, every frame
 * independent of the others).  Work is ordered after everything enqueued on
 * `hip_stream` before the call, and everything enqueued on it afterwards waits
 * for the whole batch.  Internally the stacks run longest-first on up to
 * `lanes` streams of the context (0: the library's choice, at most 8), each
 * with its own slice of the context's scratch budget; results do not depend on
 * the lanes, the order or the chunking.  All stacks are validated before any
 * work is enqueued (MOCO_EINVAL names the first bad stack); `form` applies to
 * every stack (MOCO_FORM_AUTO resolves per stack).  Errors: MOCO_EINVAL,
 * MOCO_ENOMEM (a slice cannot hold one frame of some stack), MOCO_EDEVICE. */
int moco_align_batch(moco_ctx *ctx, const moco_stack *stacks, int nstacks, moco_form form,
                     int lanes, void *hip_stream);

/* moco_align_batch captured as one HIP graph, for callers that repeat the same
 * batch (buffers refilled between calls): the stacks' launch sequences, spread
 * over `lanes` streams as moco_align_batch spreads them (forked from and
 * joined to one origin inside the capture), replay with a single launch
 * (moco_graph_launch) over whatever the frame buffers then hold, into the
 * same outputs.  The graph has its own scratch (lanes x the slice
 * moco_align_batch would use, allocated here) and captures on streams of its
 * own, with stage timing off; it refers to every stack's frames, template and
 * outputs, which must outlive it.  Arguments and errors are
 * moco_align_batch's; a batch with no frame is MOCO_EINVAL.  Release with
 * moco_graph_destroy. */
int moco_graph_create_batch(moco_ctx *ctx, const moco_stack *stacks, int nstacks, moco_form form,
                            int lanes, moco_graph **graph);

/* Apply the correction (sec. 2: each frame moved by the translation found for
 * it is the motion-corrected video; sec. 3, fig. 1 and 2: corrected frames are
 * black outside their overlap with the template, and the mean of the
 * corrected video is the check of a correction).
 *
 * d_frames: T x m x n row-major (device, `dtype`), d_shifts: T x 2 int32 (S,T)
 * per frame (device; any values, typically moco_outputs.shifts).  d_out
 * (device, nullable): T x m x n of `dtype`, out[k][i][j] = frame_k[i+S][j+T]
 * when 0 <= i+S < m and 0 <= j+T < n, else 0; it must not overlap d_frames.
 * d_mean (device, nullable): m x n FP64, the mean over the T corrected frames
 * (sums in frame order within chunks, chunks in order; for uint16 data every
 * sum is exact and the mean is the correctly rounded quotient).  At least one
 * of d_out, d_mean.  The mean's partial sums (up to 32 x m x n FP64) use the
 * context's scratch.  Enqueued on hip_stream; T = 0 is a no-op.
 * Errors: MOCO_EINVAL, MOCO_ENOMEM (one m x n FP64 plane exceeds the budget),
 * MOCO_EDEVICE. */
int moco_apply(moco_ctx *ctx, const void *d_frames, const int32_t *d_shifts, int T, int m, int n,
               moco_dtype dtype, void *d_out, double *d_mean, void *hip_stream);

/* The correlation form a call with `requested` runs for this template.
 * MOCO_FORM_INT8_MFMA applies to uint16 templates with a searched grid of fewer
 * than 131072 pixels and at most 2048 columns, w <= 512, and grid values within
 * two balanced base-256 digits (|value| <= 32639); the four FFT forms apply
 * when the transform lengths (5-smooth, at least m'+w-1 by n'+w-1) are at most
 * 2048.  MOCO_FORM_AUTO resolves to a form recorded for the key where it
 * applies; else, for uint16 data, to whichever of MOCO_FORM_INT8_MFMA and
 * MOCO_FORM_FFT_CERTIFIED applies, the one a per-frame time model ranks faster
 * when both do (the int8 form's work grows with the (2w-1)^2 shifts, the FFT's
 * with P Q log(P Q): at a 256x256 grid the int8 form for w <= 32, the FFT
 * above); for float32 data to MOCO_FORM_FFT32_CERTIFIED; else to
 * MOCO_FORM_FP64_EXACT.
 * Errors: MOCO_EINVAL (null argument, or an explicit form that does not apply). */
int moco_template_form(const moco_tmpl *tmpl, moco_form requested, moco_form *resolved);

/* ---- Form choice by measurement ------------------------------------------
 *
 * MOCO_FORM_AUTO resolves through a per-process table of forms keyed by
 * (m, n, w, downsample, dtype): a form recorded for a template's key is used
 * when it applies to the template; otherwise the time model described at
 * moco_template_form decides.  The table starts empty, so AUTO is the model's
 * choice until a form is tuned or set. */

/* Time the forms that apply to `tmpl` (of MOCO_FORM_INT8_MFMA,
 * MOCO_FORM_FFT_CERTIFIED and, for float32 data, MOCO_FORM_FFT32_CERTIFIED;
 * MOCO_FORM_FP64_EXACT when none does) on `frames` copies of the template, one
 * warm-up and three timed calls each with HIP events on hip_stream, and record
 * the fastest for the template's key.  The int8 form is timed with each of its
 * shift-tile shapes that applies (two 16x16 tiles in one 32x32 product when
 * 2w-1 <= 16, one 32x32 tile per block, or 2x2 tiles of 32 when 2w-1 > 32)
 * and keeps the fastest for the key and for launches of
 * that size class (at most 64 frames, or more) whichever form wins
 * (moco_template_int8_tile).  The forms rank differently with the stack length
 * (a few frames take the int8 form's row-sliced launch), so `frames` should be
 * the length of the stacks the key will serve; 0 means 1024, the many-frame
 * regime.  *chosen receives the form; seconds_per_frame (nullable,
 * MOCO_FORM_COUNT doubles indexed by moco_form) receives each timed form's
 * seconds per frame, the int8 form's with its faster tile (-1 for forms not
 * timed).  Synchronises hip_stream; allocates the frames outside the context's
 * budget for the duration of the call.
 * Errors: MOCO_EINVAL, MOCO_ENOMEM, MOCO_EDEVICE. */
int moco_tune(moco_ctx *ctx, const moco_tmpl *tmpl, int frames, void *hip_stream,
              moco_form *chosen, double *seconds_per_frame);

/* Record `form` (a concrete form, not AUTO) for the key, e.g. from a saved
 * table of earlier measurements.  Host only.  Errors: MOCO_EINVAL. */
int moco_tune_set(int m, int n, int w, int downsample, moco_dtype dtype, moco_form form);

/* The form recorded for the key.  Errors: MOCO_EINVAL (none recorded). */
int moco_tune_get(int m, int n, int w, int downsample, moco_dtype dtype, moco_form *form);

/* Record the int8 form's shift tile for the key (uint16 data), for launches
 * of any size: 16 (two 16x16 tiles on the diagonal of one 32x32 MFMA product,
 * over the two halves of each 128-column strip; only when 2w-1 <= 16), 32
 * (one 32x32 tile per block, ceil((2w-1)/32)^2 blocks per frame) or 64 (2x2
 * tiles of 32, ceil((2w-1)/64)^2 blocks; not when 2w-1 <= 32).  Without a
 * recorded tile the form takes 16 when 2w-1 <= 16 and the template takes
 * three digit products, else 32 when 2w-1 <= 32, or when 2w-1 <= 64 and a
 * launch holds at most 64 frames; else 64.  All give the same exact results.
 * Host only.  Errors: MOCO_EINVAL. */
int moco_tune_set_tile(int m, int n, int w, int downsample, moco_dtype dtype, int tile);

/* Forget every recorded form and tile. */
void moco_tune_clear(void);

/* Error bound of the FFT forms for this template (sec. 2, the FFT construction
 * of h, evaluated in FP64): for every shift of the window the computed
 * correlation h^ satisfies |h^ - h| <= kf * sqrt(m' n' Sa Sb), and each
 * computed overlap energy is within ke * Sa (frame) or ke * Sb (template),
 * where Sa, Sb are the sums of squares of the searched grids of the frame and
 * the template.  These are the coefficients MOCO_FORM_FFT_CERTIFIED's
 * certificate uses: a first-order bound in the unit roundoff for each
 * transform pass, doubled.  Host only.
 * Errors: MOCO_EINVAL (null argument, or the FFT form does not apply). */
int moco_template_fft_bound(const moco_tmpl *tmpl, double *kf, double *ke);

/* Digit products per correlation term in the int8 form's main pass for this
 * template (sec. 2, definition of h, evaluated exactly): 3 when two balanced
 * base-128 digits hold every value of the template's searched grid (at most
 * 8127) and its Toeplitz rows fit the kernel's buffers -- the products d0 e0,
 * d1 e1 and (d0 + d1)(e0 + e1) -- else 4 (two base-256 digits each side).
 * Frames with a grid value beyond two digits take two more products in a
 * second pass.  Host only.
 * Errors: MOCO_EINVAL (null argument, or the int8 form does not apply). */
int moco_template_int8_products(const moco_tmpl *tmpl, int *products);

/* The shift tile (16, 32 or 64) the int8 form uses for this template's key now,
 * in launches of more than 64 frames: the recorded one, else the model's.
 * Host only.
 * Errors: MOCO_EINVAL (null argument, or the int8 form does not apply). */
int moco_template_int8_tile(const moco_tmpl *tmpl, int *tile);

/* ---- Serving: single frames from many sources, continuous batching ----
 *
 * A server owns its own context on the device of `ctx`, a pool of `max_slots`
 * request slots (pinned host staging plus device space for two batches in
 * flight) and the prepared template of each source, resident on the device.
 * Requests are single host frames; a worker thread takes every request waiting
 * when the GPU can accept a batch (up to max_slots), runs the search of sec. 2 on
 * the batch (frames of one source share a launch), and publishes one result per
 * request.  Requests that arrive while batches are on the GPU are admitted as
 * slots free up and go in the next batch.  A source runs the form AUTO
 * resolves to for its template, except that float32 sources run
 * MOCO_FORM_FFT_CERTIFIED (the certified FP32 form is not served); each
 * frame's result is exactly what moco_align gives for that frame alone in
 * that form.  All server calls are thread-safe. */
typedef struct moco_server moco_server;

typedef struct {
    uint64_t tag;          /* the caller's tag from moco_server_submit */
    int source;            /* the source id */
    int status;            /* MOCO_OK, MOCO_EDEVICE, or MOCO_ECANCELED */
    int32_t shift[2];      /* final (S,T) */
    int32_t coarse[2];     /* argmin on the searched grid */
    double fmin;           /* f at the coarse argmin */
    double frefine[9];     /* nine full-resolution values (NaN when not downsampled) */
    double gaps[2];        /* as moco_outputs.gaps */
    double latency_us;     /* submit -> result published */
} moco_result;

/* Create a server.  device_budget_bytes caps the device memory it may hold (0 =
 * 1 GiB); max_slots (>= 1) caps the requests admitted at once.
 * Errors: MOCO_EINVAL, MOCO_ENOMEM, MOCO_EDEVICE. */
int moco_server_create(moco_ctx *ctx, size_t device_budget_bytes, int max_slots,
                       moco_server **out);

/* Register a source and prepare its template (host memory, m x n of dtype,
 * copied during the call).  Source ids are any int, unique per server.
 * Errors: MOCO_EINVAL (bad geometry, duplicate id), MOCO_ENOMEM (the slots for
 * this frame size do not fit the device budget), MOCO_EDEVICE. */
int moco_server_add_source(moco_server *srv, int source, const void *h_template,
                           moco_dtype dtype, int m, int n, int w, int downsample);

/* Submit one frame (host memory of the source's size and dtype, copied during
 * the call).  When no batch is in flight the call also enqueues the batch
 * (this request and any others waiting) itself, instead of waking the worker
 * thread.  Returns MOCO_OK when admitted, MOCO_EBUSY when no slot is free
 * (back-pressure: poll, then retry), MOCO_EINVAL for an unknown source. */
int moco_server_submit(moco_server *srv, int source, const void *h_frame, uint64_t tag);

/* Wait up to timeout_us (0: do not wait, < 0: wait without limit) for finished
 * requests and copy up to `max` results into `results` (host), oldest first.
 * The first millisecond of a wait polls (yielding the core) rather than
 * sleeping.  Returns the number copied (>= 0) or a negative status. */
int moco_server_poll(moco_server *srv, moco_result *results, int max, int timeout_us);

/* Requests admitted and not yet published (queued or on the GPU). */
int moco_server_pending(moco_server *srv);

/* Stop the server: requests not yet on the GPU are cancelled, batches on the
 * GPU finish, then everything is freed.  Results not polled are dropped.
 * Returns the number of cancelled requests.  Safe on NULL (returns 0). */
int moco_server_destroy(moco_server *srv);

/* Stage timing (tracing).  Stages of the pipeline, in launch order. */
typedef enum {
    MOCO_STAGE_COARSE = 0,   /* 2x2 box mean / conversion of the frames */
    MOCO_STAGE_ENERGY = 1,   /* overlap energies of the frames */
    MOCO_STAGE_PREP = 2,     /* int8 form: limb split of the frames */
    MOCO_STAGE_CORR = 3,     /* cross-correlation h */
    MOCO_STAGE_COMBINE = 4,  /* f = (A+B-2h)/Area, argmin, gap */
    MOCO_STAGE_REFINE = 5,   /* nine full-resolution evaluations */
    MOCO_STAGE_APPLY = 6,    /* moco_apply: corrected frames and mean image */
    MOCO_STAGE_COUNT = 7
} moco_stage;

/* Turn stage timing on (1) or off (0) for a context.  While on, every stage
 * kernel launch is bracketed by a pair of HIP events recorded on the stream it
 * is launched on.  Errors: MOCO_EINVAL (null ctx). */
int moco_profile_enable(moco_ctx *ctx, int enable);

/* Wait for the recorded events, add their durations into ms[MOCO_STAGE_COUNT]
 * (milliseconds) and launches[MOCO_STAGE_COUNT] (kernel launches), and clear
 * the record.  Arrays are host memory of MOCO_STAGE_COUNT elements, filled
 * (not accumulated).  Errors: MOCO_EINVAL, MOCO_EDEVICE. */
int moco_profile_read(moco_ctx *ctx, double *ms, int64_t *launches);

/* The paper's default parameters for an m x n stack (sec. 3): downsample once
 * when the frame is larger than 256x256 (a side above 256), else not at all,
 * and the window w = min(m',n')/3 (floor, at least 1) on the searched grid.
 * Host only.  Errors: MOCO_EINVAL (m or n < 1, null outputs). */
int moco_default_params(int m, int n, int *w, int *downsample);

/* Human-readable message of the calling thread's last failure ("" if none). */
const char *moco_last_error(void);

/* Library version string. */
const char *moco_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MOCO_H */
