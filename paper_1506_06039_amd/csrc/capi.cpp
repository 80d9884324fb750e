// C ABI of the translation-search library: validation, context and scratch,
// resident templates, and the per-stack pipeline that enqueues the stage
// kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "moco_internal.h"

struct ProfRec {
    int stage;
    hipEvent_t a, b;
};

struct moco_ctx {
    int device = 0;
    size_t budget = 0;
    void *scratch = nullptr;
    size_t scratch_size = 0;
    void *fixed_scratch = nullptr;    // this device's copy of the allocation-free scratch
    bool profiling = false;
    std::vector<ProfRec> prof;        // recorded, not yet read
    std::vector<hipEvent_t> ev_pool;  // reusable events
    std::vector<hipStream_t> lanes;   // internal streams of moco_align_batch (default priority)
    std::vector<hipEvent_t> lane_ev;  // one join event per lane, plus one fork event
};

struct moco_tmpl {
    int device = 0;     // its own copy: a template may outlive the context that made it
    moco::Tmpl t{};
};

struct moco_graph {
    int device = 0;
    void *scratch = nullptr;        // its own: the context's scratch may be reallocated
    hipGraphExec_t exec = nullptr;
};

// Scratch of moco_align_noalloc: a module-scope device array, so that the
// entry point needs no allocation.  Each device the library runs on holds its
// own instance, from the first context created on it until the process ends.
// In host code `scratch` names a host-side stand-in; its device address on the
// current device comes from hipGetSymbolAddress (fixed_scratch_address).
constexpr size_t kFixedScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kFixedScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(MOCO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device address of `scratch` on each device, looked up once per device with
// that device current (each device holds the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {};

int fixed_scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (device < 0 || device >= kMaxDevices)
        return fail(MOCO_EINVAL, "device %d beyond the %d the library tracks", device, kMaxDevices);
    if (!g_fixed_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MOCO_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                        hipGetErrorString(e));
        g_fixed_ptr[device] = p;
    }
    *out = g_fixed_ptr[device];
    return MOCO_OK;
}

// Validation shared by template creation and alignment.
int validate(int m, int n, int w, int ds, moco_dtype dt, moco::Geom *g)
{
    if (dt != MOCO_U16 && dt != MOCO_F32) return fail(MOCO_EINVAL, "unknown dtype %d", (int)dt);
    if (ds < 0 || ds > moco::kMaxLevels)
        return fail(MOCO_EINVAL, "downsample (levels) must be 0..%d, got %d", moco::kMaxLevels, ds);
    if (m < 1 || n < 1) return fail(MOCO_EINVAL, "image size %dx%d must be positive", m, n);
    if ((m >> ds) < 1 || (n >> ds) < 1)
        return fail(MOCO_EINVAL, "%d levels of downsampling need m,n >= %d (got %dx%d)", ds,
                    1 << ds, m, n);
    int mg = m >> ds, ng = n >> ds;
    if (w < 1 || w > mg || w > ng)
        return fail(MOCO_EINVAL, "window w=%d must satisfy 1 <= w <= min(%d,%d)", w, mg, ng);
    if ((long long)m * n > (1LL << 30)) return fail(MOCO_EINVAL, "image %dx%d too large", m, n);
    if (2 * w - 1 > 1024) return fail(MOCO_EINVAL, "window w=%d too large (max 512)", w);
    g->m = m;
    g->n = n;
    g->mg = mg;
    g->ng = ng;
    g->w = w;
    g->W = 2 * w - 1;
    g->ds = ds;
    g->dtype = dt;
    return MOCO_OK;
}

size_t dtype_size(moco_dtype dt) { return dt == MOCO_U16 ? 2 : 4; }

// Ensure the context holds at least `bytes` of scratch.  Growing frees the old
// block only after the stream has drained it.
int ensure_scratch(moco_ctx *ctx, size_t bytes, hipStream_t st)
{
    if (bytes <= ctx->scratch_size) return MOCO_OK;
    if (bytes > ctx->budget)
        return fail(MOCO_ENOMEM, "scratch of %zu bytes exceeds the context budget %zu", bytes,
                    ctx->budget);
    if (ctx->scratch) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_size = 0;
    }
    hipError_t e = hipMalloc(&ctx->scratch, bytes);
    if (e != hipSuccess) {
        ctx->scratch = nullptr;
        return fail(MOCO_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    ctx->scratch_size = bytes;
    return MOCO_OK;
}

// Geometry of pyramid level l (0 = the frames) of a search.
moco::Geom level_geom(const moco::Geom &g, int l)
{
    moco::Geom q = g;
    q.ds = l;
    q.mg = g.m >> l;
    q.ng = g.n >> l;
    return q;
}

// FP64 elements of levels 1 .. ds-1 of one frame's pyramid (the levels the
// intermediate x2 steps read).
size_t inter_elems(const moco::Geom &g)
{
    size_t e = 0;
    for (int l = 1; l < g.ds; ++l) e += (size_t)(g.m >> l) * (g.n >> l);
    return e;
}

// The searched grid of C frames into `grid` (level ds; the frames in FP64
// when ds = 0) and, when ds >= 2, levels 1 .. ds-1 into `inter` (level by
// level, each C x m_l x n_l).
hipError_t build_levels(const void *frames, moco_dtype dt, int C, const moco::Geom &g,
                        double *inter, double *grid, hipStream_t st)
{
    if (g.ds <= 1) return moco::launch_coarse(frames, dt, C, g, grid, st);
    hipError_t e = moco::launch_coarse(frames, dt, C, level_geom(g, 1), inter, st);
    double *prev = inter;
    size_t off = (size_t)C * (g.m >> 1) * (g.n >> 1);
    for (int l = 2; l <= g.ds && e == hipSuccess; ++l) {
        double *out = l == g.ds ? grid : inter + off;
        e = moco::launch_half(prev, C, g.m >> (l - 1), g.n >> (l - 1), out, st);
        prev = out;
        off += (size_t)C * (g.m >> l) * (g.n >> l);
    }
    return e;
}

// Level l (1 <= l < ds) of the chunk's pyramid, and of the template's.
double *inter_level(double *inter, int C, const moco::Geom &g, int l)
{
    size_t off = 0;
    for (int k = 1; k < l; ++k) off += (size_t)C * (g.m >> k) * (g.n >> k);
    return inter + off;
}

// The x2 steps above full resolution: from the searched grid's argmin `cst`
// down to level 1; returns the level-1 result (cst itself when ds <= 1).
// shA, shB: C x 2 int32 each; partial: the level refine's partial sums.
hipError_t refine_levels(const moco::Tmpl &tt, int C, const moco::Geom &g, double *inter,
                         const int32_t *cst, int32_t *shA, int32_t *shB, double *partial,
                         hipStream_t st, const int32_t **level1)
{
    const int32_t *cur = cst;
    for (int l = g.ds - 1; l >= 1; --l) {
        int32_t *out = (g.ds - 1 - l) % 2 == 0 ? shA : shB;
        hipError_t e = moco::launch_refine_level(inter_level(inter, C, g, l),
                                                 inter_level(tt.pyr, 1, g, l), C, g.m >> l,
                                                 g.n >> l, cur, out, partial, st);
        if (e != hipSuccess) return e;
        cur = out;
    }
    *level1 = cur;
    return hipSuccess;
}

// Partial sums of every refine step of a search, per frame.
size_t refine_steps_partial_bytes(const moco::Geom &g)
{
    size_t b = moco::refine_partial_bytes(g);
    for (int l = 1; l < g.ds; ++l) b = std::max(b, moco::refine_level_partial_bytes(g.m >> l, g.n >> l));
    return b;
}

// Per-frame scratch of the energy kernels: the uint16 prep kernel's integer
// border tables (0 where it does not apply).
size_t energy_scratch_bytes(const moco::Geom &g)
{
    return moco::prep_grid_applicable(g) ? moco::prep_edge_bytes(g) : 0;
}

// Per-frame scratch of the FP64 exact form.
struct ExactLayout {
    size_t coarse, inter, atab, h, cst, pm, edge, part, total_per_frame;
};

ExactLayout exact_layout(const moco::Geom &g)
{
    ExactLayout L;
    L.coarse = align_up((size_t)g.mg * g.ng * sizeof(double), 256);
    L.inter = align_up(inter_elems(g) * sizeof(double), 256);
    L.atab = align_up((size_t)g.W * g.W * sizeof(double), 256);
    L.h = align_up((size_t)g.W * g.W * sizeof(double), 256);
    L.cst = 3 * 2 * sizeof(int32_t);   // the searched grid's argmin, two x2-step buffers
    L.pm = 2 * sizeof(int32_t);         // padded: the partials after it stay 8-byte aligned
    L.edge = align_up(energy_scratch_bytes(g), 256);
    L.part = align_up(refine_steps_partial_bytes(g), 8);
    L.total_per_frame = L.coarse + L.inter + L.atab + L.h + L.cst + L.pm + L.edge + L.part;
    return L;
}

class DeviceGuard {
public:
    explicit DeviceGuard(int dev)
    {
        ok_ = hipGetDevice(&prev_) == hipSuccess;
        if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

private:
    int prev_ = 0;
    bool ok_ = false;
};

hipEvent_t pool_event(moco_ctx *ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one stage launch with events when profiling is on.
class StageTimer {
public:
    StageTimer(moco_ctx *ctx, int stage, hipStream_t st) : ctx_(ctx), st_(st)
    {
        if (!ctx->profiling) return;
        rec_.stage = stage;
        rec_.a = pool_event(ctx);
        rec_.b = pool_event(ctx);
        if (rec_.a && rec_.b && hipEventRecord(rec_.a, st) == hipSuccess) on_ = true;
    }
    ~StageTimer()
    {
        if (on_ && hipEventRecord(rec_.b, st_) == hipSuccess) ctx_->prof.push_back(rec_);
    }

private:
    moco_ctx *ctx_;
    hipStream_t st_;
    ProfRec rec_{};
    bool on_ = false;
};

// The searched grid and its overlap energies: uint16 frames with at most one
// level in one pass over the raw frames, else the FP64 pyramid and k_energy.
hipError_t grid_and_energies(moco_ctx *ctx, const void *fr, const moco::Geom &g, int c,
                             double *inter, double *coarse, double *atab, int32_t *pm,
                             long long *edge, hipStream_t st)
{
    if (edge && moco::prep_grid_applicable(g)) {
        StageTimer tm(ctx, MOCO_STAGE_PREP, st);
        return moco::launch_prep_grid((const uint16_t *)fr, c, g, coarse, atab, pm, edge, st);
    }
    hipError_t e;
    {
        StageTimer tm(ctx, MOCO_STAGE_COARSE, st);
        if ((e = build_levels(fr, g.dtype, c, g, inter, coarse, st)) != hipSuccess) return e;
    }
    StageTimer tm(ctx, MOCO_STAGE_ENERGY, st);
    return moco::launch_energy(coarse, c, g, false, atab, pm, st);
}

void free_tmpl(moco::Tmpl &t)
{
    if (t.raw) (void)hipFree(t.raw);
    if (t.coarse) (void)hipFree(t.coarse);
    if (t.btab) (void)hipFree(t.btab);
    if (t.i8.tp) (void)hipFree(t.i8.tp);
    if (t.i8.atab) (void)hipFree(t.i8.atab);
    if (t.fft.twp) (void)hipFree(t.fft.twp);
    if (t.fft.twq) (void)hipFree(t.fft.twq);
    if (t.fft.spec) (void)hipFree(t.fft.spec);
    if (t.fft.twp32) (void)hipFree(t.fft.twp32);
    if (t.fft.twq32) (void)hipFree(t.fft.twq32);
    if (t.fft.spec32) (void)hipFree(t.fft.spec32);
    if (t.fft.btab32) (void)hipFree(t.fft.btab32);
    if (t.pyr) (void)hipFree(t.pyr);
    t.fft.twp32 = t.fft.twq32 = t.fft.spec32 = nullptr;
    t.fft.btab32 = nullptr;
    t.pyr = nullptr;
    t.fft.twp = nullptr;
    t.fft.twq = nullptr;
    t.fft.spec = nullptr;
    t.raw = nullptr;
    t.coarse = nullptr;
    t.btab = nullptr;
    t.i8.tp = nullptr;
    t.i8.atab = nullptr;
}

// Most frames one launch sequence processes (a chunk); larger stacks run in
// chunks of at most this many frames, so scratch beyond it is never used.
constexpr int kChunkInt8 = 8192;
constexpr int kChunkOther = 4096;   // FFT and FP64 forms

// Per-frame scratch of the int8 form.
struct Int8Layout {
    size_t limbs, nlimb, atab, edge, h, cst, part, total_per_frame;
};

Int8Layout int8_layout(const moco::Geom &g, int npad)
{
    Int8Layout L;
    L.limbs = align_up((size_t)3 * g.mg * npad, 256);
    L.nlimb = 256;
    L.atab = align_up((size_t)g.W * g.W * sizeof(long long), 256);
    L.edge = align_up(moco::prep_edge_bytes(g), 256);
    L.h = align_up((size_t)g.W * g.W * sizeof(long long), 256);
    L.cst = 2 * sizeof(int32_t);
    L.part = align_up(moco::refine_partial_bytes(g), 8);
    L.total_per_frame = L.limbs + L.nlimb + L.atab + L.edge + L.h + L.cst + L.part;
    return L;
}

// Prepare the template side of the int8 form: digit planes, Toeplitz rows and
// the exact energy table.  Base-128 digits with a digit-sum plane (three
// products per term) when two such digits hold every template value and the
// rows fit the kernel's buffers, else base-256 digits (four products); leaves
// t.int8_ok false when the template needs a third base-256 digit.
int prepare_int8_template(moco::Tmpl &t, hipStream_t st)
{
    const moco::Geom &g = t.g;
    t.int8_ok = false;
    if (!moco::int8_applicable(g)) return MOCO_OK;
    moco::Int8Geom ig = moco::int8_geom(g);
    Int8Layout L = int8_layout(g, ig.npad);
    char *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, L.total_per_frame);
    if (e != hipSuccess) return fail(MOCO_ENOMEM, "template scratch: %s", hipGetErrorString(e));
    int8_t *limbs = (int8_t *)tmp;
    int32_t *nl = (int32_t *)(tmp + L.limbs);
    int32_t *vm = nl + 1;
    long long *atab = (long long *)(tmp + L.limbs + L.nlimb);
    long long *edge = (long long *)(tmp + L.limbs + L.nlimb + L.atab);
    int32_t nlimb = 0;
    int rc = MOCO_OK;
    t.i8.npad = ig.npad;
    t.i8.padl = ig.padl;
    t.i8.trow = ig.trow;
    int32_t vmaxv = 0;
    for (int dbits = ig.trow <= moco::kInt8SumMaxTrow ? 7 : 8; dbits <= 8; ++dbits) {
        t.i8.dbits = dbits;
        t.i8.nq = dbits == 7 ? 3 : 2;
        if ((e = moco::launch_prep_u16((const uint16_t *)t.raw, 1, g, ig.npad, dbits, limbs, nl,
                                       vm, atab, edge, st)) != hipSuccess ||
            (e = hipMemcpyAsync(&nlimb, nl, sizeof nlimb, hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(&vmaxv, vm, sizeof vmaxv, hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            rc = fail(MOCO_EDEVICE, "int8 template preparation: %s", hipGetErrorString(e));
            break;
        }
        if (nlimb == 2) break;
    }
    if (rc == MOCO_OK && nlimb == 2) {
        const size_t tbytes = moco::int8_template_bytes(g, t.i8.nq);
        if ((e = hipMalloc(&t.i8.tp, tbytes)) != hipSuccess ||
            (e = hipMalloc(&t.i8.atab, (size_t)g.W * g.W * sizeof(long long))) != hipSuccess) {
            rc = fail(MOCO_ENOMEM, "int8 template allocation: %s", hipGetErrorString(e));
        } else if ((e = moco::launch_tpad(limbs, g, t.i8, st)) != hipSuccess ||
                   (e = hipMemsetAsync(t.i8.tp + tbytes - moco::kInt8ZeroTail,
                                       0, moco::kInt8ZeroTail, st)) != hipSuccess ||
                   (e = hipMemcpyAsync(t.i8.atab, atab, (size_t)g.W * g.W * sizeof(long long),
                                       hipMemcpyDeviceToDevice, st)) != hipSuccess ||
                   (e = hipStreamSynchronize(st)) != hipSuccess) {
            rc = fail(MOCO_EDEVICE, "int8 template preparation: %s", hipGetErrorString(e));
        } else {
            t.int8_ok = true;
            t.i8.vmax = vmaxv == INT32_MAX ? -1 : vmaxv;
        }
    }
    (void)hipFree(tmp);
    return rc;
}

// Twiddle table w_n^k = exp(-2 pi i k/n), k < n, rounded from long double.
int upload_twiddles(int n, double2 **dst)
{
    std::vector<double2> h((size_t)n);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < n; ++k) {
        const long double a = two_pi * (long double)k / (long double)n;
        h[(size_t)k] = double2{(double)cosl(a), (double)-sinl(a)};
    }
    hipError_t e = hipMalloc(dst, (size_t)n * sizeof(double2));
    if (e == hipSuccess) e = hipMemcpy(*dst, h.data(), (size_t)n * sizeof(double2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MOCO_ENOMEM, "FFT twiddle table: %s", hipGetErrorString(e));
    return MOCO_OK;
}

// The same table rounded to FP32 (from the long double values).
int upload_twiddles32(int n, float2 **dst)
{
    std::vector<float2> h((size_t)n);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < n; ++k) {
        const long double a = two_pi * (long double)k / (long double)n;
        h[(size_t)k] = float2{(float)cosl(a), (float)-sinl(a)};
    }
    hipError_t e = hipMalloc(dst, (size_t)n * sizeof(float2));
    if (e == hipSuccess) e = hipMemcpy(*dst, h.data(), (size_t)n * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MOCO_ENOMEM, "FFT twiddle table: %s", hipGetErrorString(e));
    return MOCO_OK;
}

// The single-precision form's template side: the offset c (the mean of the
// template's grid, rounded to an integer for uint16 data so that centred
// uint16 grids stay exact in FP32), the energies of b' - c, and the transform
// of the zero-padded b' - c, computed in FP64 and rounded to FP32.
int prepare_fft32_template(moco::Tmpl &t, hipStream_t st)
{
    const moco::Geom &g = t.g;
    moco::FftTmpl &f = t.fft;
    const size_t ne = (size_t)g.mg * g.ng;
    std::vector<double> grid(ne);
    hipError_t e = hipMemcpyAsync(grid.data(), t.coarse, ne * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(MOCO_EDEVICE, "FFT32 template: %s", hipGetErrorString(e));
    long double acc = 0.0L;
    for (double v : grid) acc += v;
    const double mean = (double)(acc / (long double)ne);
    f.center = g.dtype == MOCO_U16 ? std::nearbyint(mean) : mean;
    for (double &v : grid) v -= f.center;
    int rc = upload_twiddles32(f.pp.n, &f.twp32);
    if (!rc) rc = upload_twiddles32(f.pq.n, &f.twq32);
    if (rc) return rc;
    const size_t nspec = (size_t)f.qh * f.pp.n;
    double *dgrid = nullptr;
    double2 *s1 = nullptr, *spec = nullptr;
    std::vector<double2> hspec(nspec);
    std::vector<float2> hspec32(nspec);
    if ((e = hipMalloc(&f.btab32, (size_t)g.W * g.W * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&f.spec32, nspec * sizeof(float2))) != hipSuccess ||
        (e = hipMalloc(&dgrid, ne * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&s1, moco::fft_s1_bytes(g))) != hipSuccess ||
        (e = hipMalloc(&spec, nspec * sizeof(double2))) != hipSuccess) {
        rc = fail(MOCO_ENOMEM, "FFT32 template allocation: %s", hipGetErrorString(e));
    } else if ((e = moco::launch_energy(t.coarse, 1, g, true, f.btab32, nullptr, st,
                                        f.center)) != hipSuccess ||
               (e = hipMemcpyAsync(dgrid, grid.data(), ne * sizeof(double),
                                   hipMemcpyHostToDevice, st)) != hipSuccess ||
               (e = moco::launch_fft_rows(dgrid, 1, g, f, s1, st)) != hipSuccess ||
               (e = moco::launch_fft_spec(s1, g, f, spec, st)) != hipSuccess ||
               (e = hipMemcpyAsync(hspec.data(), spec, nspec * sizeof(double2),
                                   hipMemcpyDeviceToHost, st)) != hipSuccess ||
               (e = hipStreamSynchronize(st)) != hipSuccess) {
        rc = fail(MOCO_EDEVICE, "FFT32 template preparation: %s", hipGetErrorString(e));
    } else {
        double ymax = 0.0;
        for (size_t k = 0; k < nspec; ++k) {
            hspec32[k] = float2{(float)hspec[k].x, (float)hspec[k].y};
            const double yx = hspec32[k].x, yy = hspec32[k].y;
            ymax = std::max(ymax, std::sqrt(yx * yx + yy * yy));
        }
        f.yinf32 = ymax * (1.0 + 0x1p-50);
        e = hipMemcpy(f.spec32, hspec32.data(), nspec * sizeof(float2), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(MOCO_EDEVICE, "FFT32 template: %s", hipGetErrorString(e));
    }
    if (dgrid) (void)hipFree(dgrid);
    if (s1) (void)hipFree(s1);
    if (spec) (void)hipFree(spec);
    return rc;
}

// Prepare the template side of the FFT form: plans, twiddles and the 2-D
// transform of the zero-padded b'.  Leaves t.fft_ok false when the transform
// lengths exceed the supported maximum.
int prepare_fft_template(moco::Tmpl &t, hipStream_t st)
{
    const moco::Geom &g = t.g;
    t.fft_ok = false;
    if (!moco::fft_applicable(g)) return MOCO_OK;
    const moco::FftGeom fg = moco::fft_geom(g);
    moco::FftTmpl &f = t.fft;
    if (!moco::fft_plan(fg.P, &f.pp) || !moco::fft_plan(fg.Q, &f.pq))
        return fail(MOCO_EINVAL, "no FFT plan for %dx%d", fg.P, fg.Q);
    f.qh = fg.qh;
    int rc = upload_twiddles(fg.P, &f.twp);
    if (!rc) rc = upload_twiddles(fg.Q, &f.twq);
    if (rc) return rc;
    double2 *s1 = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&f.spec, (size_t)fg.qh * fg.P * sizeof(double2))) != hipSuccess ||
        (e = hipMalloc(&s1, moco::fft_s1_bytes(g))) != hipSuccess) {
        if (s1) (void)hipFree(s1);
        return fail(MOCO_ENOMEM, "FFT template allocation: %s", hipGetErrorString(e));
    }
    if ((e = moco::launch_fft_rows(t.coarse, 1, g, f, s1, st)) != hipSuccess ||
        (e = moco::launch_fft_spec(s1, g, f, f.spec, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        (void)hipFree(s1);
        return fail(MOCO_EDEVICE, "FFT template preparation: %s", hipGetErrorString(e));
    }
    (void)hipFree(s1);
    int rc32 = prepare_fft32_template(t, st);
    if (rc32) return rc32;
    t.fft_ok = true;
    return MOCO_OK;
}

// The int8 correlation's shift tile for a template's key: a tile recorded by
// moco_tune (or moco_tune_set_tile), else the model's (int8_model_tile).
int int8_tile(const moco::Tmpl &t, int C);

// The int8 pipeline over one stack, in chunks that fit `sbytes` of scratch at
// `sbase`; every launch goes to stream st.
int run_int8(moco_ctx *ctx, const void *d_frames, const moco::Tmpl &tt, int T,
             const moco::Geom &g, const moco_outputs *out, hipStream_t st, char *sbase,
             size_t sbytes)
{
    const int npad = tt.i8.npad;
    Int8Layout L = int8_layout(g, npad);
    int C = (int)std::min<size_t>((size_t)T, sbytes / L.total_per_frame);
    C = std::min(C, kChunkInt8);
    if (C < 1) return fail(MOCO_ENOMEM, "scratch slice too small for one frame");
    char *base = sbase;
    int8_t *limbs = (int8_t *)base;
    int32_t *nl = (int32_t *)(base + L.limbs * C);
    int32_t *vm = nl + C;   // the per-frame slot of L.nlimb bytes holds both arrays
    long long *atab = (long long *)(base + (L.limbs + L.nlimb) * C);
    long long *edge = (long long *)(base + (L.limbs + L.nlimb + L.atab) * C);
    long long *h = (long long *)(base + (L.limbs + L.nlimb + L.atab + L.edge) * C);
    int32_t *cst = (int32_t *)(base + (L.limbs + L.nlimb + L.atab + L.edge + L.h) * C);
    double *part = (double *)(base + (L.limbs + L.nlimb + L.atab + L.edge + L.h + L.cst) * C);
    const size_t fbytes = (size_t)g.m * g.n * sizeof(uint16_t);
    const int W = g.W;
    for (int f0 = 0; f0 < T; f0 += C) {
        int c = std::min(C, T - f0);
        const int tile = int8_tile(tt, c);
        const uint16_t *fr = (const uint16_t *)((const char *)d_frames + (size_t)f0 * fbytes);
        int32_t *coarse = out->coarse ? out->coarse + 2 * (size_t)f0 : cst;
        // a correlation over row slices adds into a table the prep launch clears
        const bool zero_h = moco::int8_corr_adds_slices(c, g, tile);
        {
            StageTimer tm(ctx, MOCO_STAGE_PREP, st);
            HIP_TRY(moco::launch_prep_u16(fr, c, g, npad, tt.i8.dbits, limbs, nl, vm, atab, edge,
                                          st, zero_h ? (int32_t *)h : nullptr));
        }
        {
            StageTimer tm(ctx, MOCO_STAGE_CORR, st);
            HIP_TRY(moco::launch_corr_int8(limbs, nl, tt.i8, c, g, h, st, nullptr, tile, zero_h));
        }
        {
            StageTimer tm(ctx, MOCO_STAGE_COMBINE, st);
            HIP_TRY(moco::launch_combine_i64(
                atab, tt.i8.atab, h, c, g, out->fsurf ? out->fsurf + (size_t)f0 * W * W : nullptr,
                out->fmin ? out->fmin + f0 : nullptr, coarse, out->shifts + 2 * (size_t)f0,
                out->gaps ? out->gaps + 2 * (size_t)f0 : nullptr,
                out->frefine ? out->frefine + 9 * (size_t)f0 : nullptr, st));
        }
        if (g.ds) {
            StageTimer tm(ctx, MOCO_STAGE_REFINE, st);
            HIP_TRY(moco::launch_refine(fr, tt.raw, c, g, coarse, out->shifts + 2 * (size_t)f0,
                                        out->frefine ? out->frefine + 9 * (size_t)f0 : nullptr,
                                        out->gaps ? out->gaps + 2 * (size_t)f0 : nullptr, part,
                                        st, vm, tt.i8.vmax));
        }
    }
    return MOCO_OK;
}

// Device tables of a multi-template int8 run: F frames, the i-th against the
// template of tmpls[i] (one geometry, digit base and plane count for all).
struct Int8MultiTables {
    const int8_t **btp;          // [F] per correlation block-column (at most F used)
    int *bf0, *bfe;              // [F]
    const uint16_t **traws;      // [F] per frame
    int32_t *tmaxs;              // [F]
    const long long **btabs;     // [F]
    static size_t bytes(int F) { return (size_t)F * (8 + 4 + 4 + 8 + 4 + 8) + 6 * 8; }
    // lay the tables out in `base` (8-byte aligned), F entries each
    void place(char *base, int F)
    {
        size_t o = 0;
        auto take = [&](size_t sz) { char *p = base + o; o = align_up(o + sz, 8); return p; };
        btp = (const int8_t **)take((size_t)F * 8);
        traws = (const uint16_t **)take((size_t)F * 8);
        btabs = (const long long **)take((size_t)F * 8);
        bf0 = (int *)take((size_t)F * 4);
        bfe = (int *)take((size_t)F * 4);
        tmaxs = (int32_t *)take((size_t)F * 4);
    }
};

// Fill the host copy of a multi-template run's tables for frames whose
// templates are tmpls[0..F-1] (frames of one template consecutive); returns
// the number of correlation block-columns (at most four frames each, of one
// template).
int fill_int8_multi(const moco::Tmpl *const *tmpls, int F, Int8MultiTables &h)
{
    int nb = 0;
    for (int f = 0; f < F;) {
        int e = f;
        while (e < F && tmpls[e] == tmpls[f]) ++e;
        for (int k = f; k < e; k += 4) {
            h.btp[nb] = tmpls[f]->i8.tp;
            h.bf0[nb] = k;
            h.bfe[nb] = std::min(k + 4, e);
            ++nb;
        }
        f = e;
    }
    for (int f = 0; f < F; ++f) {
        h.traws[f] = (const uint16_t *)tmpls[f]->raw;
        h.tmaxs[f] = tmpls[f]->i8.vmax;
        h.btabs[f] = tmpls[f]->i8.atab;
    }
    return nb;
}

// Whether frames of these templates can share one multi-template int8 run:
// the int8 form with the same geometry, digit base and planes, and the
// rolling refine (uint16, even rows, aligned buffers) when downsampling.
bool int8_multi_key_equal(const moco::Tmpl &a, const moco::Tmpl &b)
{
    const moco::Geom &x = a.g, &y = b.g;
    return x.m == y.m && x.n == y.n && x.w == y.w && x.ds == y.ds && x.dtype == y.dtype &&
           a.i8.npad == b.i8.npad && a.i8.trow == b.i8.trow && a.i8.padl == b.i8.padl &&
           a.i8.dbits == b.i8.dbits && a.i8.nq == b.i8.nq;
}

// The int8 pipeline over F frames of several templates (device tables `dt`
// already on the device), in one launch per stage; the frames must fit one
// chunk of `sbytes` of scratch.  Outputs as run_int8 (no surface).
int run_int8_multi(moco_ctx *ctx, const void *d_frames, const moco::Tmpl &tref, int F, int nblocks,
                   const Int8MultiTables &dt, const moco_outputs *out, hipStream_t st, char *sbase,
                   size_t sbytes)
{
    const moco::Geom &g = tref.g;
    const int npad = tref.i8.npad;
    Int8Layout L = int8_layout(g, npad);
    if ((size_t)F * L.total_per_frame > sbytes)
        return fail(MOCO_ENOMEM, "multi-template run of %d frames exceeds its scratch", F);
    char *base = sbase;
    int8_t *limbs = (int8_t *)base;
    int32_t *nl = (int32_t *)(base + L.limbs * F);
    int32_t *vm = nl + F;
    long long *atab = (long long *)(base + (L.limbs + L.nlimb) * F);
    long long *edge = (long long *)(base + (L.limbs + L.nlimb + L.atab) * F);
    long long *h = (long long *)(base + (L.limbs + L.nlimb + L.atab + L.edge) * F);
    int32_t *cst = (int32_t *)(base + (L.limbs + L.nlimb + L.atab + L.edge + L.h) * F);
    double *part = (double *)(base + (L.limbs + L.nlimb + L.atab + L.edge + L.h + L.cst) * F);
    const uint16_t *fr = (const uint16_t *)d_frames;
    int32_t *coarse = out->coarse ? out->coarse : cst;
    const moco::Int8Multi mm{nblocks, dt.btp, dt.bf0, dt.bfe};
    const int tile = int8_tile(tref, F);
    const bool zero_h = moco::int8_corr_adds_slices(F, g, tile, mm.nblocks);
    HIP_TRY(moco::launch_prep_u16(fr, F, g, npad, tref.i8.dbits, limbs, nl, vm, atab, edge, st,
                                  zero_h ? (int32_t *)h : nullptr));
    HIP_TRY(moco::launch_corr_int8(limbs, nl, tref.i8, F, g, h, st, &mm, tile, zero_h));
    HIP_TRY(moco::launch_combine_i64(atab, nullptr, h, F, g, nullptr, out->fmin, coarse,
                                     out->shifts, out->gaps, out->frefine, st, dt.btabs));
    if (g.ds)
        HIP_TRY(moco::launch_refine_multi(fr, dt.traws, dt.tmaxs, F, g, coarse, out->shifts,
                                          out->frefine, out->gaps, part, st, vm));
    return MOCO_OK;
}

// The FP64 exact pipeline over one stack, in chunks that fit `sbytes` of
// scratch at `sbase`; every launch goes to stream st.
int run_exact(moco_ctx *ctx, const void *d_frames, const moco::Tmpl &tt, int T,
              const moco::Geom &g, const moco_outputs *out, hipStream_t st, char *sbase,
              size_t sbytes)
{
    ExactLayout L = exact_layout(g);
    int C = (int)std::min<size_t>((size_t)T, sbytes / L.total_per_frame);
    C = std::min(C, kChunkOther);
    if (C < 1) return fail(MOCO_ENOMEM, "scratch slice too small for one frame");
    char *base = sbase;
    const moco_dtype dtype = g.dtype;
    size_t off = 0;
    double *coarse = (double *)(base + off);
    off += L.coarse * C;
    double *inter = (double *)(base + off);
    off += L.inter * C;
    double *atab = (double *)(base + off);
    off += L.atab * C;
    long long *edge = L.edge ? (long long *)(base + off) : nullptr;
    off += L.edge * C;
    double *h = (double *)(base + off);
    off += L.h * C;
    int32_t *cst = (int32_t *)(base + off);
    int32_t *shA = cst + 2 * (size_t)C, *shB = cst + 4 * (size_t)C;
    off += L.cst * C;
    int32_t *pm = (int32_t *)(base + off);
    off += L.pm * C;
    double *part = (double *)(base + align_up(off, 8));
    const size_t fbytes = (size_t)g.m * g.n * dtype_size(dtype);
    const int W = g.W;
    for (int f0 = 0; f0 < T; f0 += C) {
        int c = std::min(C, T - f0);
        const char *fr = (const char *)d_frames + (size_t)f0 * fbytes;
        int32_t *coarse_st = out->coarse ? out->coarse + 2 * (size_t)f0 : cst;
        HIP_TRY(grid_and_energies(ctx, fr, g, c, inter, coarse, atab, pm, edge, st));
        {
            StageTimer tm(ctx, MOCO_STAGE_CORR, st);
            HIP_TRY(moco::launch_corr_fp64(coarse, tt.coarse, c, g, h, st));
        }
        {
            StageTimer tm(ctx, MOCO_STAGE_COMBINE, st);
            HIP_TRY(moco::launch_combine(atab, tt.btab, h, c, g,
                                     out->fsurf ? out->fsurf + (size_t)f0 * W * W : nullptr,
                                     out->fmin ? out->fmin + f0 : nullptr, coarse_st,
                                     out->shifts + 2 * (size_t)f0,
                                     out->gaps ? out->gaps + 2 * (size_t)f0 : nullptr,
                                     out->frefine ? out->frefine + 9 * (size_t)f0 : nullptr, st));
        }
        if (g.ds) {
            StageTimer tm(ctx, MOCO_STAGE_REFINE, st);
            const int32_t *lvl1 = nullptr;
            HIP_TRY(refine_levels(tt, c, g, inter, coarse_st, shA, shB, part, st, &lvl1));
            HIP_TRY(moco::launch_refine(fr, tt.raw, c, g, lvl1, out->shifts + 2 * (size_t)f0,
                                        out->frefine ? out->frefine + 9 * (size_t)f0 : nullptr,
                                        out->gaps ? out->gaps + 2 * (size_t)f0 : nullptr, part,
                                        st, pm, tt.pbound));
        }
    }
    return MOCO_OK;
}

// Per-frame scratch of the FFT form.
struct FftLayout {
    size_t coarse, inter, atab, s1, s2, h, cst, pm, flag, edge, part, xmax, f1, total_per_frame;
};

// fp32: the single-precision form's half spectra (FP32 complex); cert32: its
// certified variant, whose FP64 pass over uncertified frames needs FP64 half
// spectra, the spectrum maxima, a second flag and the combine's f
FftLayout fft_layout(const moco::Geom &g, bool fp32 = false, bool cert32 = false)
{
    FftLayout L;
    const size_t esz = fp32 && !cert32 ? sizeof(float2) : sizeof(double2);
    L.coarse = align_up((size_t)g.mg * g.ng * sizeof(double), 256);
    L.inter = align_up(inter_elems(g) * sizeof(double), 256);
    L.atab = align_up((size_t)g.W * g.W * sizeof(double), 256);
    L.s1 = align_up(moco::fft_s1_bytes(g, esz), 256);
    L.s2 = align_up(moco::fft_s2_bytes(g, esz), 256);
    L.h = align_up((size_t)g.W * g.W * sizeof(double), 256);
    L.cst = 3 * 2 * sizeof(int32_t);   // the searched grid's argmin, two x2-step buffers
    L.pm = sizeof(int32_t);
    // two flags for cert32, padded so that the refine partials after them stay
    // 8-byte aligned for any chunk length
    L.flag = cert32 ? 3 * sizeof(int32_t) : sizeof(int32_t);
    L.edge = align_up(energy_scratch_bytes(g), 256);
    L.part = align_up(refine_steps_partial_bytes(g), 8);
    // at most one column block per bin
    L.xmax = cert32 ? align_up((size_t)moco::fft_geom(g).qh * sizeof(float), 256) : 0;
    L.f1 = cert32 ? sizeof(double) : 0;
    L.total_per_frame = L.coarse + L.inter + L.atab + L.s1 + L.s2 + L.h + L.cst + L.pm + L.flag +
                        L.edge + L.part + L.xmax + L.f1;
    return L;
}

// The FFT pipeline over one stack: the exact form's grid, energies, combine
// and refine around the transform-based correlation.  With `certify`, frames
// whose argmin the error bound of the transforms does not certify get their
// correlation recomputed by direct FP64 sums and are combined again before the
// x2 steps.  With `fp32`, the single-precision form: the transforms in FP32 on
// the grids less the template's offset c, the energies of the centred grids
// (FP64; exact integers for uint16), the same combine.  Both: the FP32 form
// certified by the a-posteriori bound of Cert32; certified frames get f at
// their argmin by its definition (k_polish), the others go through the
// certified FP64 form (uncentred energies, FP64 transforms, then direct sums
// for what that leaves), and recomputed[f] counts the passes they took.
int run_fft(moco_ctx *ctx, const void *d_frames, const moco::Tmpl &tt, int T,
            const moco::Geom &g, const moco_outputs *out, hipStream_t st, char *sbase,
            size_t sbytes, bool certify, bool fp32 = false)
{
    const bool cert32 = certify && fp32;
    FftLayout L = fft_layout(g, fp32, cert32);
    int C = (int)std::min<size_t>((size_t)T, sbytes / L.total_per_frame);
    C = std::min(C, kChunkOther);
    if (C < 1) return fail(MOCO_ENOMEM, "scratch slice too small for one frame");
    char *base = sbase;
    const moco_dtype dtype = g.dtype;
    size_t off = 0;
    double *coarse = (double *)(base + off);
    off += L.coarse * C;
    double *inter = (double *)(base + off);
    off += L.inter * C;
    double *atab = (double *)(base + off);
    off += L.atab * C;
    long long *edge = L.edge ? (long long *)(base + off) : nullptr;
    off += L.edge * C;
    char *s1 = base + off;
    off += L.s1 * C;
    char *s2 = base + off;
    off += L.s2 * C;
    double *h = (double *)(base + off);
    off += L.h * C;
    float *xmax = L.xmax ? (float *)(base + off) : nullptr;   // 256-aligned, as all above
    off += L.xmax * C;
    double *f1buf = L.f1 ? (double *)(base + off) : nullptr;
    off += L.f1 * C;
    int32_t *cst = (int32_t *)(base + off);
    int32_t *shA = cst + 2 * (size_t)C, *shB = cst + 4 * (size_t)C;
    off += L.cst * C;
    int32_t *pm = (int32_t *)(base + off);
    off += L.pm * C;
    int32_t *flag = (int32_t *)(base + off);
    int32_t *flag2 = flag + C;
    off += L.flag * C;
    double *part = (double *)(base + align_up(off, 8));
    const size_t fbytes = (size_t)g.m * g.n * dtype_size(dtype);
    const int W = g.W;
    double kf = 0.0, ke = 0.0;
    if (certify) moco::fft_error_coefs(g, tt.fft, &kf, &ke);
    moco::Cert32 c32;
    if (cert32) {
        moco::fft32_cert_coefs(tt.fft, &c32.e1, &c32.e2);
        c32.yinf = tt.fft.yinf32;
        c32.sqrtpq = std::sqrt((double)tt.fft.pp.n * (double)tt.fft.pq.n);
        c32.xmax = xmax;
    }
    // at most one 2x2 level: no FP64 grid in HBM (the energies and the row
    // transforms form its values from the pixels)
    const bool raw_rows = g.ds <= 1;
    const bool int_energy = edge && moco::prep_grid_applicable(g);   // uint16
    // the single-precision form's centring: c in grid units, xc in the prep
    // kernel's integer units (box sums when downsampling)
    const double center = fp32 ? tt.fft.center : 0.0;
    const int xc = (int)(center * (g.ds ? 4.0 : 1.0));
    const double *btab = fp32 ? tt.fft.btab32 : tt.btab;
    // the candidate pass of the single-precision certificate: its largest
    // squared difference is (4 x 65535)^2 with 2x2 box sums, 65535^2 without
    const double term_max = g.ds ? 262140.0 * 262140.0 : 65535.0 * 65535.0;
    const bool cand32 = cert32 && raw_rows && int_energy && g.W * g.W <= moco::kCand32MaxShifts &&
                        (double)g.mg * (double)g.ng * term_max < 0x1p53;
    for (int f0 = 0; f0 < T; f0 += C) {
        int c = std::min(C, T - f0);
        const char *fr = (const char *)d_frames + (size_t)f0 * fbytes;
        int32_t *coarse_st = out->coarse ? out->coarse + 2 * (size_t)f0 : cst;
        int32_t *recheck = out->recomputed ? out->recomputed + f0 : flag;
        double *fsurf = out->fsurf ? out->fsurf + (size_t)f0 * W * W : nullptr;
        double *fmin = out->fmin ? out->fmin + f0 : f1buf;
        double *gaps = out->gaps ? out->gaps + 2 * (size_t)f0 : nullptr;
        double *frefine = out->frefine ? out->frefine + 9 * (size_t)f0 : nullptr;
        if (raw_rows && int_energy) {
            // exact integer energies only: the row transforms read the pixels
            StageTimer tm(ctx, MOCO_STAGE_PREP, st);
            HIP_TRY(moco::launch_prep_grid((const uint16_t *)fr, c, g, nullptr, atab, pm, edge,
                                           st, nullptr, xc));
        } else if (raw_rows) {
            StageTimer tm(ctx, MOCO_STAGE_ENERGY, st);
            HIP_TRY(moco::launch_energy_px(fr, c, g, atab, pm, st, center));
        } else if (fp32) {
            {
                StageTimer tm(ctx, MOCO_STAGE_COARSE, st);
                HIP_TRY(build_levels(fr, g.dtype, c, g, inter, coarse, st));
            }
            StageTimer tm(ctx, MOCO_STAGE_ENERGY, st);
            HIP_TRY(moco::launch_energy(coarse, c, g, false, atab, pm, st, center));
        } else {
            HIP_TRY(grid_and_energies(ctx, fr, g, c, inter, coarse, atab, pm, edge, st));
        }
        {
            StageTimer tm(ctx, MOCO_STAGE_CORR, st);
            if (fp32) {
                if (raw_rows)
                    HIP_TRY(moco::launch_fft32_rows_px(fr, c, g, tt.fft, (float2 *)s1, st));
                else
                    HIP_TRY(moco::launch_fft32_rows(coarse, c, g, tt.fft, (float2 *)s1, st));
                HIP_TRY(moco::launch_fft32_corr((const float2 *)s1, c, g, tt.fft, (float2 *)s2,
                                                h, st, xmax, &c32.nxb));
            } else {
                if (raw_rows)
                    HIP_TRY(moco::launch_fft_rows_px(fr, c, g, tt.fft, (double2 *)s1, st));
                else
                    HIP_TRY(moco::launch_fft_rows(coarse, c, g, tt.fft, (double2 *)s1, st));
                HIP_TRY(moco::launch_fft_corr((const double2 *)s1, c, g, tt.fft, (double2 *)s2,
                                              h, st));
            }
        }
        {
            StageTimer tm(ctx, MOCO_STAGE_COMBINE, st);
            HIP_TRY(moco::launch_combine(atab, btab, h, c, g, fsurf, fmin, coarse_st,
                                         out->shifts + 2 * (size_t)f0, gaps, frefine, st,
                                         nullptr, certify ? recheck : nullptr, kf, ke,
                                         cert32 ? &c32 : nullptr));
        }
        if (cert32) {
            {
                // certified frames: f at the argmin by its definition
                StageTimer tm(ctx, MOCO_STAGE_COMBINE, st);
                HIP_TRY(moco::launch_polish(raw_rows ? (const void *)fr : (const void *)coarse,
                                            raw_rows, c, g, tt.coarse, coarse_st, recheck, fmin,
                                            fsurf, gaps, st));
            }
            // the others: first their candidates, where exact integer sums
            // settle them (uint16 pixels, one 2x2 level or none, sums of
            // squared differences below 2^53 so that f is exact)
            int32_t *resolved = flag + 2 * (size_t)C;
            if (cand32) {
                StageTimer tm(ctx, MOCO_STAGE_COMBINE, st);
                HIP_TRY(moco::launch_cand32(fr, c, g, atab, btab, h, tt.coarse, ke, c32,
                                            coarse_st, fmin, fsurf, gaps,
                                            out->shifts + 2 * (size_t)f0, recheck, resolved,
                                            st));
            }
            StageTimer tm(ctx, MOCO_STAGE_CORR, st);
            // then uncentred energies, FP64 transforms, the FP64 certificate
            if (raw_rows && int_energy)
                HIP_TRY(moco::launch_prep_grid((const uint16_t *)fr, c, g, nullptr, atab, pm, edge,
                                               st, recheck));
            else if (raw_rows)
                HIP_TRY(moco::launch_energy_px(fr, c, g, atab, pm, st, 0.0, recheck));
            else
                HIP_TRY(moco::launch_energy(coarse, c, g, false, atab, pm, st, 0.0, recheck));
            if (raw_rows)
                HIP_TRY(moco::launch_fft_rows_px(fr, c, g, tt.fft, (double2 *)s1, st, recheck));
            else
                HIP_TRY(moco::launch_fft_rows(coarse, c, g, tt.fft, (double2 *)s1, st, recheck));
            HIP_TRY(moco::launch_fft_corr((const double2 *)s1, c, g, tt.fft, (double2 *)s2, h, st,
                                          recheck));
            HIP_TRY(moco::launch_fill_i32(flag2, c, 0, st));
            HIP_TRY(moco::launch_combine(atab, tt.btab, h, c, g, fsurf, fmin, coarse_st,
                                         out->shifts + 2 * (size_t)f0, gaps, frefine, st,
                                         recheck, flag2, kf, ke));
            // and what the FP64 bound leaves: direct sums
            if (raw_rows && int_energy)
                HIP_TRY(moco::launch_prep_grid((const uint16_t *)fr, c, g, coarse, atab, pm, edge,
                                               st, flag2));
            else if (raw_rows)
                HIP_TRY(moco::launch_coarse(fr, dtype, c, g, coarse, st, flag2));
            HIP_TRY(moco::launch_corr_fp64(coarse, tt.coarse, c, g, h, st, flag2));
            HIP_TRY(moco::launch_combine(atab, tt.btab, h, c, g, fsurf, fmin, coarse_st,
                                         out->shifts + 2 * (size_t)f0, gaps, frefine, st,
                                         flag2));
            HIP_TRY(moco::launch_add_i32(recheck, flag2, c, st));
            if (cand32) HIP_TRY(moco::launch_add_i32(recheck, resolved, c, st));
        } else if (certify) {
            // the frames left uncertified: direct sums, combined again (their
            // FP64 grid first, when the row transforms read the pixels)
            StageTimer tm(ctx, MOCO_STAGE_CORR, st);
            if (raw_rows && int_energy)
                HIP_TRY(moco::launch_prep_grid((const uint16_t *)fr, c, g, coarse, atab, pm, edge,
                                               st, recheck));
            else if (raw_rows)
                HIP_TRY(moco::launch_coarse(fr, dtype, c, g, coarse, st, recheck));
            HIP_TRY(moco::launch_corr_fp64(coarse, tt.coarse, c, g, h, st, recheck));
            HIP_TRY(moco::launch_combine(atab, tt.btab, h, c, g, fsurf, fmin, coarse_st,
                                         out->shifts + 2 * (size_t)f0, gaps, frefine, st,
                                         recheck));
        } else if (out->recomputed) {
            HIP_TRY(moco::launch_fill_i32(out->recomputed + f0, c, 0, st));
        }
        if (g.ds) {
            StageTimer tm(ctx, MOCO_STAGE_REFINE, st);
            const int32_t *lvl1 = nullptr;
            HIP_TRY(refine_levels(tt, c, g, inter, coarse_st, shA, shB, part, st, &lvl1));
            HIP_TRY(moco::launch_refine(fr, tt.raw, c, g, lvl1, out->shifts + 2 * (size_t)f0,
                                        out->frefine ? out->frefine + 9 * (size_t)f0 : nullptr,
                                        out->gaps ? out->gaps + 2 * (size_t)f0 : nullptr, part,
                                        st, pm, tt.pbound));
        }
    }
    return MOCO_OK;
}

bool is_fft_form(moco_form f)
{
    return f == MOCO_FORM_FFT || f == MOCO_FORM_FFT_CERTIFIED || f == MOCO_FORM_FFT32 ||
           f == MOCO_FORM_FFT32_CERTIFIED;
}

int chunk_cap(moco_form form) { return form == MOCO_FORM_INT8_MFMA ? kChunkInt8 : kChunkOther; }

size_t per_frame_scratch(const moco::Geom &g, moco_form form, const moco::Tmpl &tt)
{
    if (form == MOCO_FORM_INT8_MFMA) return int8_layout(g, tt.i8.npad).total_per_frame;
    if (form == MOCO_FORM_FFT || form == MOCO_FORM_FFT_CERTIFIED)
        return fft_layout(g).total_per_frame;
    if (form == MOCO_FORM_FFT32) return fft_layout(g, true).total_per_frame;
    if (form == MOCO_FORM_FFT32_CERTIFIED) return fft_layout(g, true, true).total_per_frame;
    return exact_layout(g).total_per_frame;
}

int run_stack(moco_ctx *ctx, const void *d_frames, const moco::Tmpl &tt, int T,
              const moco::Geom &g, moco_form form, const moco_outputs *out, hipStream_t st,
              char *sbase, size_t sbytes)
{
    if (is_fft_form(form))
        return run_fft(ctx, d_frames, tt, T, g, out, st, sbase, sbytes,
                       form == MOCO_FORM_FFT_CERTIFIED || form == MOCO_FORM_FFT32_CERTIFIED,
                       form == MOCO_FORM_FFT32 || form == MOCO_FORM_FFT32_CERTIFIED);
    // the exact forms recompute nothing
    if (out->recomputed && T > 0) {
        hipError_t e = moco::launch_fill_i32(out->recomputed, T, 0, st);
        if (e != hipSuccess) return fail(MOCO_EDEVICE, "fill: %s", hipGetErrorString(e));
    }
    if (form == MOCO_FORM_INT8_MFMA) return run_int8(ctx, d_frames, tt, T, g, out, st, sbase, sbytes);
    return run_exact(ctx, d_frames, tt, T, g, out, st, sbase, sbytes);
}

// MFMA tiles of 32x32 shifts a frame's correlation issues with each tile
// shape: half a tile (16), ceil(W/32)^2 one-tile blocks, or ceil(W/64)^2
// blocks of 2x2 tiles.
double int8_tiles(const moco::Geom &g, int tile)
{
    if (tile == 16) return 0.5;   // one tile's MFMAs over half the K-chunks
    const double gs = std::ceil(g.W / (double)tile);
    return tile == 32 ? gs * gs : 4.0 * gs * gs;
}

// Launches of at most this many frames form the small size class of the
// int8 tile choice (their correlation splits the template rows over blocks).
constexpr int kInt8SmallBatch = 64;
int tile_class(int C) { return C <= kInt8SmallBatch ? 0 : 1; }

// Two 16x16 tiles on the diagonal of one 32x32 MFMA product when 2w-1 <= 16
// with three digit products (half the MFMAs of a single tile: 256x256 frames
// at w = 8, correlation 0.19 against 0.33 us per frame; with four products,
// whose LDS reads per MFMA are more, it gained nothing at 512x796, 0.58
// against 0.56); one 32x32 tile when 2w-1 <= 32, else 2x2 groups: a group
// reads each frame
// and template operand once for two tiles, and at 2w-1 = 79 on a 256x256 grid
// the groups (16 tiles) ran faster than single tiles (9 tiles).  A launch of
// at most kInt8SmallBatch frames takes single tiles up to 2w-1 = 64: four
// times the blocks fill more of the device (512x512 frames, w = 32:
// correlation 21 against 35 us for one frame, 109 against 128 us for 64,
// 176 against 165 us for 128).  moco_tune times both shapes.
int int8_model_tile(const moco::Tmpl &t, int cls)
{
    const moco::Geom &g = t.g;
    if (g.W <= 16 && t.i8.nq == 3) return 16;
    return g.W <= 32 || (cls == 0 && g.W <= 64) ? 32 : 64;
}

// Per-frame time models of the two fast forms (seconds), from their kernels'
// rates measured on MI355X at the 512x512, w = 32 workload: the int8 form
// issues the MFMA tiles of its tile shape (int8_tiles) of three
// digit products (base-128 digits with their
// sums) at about 2.7e15 ops/s or four (base 256) at about 2.8e15, beside 0.31
// us of prep, combine and refine per 512x512 frame; the FFT form's three
// transform passes took 0.72 us at 288x288 (FP64, wave-level kernels) and
// scale with P Q log2(P Q), beside 0.28 us of energies, combine and refine per
// 512x512 frame (those parts scale with the frame's pixels).  At that
// workload the models give 0.91 and 1.00 us per frame; measured 0.92 and 1.01.
double int8_model_s(const moco::Tmpl &t)
{
    const moco::Geom &g = t.g;
    const double macs =
        int8_tiles(g, int8_tile(t, kInt8SmallBatch + 1)) * 1024.0 * g.mg * (double)t.i8.npad;
    const double ops = macs * 2.0 * (t.i8.nq == 3 ? 3.0 : 4.0);
    return 0.31e-6 * ((double)g.m * g.n / 262144.0) + ops / (t.i8.nq == 3 ? 2.7e15 : 2.8e15);
}

double fft_model_s(const moco::Tmpl &t)
{
    const moco::Geom &g = t.g;
    const double pq = (double)t.fft.pp.n * t.fft.pq.n;
    const double ref = 288.0 * 288.0 * std::log2(288.0 * 288.0);
    return 0.28e-6 * ((double)g.m * g.n / 262144.0) + 0.72e-6 * pq * std::log2(pq) / ref;
}

// Forms chosen by measurement (moco_tune) or set by the caller, per search
// key; AUTO follows them where the form applies to the template.
struct TuneKey {
    int m, n, w, ds, dtype;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(m, n, w, ds, dtype) < std::tie(o.m, o.n, o.w, o.ds, o.dtype);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, moco_form> g_tune;
// the int8 form's shift tile (32 or 64) per key and launch size class
std::map<std::pair<TuneKey, int>, int> g_tune_tile;

TuneKey tune_key(const moco::Geom &g) { return TuneKey{g.m, g.n, g.w, g.ds, (int)g.dtype}; }

int int8_tile(const moco::Tmpl &t, int C)
{
    const int cls = tile_class(C);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_tile.find({tune_key(t.g), cls});
        if (it != g_tune_tile.end()) return it->second;
    }
    return int8_model_tile(t, cls);
}

bool form_applies(const moco::Tmpl &t, moco_form f)
{
    switch (f) {
    case MOCO_FORM_FP64_EXACT: return true;
    case MOCO_FORM_INT8_MFMA: return t.int8_ok;
    case MOCO_FORM_FFT:
    case MOCO_FORM_FFT_CERTIFIED:
    case MOCO_FORM_FFT32:
    case MOCO_FORM_FFT32_CERTIFIED: return t.fft_ok;
    default: return false;
    }
}

// The form AUTO runs: a form recorded for the template's key (moco_tune,
// moco_tune_set) when it applies; else the faster of the exact int8 form and
// the FFT form by the models above when both apply, else whichever applies
// (for float32 data the FFT in FP32), else direct FP64 sums.  The FFT forms
// run with their argmin certificates.
moco_form auto_form(const moco::Tmpl &t)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(t.g));
        if (it != g_tune.end() && form_applies(t, it->second)) return it->second;
    }
    if (t.int8_ok && t.fft_ok)
        return int8_model_s(t) <= fft_model_s(t) ? MOCO_FORM_INT8_MFMA : MOCO_FORM_FFT_CERTIFIED;
    if (t.int8_ok) return MOCO_FORM_INT8_MFMA;
    if (t.fft_ok && t.g.dtype == MOCO_F32) return MOCO_FORM_FFT32_CERTIFIED;
    if (t.fft_ok) return MOCO_FORM_FFT_CERTIFIED;
    return MOCO_FORM_FP64_EXACT;
}

// Validation shared by moco_align and moco_align_batch; resolves AUTO.
int check_stack(const moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m,
                int n, int w, int downsample, moco_dtype dtype, moco_form form,
                const moco_outputs *out, moco::Geom *g, moco_form *resolved)
{
    if (!tmpl || !out) return fail(MOCO_EINVAL, "null template or outputs");
    int rc = validate(m, n, w, downsample, dtype, g);
    if (rc) return rc;
    if (T < 0) return fail(MOCO_EINVAL, "T=%d must be >= 0", T);
    if (tmpl->device != ctx->device)
        return fail(MOCO_EINVAL, "template lives on device %d, context on device %d", tmpl->device,
                    ctx->device);
    const moco::Geom &tg = tmpl->t.g;
    if (tg.m != m || tg.n != n || tg.w != w || tg.ds != downsample || tg.dtype != dtype)
        return fail(MOCO_EINVAL,
                    "template prepared for (m=%d n=%d w=%d ds=%d dtype=%d), call has "
                    "(m=%d n=%d w=%d ds=%d dtype=%d)",
                    tg.m, tg.n, tg.w, tg.ds, (int)tg.dtype, m, n, w, downsample, (int)dtype);
    if (form != MOCO_FORM_AUTO && form != MOCO_FORM_FP64_EXACT && form != MOCO_FORM_INT8_MFMA &&
        !is_fft_form(form))
        return fail(MOCO_EINVAL, "unknown form %d", (int)form);
    if (form == MOCO_FORM_INT8_MFMA && dtype != MOCO_U16)
        return fail(MOCO_EINVAL, "the int8 matrix-core form needs uint16 data");
    if (T > 0 && (!d_frames || !out->shifts)) return fail(MOCO_EINVAL, "null frames or shifts");
    const moco::Tmpl &tt = tmpl->t;
    if (form == MOCO_FORM_INT8_MFMA && !tt.int8_ok)
        return fail(MOCO_EINVAL,
                    "the int8 matrix-core form does not apply to this template (needs uint16, "
                    "grid area below 131072, grid width at most 2048 and template values "
                    "within two base-256 digits)");
    if (is_fft_form(form) &&
        !tt.fft_ok)
        return fail(MOCO_EINVAL, "the FFT form does not apply to this template (transform "
                                 "lengths above %d)", moco::kFftMaxLen);
    if (form == MOCO_FORM_AUTO) form = auto_form(tt);
    *resolved = form;
    return MOCO_OK;
}

}  // namespace

extern "C" {

const char *moco_last_error(void) { return g_err.c_str(); }

const char *moco_version(void) { return "moco-mi355x 0.1"; }

int moco_default_params(int m, int n, int *w, int *downsample)
{
    if (!w || !downsample) return fail(MOCO_EINVAL, "moco_default_params: null output");
    if (m < 1 || n < 1) return fail(MOCO_EINVAL, "image size %dx%d must be positive", m, n);
    const int ds = (m > 256 || n > 256) ? 1 : 0;
    const int mg = m >> ds, ng = n >> ds;
    const int ww = std::min(mg, ng) / 3;
    *w = ww < 1 ? 1 : ww;
    *downsample = ds;
    return MOCO_OK;
}

int moco_create(int device, size_t scratch_budget_bytes, moco_ctx **out)
{
    if (!out) return fail(MOCO_EINVAL, "moco_create: out is null");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(MOCO_EINVAL, "device %d out of range (%d devices)", device, count);
    moco_ctx *ctx = new (std::nothrow) moco_ctx;
    if (!ctx) return fail(MOCO_ENOMEM, "out of host memory");
    ctx->device = device;
    ctx->budget = scratch_budget_bytes ? scratch_budget_bytes : (size_t)1 << 30;
    {
        // the allocation-free entry point's scratch on this device
        DeviceGuard dg(device);
        int rc = dg.ok() ? fixed_scratch_address(device, &ctx->fixed_scratch)
                         : fail(MOCO_EDEVICE, "cannot select device %d", device);
        if (rc) {
            delete ctx;
            return rc;
        }
    }
    *out = ctx;
    return MOCO_OK;
}

void moco_destroy(moco_ctx *ctx)
{
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    for (auto &r : ctx->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto e : ctx->lane_ev) (void)hipEventDestroy(e);
    for (auto l : ctx->lanes) (void)hipStreamDestroy(l);
    delete ctx;
}

int moco_apply(moco_ctx *ctx, const void *d_frames, const int32_t *d_shifts, int T, int m, int n,
               moco_dtype dtype, void *d_out, double *d_mean, void *hip_stream)
{
    if (!ctx) return fail(MOCO_EINVAL, "moco_apply: null ctx");
    if (dtype != MOCO_U16 && dtype != MOCO_F32) return fail(MOCO_EINVAL, "unknown dtype %d", (int)dtype);
    if (m < 1 || n < 1) return fail(MOCO_EINVAL, "image size %dx%d must be positive", m, n);
    if ((long long)m * n > (1LL << 30)) return fail(MOCO_EINVAL, "image %dx%d too large", m, n);
    if (T < 0) return fail(MOCO_EINVAL, "T=%d must be >= 0", T);
    if (T == 0) return MOCO_OK;
    if (!d_frames || !d_shifts) return fail(MOCO_EINVAL, "null frames or shifts");
    if (!d_out && !d_mean) return fail(MOCO_EINVAL, "neither corrected frames nor a mean asked for");
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)hip_stream;
    int kchunk = T;
    double *partial = nullptr;
    if (d_mean) {
        kchunk = moco::apply_chunk_frames(T, m, n, ctx->budget);
        if (kchunk == 0)
            return fail(MOCO_ENOMEM, "the mean's partial sums (%zu bytes) exceed the budget %zu",
                        (size_t)m * n * sizeof(double), ctx->budget);
        const size_t need = (size_t)((T + kchunk - 1) / kchunk) * m * n * sizeof(double);
        int rc = ensure_scratch(ctx, need, st);
        if (rc) return rc;
        partial = (double *)ctx->scratch;
    } else if (T > 16) {
        kchunk = (T + 31) / 32;
    }
    {
        StageTimer tm(ctx, MOCO_STAGE_APPLY, st);
        HIP_TRY(moco::launch_apply(d_frames, dtype, d_shifts, T, m, n, kchunk, d_out, partial,
                                   d_mean, st));
    }
    return MOCO_OK;
}

int moco_template_form(const moco_tmpl *tmpl, moco_form requested, moco_form *resolved)
{
    if (!tmpl || !resolved) return fail(MOCO_EINVAL, "moco_template_form: null argument");
    const moco::Tmpl &t = tmpl->t;
    switch (requested) {
    case MOCO_FORM_AUTO:
        *resolved = auto_form(t);
        return MOCO_OK;
    case MOCO_FORM_FP64_EXACT:
        *resolved = requested;
        return MOCO_OK;
    case MOCO_FORM_INT8_MFMA:
        if (!t.int8_ok) return fail(MOCO_EINVAL, "the int8 matrix-core form does not apply");
        *resolved = requested;
        return MOCO_OK;
    case MOCO_FORM_FFT:
    case MOCO_FORM_FFT_CERTIFIED:
    case MOCO_FORM_FFT32:
    case MOCO_FORM_FFT32_CERTIFIED:
        if (!t.fft_ok) return fail(MOCO_EINVAL, "the FFT form does not apply");
        *resolved = requested;
        return MOCO_OK;
    default:
        return fail(MOCO_EINVAL, "unknown form %d", (int)requested);
    }
}

int moco_template_fft_bound(const moco_tmpl *tmpl, double *kf, double *ke)
{
    if (!tmpl || !kf || !ke) return fail(MOCO_EINVAL, "moco_template_fft_bound: null argument");
    if (!tmpl->t.fft_ok) return fail(MOCO_EINVAL, "the FFT form does not apply");
    moco::fft_error_coefs(tmpl->t.g, tmpl->t.fft, kf, ke);
    return MOCO_OK;
}

int moco_template_int8_products(const moco_tmpl *tmpl, int *products)
{
    if (!tmpl || !products) return fail(MOCO_EINVAL, "moco_template_int8_products: null argument");
    if (!tmpl->t.int8_ok) return fail(MOCO_EINVAL, "the int8 form does not apply");
    *products = tmpl->t.i8.nq == 3 ? 3 : 4;
    return MOCO_OK;
}

int moco_tune(moco_ctx *ctx, const moco_tmpl *tmpl, int frames, void *hip_stream,
              moco_form *chosen, double *seconds_per_frame)
{
    if (!ctx || !tmpl || !chosen) return fail(MOCO_EINVAL, "moco_tune: null argument");
    if (tmpl->device != ctx->device)
        return fail(MOCO_EINVAL, "template lives on device %d, context on device %d",
                    tmpl->device, ctx->device);
    const moco::Tmpl &t = tmpl->t;
    const moco::Geom &g = t.g;
    const int T = frames > 0 ? frames : 1024;
    hipStream_t st = (hipStream_t)hip_stream;
    if (seconds_per_frame)
        for (int k = 0; k < MOCO_FORM_COUNT; ++k) seconds_per_frame[k] = -1.0;
    // (form, int8 tile) candidates: the int8 form with each tile shape that
    // applies (32 only when 2w-1 <= 32)
    std::vector<std::pair<moco_form, int>> cand;
    if (t.int8_ok) {
        if (g.W <= 16) cand.push_back({MOCO_FORM_INT8_MFMA, 16});
        cand.push_back({MOCO_FORM_INT8_MFMA, 32});
        if (g.W > 32) cand.push_back({MOCO_FORM_INT8_MFMA, 64});
    }
    if (t.fft_ok) cand.push_back({MOCO_FORM_FFT_CERTIFIED, 0});
    // (copies of the template pass the FP32 bound at once, which says little of
    // uint16 frames whose gaps are a few per cent of f: timed for float32 only)
    if (t.fft_ok && g.dtype == MOCO_F32) cand.push_back({MOCO_FORM_FFT32_CERTIFIED, 0});
    if (cand.empty()) cand.push_back({MOCO_FORM_FP64_EXACT, 0});
    DeviceGuard dg(ctx->device);
    // T copies of the template (its own frame: a realistic image, the shift at
    // zero) and a shift output
    const size_t fbytes = (size_t)g.m * g.n * dtype_size(g.dtype);
    char *d_frames = nullptr;
    int32_t *d_shifts = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&d_frames, fbytes * T);
    if (e == hipSuccess) e = hipMalloc(&d_shifts, sizeof(int32_t) * 2 * T);
    for (int k = 0; k < T && e == hipSuccess; ++k)
        e = hipMemcpyAsync(d_frames + fbytes * k, t.raw, fbytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = e == hipSuccess ? MOCO_OK : fail(MOCO_ENOMEM, "moco_tune: %s", hipGetErrorString(e));
    moco_form best = cand[0].first;
    int int8_tile_best = 0;
    double best_s = INFINITY, int8_best_s = INFINITY;
    moco_outputs out{};
    out.shifts = d_shifts;
    const TuneKey key = tune_key(g);
    const std::pair<TuneKey, int> tkey{key, tile_class(T)};   // the tile for launches of T frames
    int prev_tile = 0;   // a tile recorded before the call, restored if int8 is not timed
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_tile.find(tkey);
        if (it != g_tune_tile.end()) prev_tile = it->second;
    }
    for (size_t c = 0; c < cand.size() && rc == MOCO_OK; ++c) {
        const moco_form f = cand[c].first;
        if (cand[c].second) {
            // the tile the int8 runs below take
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_tile[tkey] = cand[c].second;
        }
        rc = moco_align(ctx, d_frames, tmpl, T, g.m, g.n, g.w, g.ds, g.dtype, f, &out, st);
        const int reps = 3;
        if (rc == MOCO_OK && (e = hipEventRecord(e0, st)) != hipSuccess)
            rc = fail(MOCO_EDEVICE, "moco_tune: %s", hipGetErrorString(e));
        for (int r = 0; r < reps && rc == MOCO_OK; ++r)
            rc = moco_align(ctx, d_frames, tmpl, T, g.m, g.n, g.w, g.ds, g.dtype, f, &out, st);
        float ms = 0.f;
        if (rc == MOCO_OK && ((e = hipEventRecord(e1, st)) != hipSuccess ||
                              (e = hipEventSynchronize(e1)) != hipSuccess ||
                              (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess))
            rc = fail(MOCO_EDEVICE, "moco_tune: %s", hipGetErrorString(e));
        if (rc != MOCO_OK) break;
        const double sec = ms / 1000.0 / reps / T;
        if (f == MOCO_FORM_INT8_MFMA && sec < int8_best_s) {
            int8_best_s = sec;
            int8_tile_best = cand[c].second;
        }
        if (seconds_per_frame && (f != MOCO_FORM_INT8_MFMA || sec <= int8_best_s))
            seconds_per_frame[(int)f] = sec;
        if (sec < best_s) {
            best_s = sec;
            best = f;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    if (d_frames) (void)hipFree(d_frames);
    if (d_shifts) (void)hipFree(d_shifts);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        // the int8 form keeps its faster tile whichever form won
        if (rc == MOCO_OK && int8_tile_best) g_tune_tile[tkey] = int8_tile_best;
        else if (prev_tile) g_tune_tile[tkey] = prev_tile;
        else g_tune_tile.erase(tkey);
        if (rc == MOCO_OK) g_tune[key] = best;
    }
    if (rc != MOCO_OK) return rc;
    *chosen = best;
    return MOCO_OK;
}

int moco_tune_set_tile(int m, int n, int w, int downsample, moco_dtype dtype, int tile)
{
    if (tile != 16 && tile != 32 && tile != 64)
        return fail(MOCO_EINVAL, "moco_tune_set_tile: tile %d", tile);
    if (tile == 16 && 2 * w - 1 > 16)
        return fail(MOCO_EINVAL, "moco_tune_set_tile: 2w-1 = %d exceeds a 16x16 tile", 2 * w - 1);
    if (dtype != MOCO_U16) return fail(MOCO_EINVAL, "moco_tune_set_tile: the int8 form is uint16 only");
    if (tile == 64 && 2 * w - 1 <= 32)
        return fail(MOCO_EINVAL, "moco_tune_set_tile: 2w-1 = %d takes one 32x32 tile", 2 * w - 1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int cls = 0; cls < 2; ++cls) g_tune_tile[{TuneKey{m, n, w, downsample, (int)dtype}, cls}] = tile;
    return MOCO_OK;
}

int moco_template_int8_tile(const moco_tmpl *tmpl, int *tile)
{
    if (!tmpl || !tile) return fail(MOCO_EINVAL, "moco_template_int8_tile: null argument");
    if (!tmpl->t.int8_ok) return fail(MOCO_EINVAL, "the int8 form does not apply");
    *tile = int8_tile(tmpl->t, kInt8SmallBatch + 1);
    return MOCO_OK;
}

int moco_tune_set(int m, int n, int w, int downsample, moco_dtype dtype, moco_form form)
{
    if (form != MOCO_FORM_FP64_EXACT && form != MOCO_FORM_INT8_MFMA && !is_fft_form(form))
        return fail(MOCO_EINVAL, "moco_tune_set: form %d is not a concrete form", (int)form);
    if (dtype != MOCO_U16 && dtype != MOCO_F32)
        return fail(MOCO_EINVAL, "moco_tune_set: unknown dtype %d", (int)dtype);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{m, n, w, downsample, (int)dtype}] = form;
    return MOCO_OK;
}

int moco_tune_get(int m, int n, int w, int downsample, moco_dtype dtype, moco_form *form)
{
    if (!form) return fail(MOCO_EINVAL, "moco_tune_get: null form");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{m, n, w, downsample, (int)dtype});
    if (it == g_tune.end()) return fail(MOCO_EINVAL, "moco_tune_get: no form recorded");
    *form = it->second;
    return MOCO_OK;
}

void moco_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_tile.clear();
}

int moco_profile_enable(moco_ctx *ctx, int enable)
{
    if (!ctx) return fail(MOCO_EINVAL, "moco_profile_enable: null ctx");
    ctx->profiling = enable != 0;
    return MOCO_OK;
}

int moco_profile_read(moco_ctx *ctx, double *ms, int64_t *launches)
{
    if (!ctx || !ms || !launches) return fail(MOCO_EINVAL, "moco_profile_read: null argument");
    DeviceGuard dg(ctx->device);
    for (int k = 0; k < MOCO_STAGE_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : ctx->prof) {
        HIP_TRY(hipEventSynchronize(r.b));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.stage] += t;
        launches[r.stage] += 1;
        ctx->ev_pool.push_back(r.a);
        ctx->ev_pool.push_back(r.b);
    }
    ctx->prof.clear();
    return MOCO_OK;
}

int moco_template_create(moco_ctx *ctx, const void *d_template, moco_dtype dtype, int m, int n,
                         int w, int downsample, void *hip_stream, moco_tmpl **out)
{
    if (!ctx || !out || !d_template)
        return fail(MOCO_EINVAL, "moco_template_create: null ctx, template or out");
    *out = nullptr;
    moco::Geom g;
    int rc = validate(m, n, w, downsample, dtype, &g);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)hip_stream;
    moco_tmpl *tp = new (std::nothrow) moco_tmpl;
    if (!tp) return fail(MOCO_ENOMEM, "out of host memory");
    tp->device = ctx->device;
    moco::Tmpl &t = tp->t;
    t.g = g;
    size_t raw_bytes = (size_t)m * n * dtype_size(dtype);
    int32_t *pb = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&](int code) {
        if (pb) (void)hipStreamSynchronize(st), (void)hipFree(pb);
        free_tmpl(t);
        delete tp;
        return code;
    };
    t.pbound = -1;
    int32_t pbv = INT32_MAX;
    t.pyr = nullptr;
    if ((e = hipMalloc(&t.raw, raw_bytes)) != hipSuccess ||
        (e = hipMalloc(&t.coarse, (size_t)g.mg * g.ng * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&t.btab, (size_t)g.W * g.W * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&pb, sizeof(int32_t))) != hipSuccess ||
        (inter_elems(g) &&
         (e = hipMalloc(&t.pyr, inter_elems(g) * sizeof(double))) != hipSuccess))
        return cleanup(fail(MOCO_ENOMEM, "template allocation failed: %s", hipGetErrorString(e)));
    // the template's energies over D at (s,t) are its frame-side energies at (-s,-t)
    if ((e = hipMemcpyAsync(t.raw, d_template, raw_bytes, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess ||
        (e = build_levels(t.raw, dtype, 1, g, t.pyr, t.coarse, st)) != hipSuccess ||
        (e = moco::launch_energy(t.coarse, 1, g, true, t.btab, pb, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&pbv, pb, sizeof pbv, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return cleanup(fail(MOCO_EDEVICE, "template preparation failed: %s", hipGetErrorString(e)));
    (void)hipFree(pb);
    pb = nullptr;
    t.pbound = pbv == INT32_MAX ? -1 : pbv;
    if (dtype == MOCO_U16) {
        int rc8 = prepare_int8_template(t, st);
        if (rc8) return cleanup(rc8);
    }
    int rcf = prepare_fft_template(t, st);
    if (rcf) return cleanup(rcf);
    *out = tp;
    return MOCO_OK;
}

void moco_template_destroy(moco_tmpl *tmpl)
{
    if (!tmpl) return;
    DeviceGuard dg(tmpl->device);
    free_tmpl(tmpl->t);
    delete tmpl;
}

int moco_align(moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m, int n,
               int w, int downsample, moco_dtype dtype, moco_form form, const moco_outputs *out,
               void *hip_stream)
{
    if (!ctx || !tmpl || !out) return fail(MOCO_EINVAL, "moco_align: null ctx, template or outputs");
    moco::Geom g;
    int rc = check_stack(ctx, d_frames, tmpl, T, m, n, w, downsample, dtype, form, out, &g, &form);
    if (rc) return rc;
    if (T == 0) return MOCO_OK;
    const moco::Tmpl &tt = tmpl->t;
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t pf = per_frame_scratch(g, form, tt);
    if (pf > ctx->budget)
        return fail(MOCO_ENOMEM, "one frame needs %zu bytes of scratch, budget is %zu", pf,
                    ctx->budget);
    const size_t frames = std::min<size_t>(std::min<size_t>((size_t)T, (size_t)chunk_cap(form)),
                                           std::max<size_t>(1, ctx->budget / pf));
    const size_t need = pf * frames;
    rc = ensure_scratch(ctx, need, st);
    if (rc) return rc;
    return run_stack(ctx, d_frames, tt, T, g, form, out, st, (char *)ctx->scratch, need);
}

int moco_align_noalloc(moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m,
                       int n, int w, int downsample, moco_dtype dtype, moco_form form,
                       const moco_outputs *out, void *hip_stream)
{
    if (!ctx || !tmpl || !out)
        return fail(MOCO_EINVAL, "moco_align_noalloc: null ctx, template or outputs");
    moco::Geom g;
    int rc = check_stack(ctx, d_frames, tmpl, T, m, n, w, downsample, dtype, form, out, &g, &form);
    if (rc) return rc;
    if (T == 0) return MOCO_OK;
    const moco::Tmpl &tt = tmpl->t;
    const size_t pf = per_frame_scratch(g, form, tt);
    if (pf > kFixedScratchBytes)
        return fail(MOCO_ENOMEM,
                    "moco_align_noalloc: one frame needs %zu bytes of scratch, the fixed "
                    "scratch holds %zu (use moco_align)", pf, kFixedScratchBytes);
    if (!ctx->fixed_scratch) return fail(MOCO_EDEVICE, "moco_align_noalloc: no fixed scratch");
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    const size_t frames = std::min<size_t>(std::min<size_t>((size_t)T, (size_t)chunk_cap(form)),
                                           kFixedScratchBytes / pf);
    // no stage timing here: recording it creates events and grows a host list
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    rc = run_stack(ctx, d_frames, tt, T, g, form, out, (hipStream_t)hip_stream,
                   (char *)ctx->fixed_scratch, pf * frames);
    ctx->profiling = prof;
    return rc;
}

}  // extern "C"

namespace {

// A batch's validated stacks, lanes, lane slice and the stacks of each lane.
struct BatchPlan {
    std::vector<moco::Geom> geo;
    std::vector<moco_form> forms;
    int nl = 0;                       // lanes; 0: no frame to align
    size_t slice = 0;                 // scratch bytes per lane
    std::vector<std::vector<int>> plan;
};

// Validate every stack (all-or-nothing, before anything is enqueued), choose
// the lanes and their scratch slice, and spread the stacks over the lanes
// longest first onto the least loaded.
int plan_batch(const moco_ctx *ctx, const moco_stack *stacks, int nstacks, moco_form form,
               int lanes, BatchPlan *bp)
{
    if (lanes < 0) return fail(MOCO_EINVAL, "lanes=%d must be >= 0", lanes);
    bp->geo.assign(nstacks, moco::Geom{});
    bp->forms.assign(nstacks, MOCO_FORM_AUTO);
    std::vector<double> cost(nstacks);
    size_t pf_max = 0, slice_need = 0;
    for (int k = 0; k < nstacks; ++k) {
        const moco_stack &sk = stacks[k];
        int rc = check_stack(ctx, sk.d_frames, sk.tmpl, sk.T, sk.m, sk.n, sk.w, sk.downsample,
                             sk.dtype, form, &sk.out, &bp->geo[k], &bp->forms[k]);
        if (rc) return fail(rc, "stack %d: %s", k, moco_last_error());
        const size_t pf = per_frame_scratch(bp->geo[k], bp->forms[k], sk.tmpl->t);
        if (sk.T > 0) {
            pf_max = std::max(pf_max, pf);
            // a lane slice never needs more than one chunk of its largest stack
            slice_need = std::max(slice_need, pf * (size_t)std::min(sk.T, chunk_cap(bp->forms[k])));
        }
        const moco::Geom &g = bp->geo[k];
        cost[k] = (double)sk.T * ((double)g.W * g.W * g.mg * g.ng + (double)g.m * g.n);
    }
    bp->nl = 0;
    if (pf_max == 0) return MOCO_OK;  // nothing to align
    if (pf_max > ctx->budget)
        return fail(MOCO_ENOMEM, "one frame needs %zu bytes of scratch, budget is %zu", pf_max,
                    ctx->budget);
    int nl = lanes ? std::min(lanes, 8) : 4;
    nl = (int)std::min<size_t>((size_t)nl, ctx->budget / pf_max);
    nl = std::max(1, std::min(nl, nstacks));
    // lane slices start 256-byte aligned; each must hold one frame of any stack
    size_t lane_cap = ctx->budget / nl / 256 * 256;
    while (nl > 1 && lane_cap < pf_max) lane_cap = ctx->budget / --nl / 256 * 256;
    bp->slice = std::min(lane_cap, align_up(slice_need, 256));
    bp->nl = nl;
    std::vector<int> order(nstacks);
    for (int k = 0; k < nstacks; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(nl, 0.0);
    bp->plan.assign(nl, {});
    for (int k : order) {
        if (stacks[k].T == 0) continue;
        int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bp->plan[best].push_back(k);
        load[best] += cost[k];
    }
    return MOCO_OK;
}

// Enqueue a planned batch: every lane stream waits for `st`, runs its stacks
// on its slice of `base`, and `st` waits for every lane.  ev: nl + 1 events.
int enqueue_batch(moco_ctx *ctx, const moco_stack *stacks, const BatchPlan &bp, hipStream_t st,
                  char *base, hipStream_t *lane_st, hipEvent_t *ev)
{
    const int nl = bp.nl;
    hipEvent_t fork = ev[nl];
    HIP_TRY(hipEventRecord(fork, st));
    for (int l = 0; l < nl; ++l) HIP_TRY(hipStreamWaitEvent(lane_st[l], fork, 0));
    for (int l = 0; l < nl; ++l) {
        for (int k : bp.plan[l]) {
            const moco_stack &sk = stacks[k];
            int rc = run_stack(ctx, sk.d_frames, sk.tmpl->t, sk.T, bp.geo[k], bp.forms[k], &sk.out,
                               lane_st[l], base + bp.slice * l, bp.slice);
            if (rc) return rc;
        }
    }
    for (int l = 0; l < nl; ++l) {
        HIP_TRY(hipEventRecord(ev[l], lane_st[l]));
        HIP_TRY(hipStreamWaitEvent(st, ev[l], 0));
    }
    return MOCO_OK;
}

}  // namespace

extern "C" {

int moco_graph_create(moco_ctx *ctx, const void *d_frames, const moco_tmpl *tmpl, int T, int m,
                      int n, int w, int downsample, moco_dtype dtype, moco_form form,
                      const moco_outputs *out, moco_graph **graph)
{
    if (!ctx || !tmpl || !out || !graph)
        return fail(MOCO_EINVAL, "moco_graph_create: null ctx, template, outputs or graph");
    *graph = nullptr;
    moco::Geom g;
    int rc = check_stack(ctx, d_frames, tmpl, T, m, n, w, downsample, dtype, form, out, &g, &form);
    if (rc) return rc;
    if (T < 1) return fail(MOCO_EINVAL, "moco_graph_create: T=%d must be >= 1", T);
    const moco::Tmpl &tt = tmpl->t;
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    const size_t pf = per_frame_scratch(g, form, tt);
    if (pf > ctx->budget)
        return fail(MOCO_ENOMEM, "one frame needs %zu bytes of scratch, budget is %zu", pf,
                    ctx->budget);
    const size_t frames = std::min<size_t>(std::min<size_t>((size_t)T, (size_t)chunk_cap(form)),
                                           std::max<size_t>(1, ctx->budget / pf));
    const size_t need = pf * frames;
    moco_graph *gr = new (std::nothrow) moco_graph;
    if (!gr) return fail(MOCO_ENOMEM, "moco_graph_create: out of host memory");
    gr->device = ctx->device;
    hipStream_t cs = nullptr;
    hipGraph_t graph_ = nullptr;
    hipError_t e = hipMalloc(&gr->scratch, need);
    if (e != hipSuccess) {
        delete gr;
        return fail(MOCO_ENOMEM, "graph scratch of %zu bytes: %s", need, hipGetErrorString(e));
    }
    // capture on a private stream (the legacy default stream cannot be
    // captured); no stage timing inside a graph
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = run_stack(ctx, d_frames, tt, T, g, form, out, cs, (char *)gr->scratch, need);
        hipError_t e2 = hipStreamEndCapture(cs, &graph_);
        if (rc == MOCO_OK && e2 != hipSuccess)
            rc = fail(MOCO_EDEVICE, "graph capture: %s", hipGetErrorString(e2));
        if (rc == MOCO_OK && (e2 = hipGraphInstantiate(&gr->exec, graph_, nullptr, nullptr, 0)) !=
                                 hipSuccess)
            rc = fail(MOCO_EDEVICE, "graph instantiation: %s", hipGetErrorString(e2));
    } else {
        rc = fail(MOCO_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    ctx->profiling = prof;
    if (graph_) (void)hipGraphDestroy(graph_);
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != MOCO_OK) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        (void)hipFree(gr->scratch);
        delete gr;
        return rc;
    }
    *graph = gr;
    return MOCO_OK;
}

int moco_graph_launch(moco_graph *graph, void *hip_stream)
{
    if (!graph || !graph->exec) return fail(MOCO_EINVAL, "moco_graph_launch: null graph");
    DeviceGuard dg(graph->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", graph->device);
    hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(MOCO_EDEVICE, "graph launch: %s", hipGetErrorString(e));
    return MOCO_OK;
}

void moco_graph_destroy(moco_graph *graph)
{
    if (!graph) return;
    DeviceGuard dg(graph->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->scratch) (void)hipFree(graph->scratch);
    delete graph;
}

int moco_align_batch(moco_ctx *ctx, const moco_stack *stacks, int nstacks, moco_form form,
                     int lanes, void *hip_stream)
{
    if (!ctx || (nstacks > 0 && !stacks) || nstacks < 0)
        return fail(MOCO_EINVAL, "moco_align_batch: null ctx or stacks, or nstacks < 0");
    BatchPlan bp;
    int rc = plan_batch(ctx, stacks, nstacks, form, lanes, &bp);
    if (rc || bp.nl == 0) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = (hipStream_t)hip_stream;
    const int nl = bp.nl;
    rc = ensure_scratch(ctx, bp.slice * nl, st);
    if (rc) return rc;
    while ((int)ctx->lanes.size() < nl) {
        hipStream_t l = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&l, hipStreamNonBlocking));
        ctx->lanes.push_back(l);
    }
    while ((int)ctx->lane_ev.size() < nl + 1) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->lane_ev.push_back(e);
    }
    return enqueue_batch(ctx, stacks, bp, st, (char *)ctx->scratch, ctx->lanes.data(),
                         ctx->lane_ev.data());
}

int moco_graph_create_batch(moco_ctx *ctx, const moco_stack *stacks, int nstacks, moco_form form,
                            int lanes, moco_graph **graph)
{
    if (!ctx || !graph || (nstacks > 0 && !stacks) || nstacks < 0)
        return fail(MOCO_EINVAL, "moco_graph_create_batch: null argument or nstacks < 0");
    *graph = nullptr;
    BatchPlan bp;
    int rc = plan_batch(ctx, stacks, nstacks, form, lanes, &bp);
    if (rc) return rc;
    if (bp.nl == 0) return fail(MOCO_EINVAL, "moco_graph_create_batch: no frame to align");
    DeviceGuard dg(ctx->device);
    if (!dg.ok()) return fail(MOCO_EDEVICE, "cannot select device %d", ctx->device);
    const int nl = bp.nl;
    moco_graph *gr = new (std::nothrow) moco_graph;
    if (!gr) return fail(MOCO_ENOMEM, "moco_graph_create_batch: out of host memory");
    gr->device = ctx->device;
    hipError_t e = hipMalloc(&gr->scratch, bp.slice * nl);
    if (e != hipSuccess) {
        delete gr;
        return fail(MOCO_ENOMEM, "graph scratch of %zu bytes: %s", bp.slice * nl,
                    hipGetErrorString(e));
    }
    // capture on streams of its own: the origin stream forks to nl lane
    // streams through events and joins them again, all inside the capture
    std::vector<hipStream_t> ls(nl, nullptr);
    std::vector<hipEvent_t> ev(nl + 1, nullptr);
    hipStream_t cs = nullptr;
    hipGraph_t graph_ = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int l = 0; l < nl && e == hipSuccess; ++l)
        e = hipStreamCreateWithFlags(&ls[l], hipStreamNonBlocking);
    for (int l = 0; l <= nl && e == hipSuccess; ++l)
        e = hipEventCreateWithFlags(&ev[l], hipEventDisableTiming);
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue_batch(ctx, stacks, bp, cs, (char *)gr->scratch, ls.data(), ev.data());
        hipError_t e2 = hipStreamEndCapture(cs, &graph_);
        if (rc == MOCO_OK && e2 != hipSuccess)
            rc = fail(MOCO_EDEVICE, "graph capture: %s", hipGetErrorString(e2));
        if (rc == MOCO_OK && (e2 = hipGraphInstantiate(&gr->exec, graph_, nullptr, nullptr, 0)) !=
                                 hipSuccess)
            rc = fail(MOCO_EDEVICE, "graph instantiation: %s", hipGetErrorString(e2));
    } else {
        rc = fail(MOCO_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    ctx->profiling = prof;
    if (graph_) (void)hipGraphDestroy(graph_);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    for (hipStream_t x : ls)
        if (x) (void)hipStreamDestroy(x);
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != MOCO_OK) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        (void)hipFree(gr->scratch);
        delete gr;
        return rc;
    }
    *graph = gr;
    return MOCO_OK;
}

}  // extern "C"

// ===========================================================================
// Serving: continuous batching of single frames from many sources.
// ===========================================================================
namespace {

using Clock = std::chrono::steady_clock;

struct SrvSource {
    moco_tmpl *tmpl = nullptr;
    moco::Geom g{};
    moco_form form = MOCO_FORM_AUTO;
    size_t fbytes = 0;
    size_t pf = 0;
};

// A request carries what the worker needs of its source, copied under the
// server's lock at submission: the worker never reads the source table.
struct SrvRequest {
    uint64_t tag;
    int source;
    int slot;
    Clock::time_point t0;
    const moco::Tmpl *tmpl;
    moco::Geom g;
    moco_form form;
    size_t fbytes;
};

// Streams on which a lane runs the source groups of a batch side by side.
constexpr int kSrvSubStreams = 4;
constexpr int kSrvLanes = 2;       // batches in flight at once (four measured slower)
constexpr long kPollSpinUs = 1000;  // moco_server_poll looks for results this long before sleeping

// Device and pinned buffers of one batch in flight.
struct SrvLane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t staged = nullptr;                 // the batch's frames are on the device
    hipStream_t sub[kSrvSubStreams] = {};        // default priority, like every stream here
    hipEvent_t sub_done[kSrvSubStreams] = {};
    char *d_frames = nullptr, *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    int32_t *d_shifts = nullptr, *d_coarse = nullptr;
    double *d_fmin = nullptr, *d_frefine = nullptr, *d_gaps = nullptr;
    int32_t *h_shifts = nullptr, *h_coarse = nullptr;
    double *h_fmin = nullptr, *h_frefine = nullptr, *h_gaps = nullptr;
    char *d_meta = nullptr, *h_meta = nullptr;   // multi-template tables of a batch
    size_t meta_bytes = 0;
    std::vector<SrvRequest> reqs;
    bool active = false;
    bool enqueuing = false;   // its launches are being issued (completion not yet recorded)
    int status = MOCO_OK;
};

}  // namespace

struct moco_server {
    moco_ctx *ctx = nullptr;  // the server's own context
    size_t budget = 0;
    int max_slots = 0;
    std::map<int, SrvSource> sources;
    size_t slot_bytes = 0;  // largest frame of any source
    size_t pf_max = 0;      // largest per-frame scratch of any source
    size_t tmpl_bytes = 0;  // device bytes held by prepared templates (estimate)
    char *h_slots = nullptr;  // pinned staging, max_slots x slot_bytes
    std::vector<int> free_slots;
    SrvLane lane[kSrvLanes];
    hipStream_t setup = nullptr;
    std::deque<SrvRequest> pending;
    std::deque<moco_result> completed;
    int inflight = 0;
    int staging = 0;  // submits holding a slot while they copy into it (lock released)
    bool launching = false;   // a batch is being enqueued (by the worker or a submit)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::thread worker;
};

namespace {

void lane_free(SrvLane &L)
{
    if (L.d_frames) (void)hipFree(L.d_frames);
    if (L.d_scratch) (void)hipFree(L.d_scratch);
    if (L.d_shifts) (void)hipFree(L.d_shifts);
    if (L.h_shifts) (void)hipHostFree(L.h_shifts);
    if (L.d_meta) (void)hipFree(L.d_meta);
    if (L.h_meta) (void)hipHostFree(L.h_meta);
    L.d_frames = L.d_scratch = nullptr;
    L.d_shifts = nullptr;
    L.h_shifts = nullptr;
    L.d_meta = L.h_meta = nullptr;
}

// Bytes of a batch's multi-template tables: a group of F frames takes
// Int8MultiTables::bytes(F) rounded up to 256, there are at most max_slots
// frames and as many groups.
size_t srv_meta_bytes(size_t ns) { return ns * (Int8MultiTables::bytes(1) + 256) + 256; }

// (Re)size the slot staging and both lanes for max_slots frames of slot_bytes
// with pf_max scratch each.  Called with no batch in flight.
int server_size_buffers(moco_server *srv, size_t slot_bytes, size_t pf_max)
{
    const size_t ns = (size_t)srv->max_slots;
    const size_t res_i32 = ns * 4 * sizeof(int32_t);            // shifts + coarse
    const size_t res_f64 = ns * (1 + 9 + 2) * sizeof(double);   // fmin, frefine, gaps
    const size_t per_lane = ns * slot_bytes + ns * pf_max + res_i32 + res_f64 + 4096;
    if (kSrvLanes * per_lane + srv->tmpl_bytes > srv->budget)
        return fail(MOCO_ENOMEM, "server needs %zu device bytes for %d slots, budget is %zu",
                    kSrvLanes * per_lane + srv->tmpl_bytes, srv->max_slots, srv->budget);
    if (srv->h_slots) (void)hipHostFree(srv->h_slots);
    srv->h_slots = nullptr;
    hipError_t e = hipHostMalloc((void **)&srv->h_slots, ns * slot_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return fail(MOCO_ENOMEM, "pinned staging: %s", hipGetErrorString(e));
    for (auto &L : srv->lane) {
        lane_free(L);
        L.meta_bytes = srv_meta_bytes(ns);
        if ((e = hipMalloc(&L.d_frames, ns * slot_bytes)) != hipSuccess ||
            (e = hipMalloc(&L.d_scratch, ns * pf_max)) != hipSuccess ||
            (e = hipMalloc(&L.d_shifts, res_i32 + res_f64)) != hipSuccess ||
            (e = hipHostMalloc((void **)&L.h_shifts, res_i32 + res_f64, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipMalloc(&L.d_meta, L.meta_bytes)) != hipSuccess ||
            (e = hipHostMalloc((void **)&L.h_meta, L.meta_bytes, hipHostMallocDefault)) !=
                hipSuccess)
            return fail(MOCO_ENOMEM, "server buffers: %s", hipGetErrorString(e));
        L.scratch_bytes = ns * pf_max;
        L.d_coarse = L.d_shifts + 2 * ns;
        L.d_fmin = (double *)(L.d_coarse + 2 * ns);
        L.d_frefine = L.d_fmin + ns;
        L.d_gaps = L.d_frefine + 9 * ns;
        L.h_coarse = L.h_shifts + 2 * ns;
        L.h_fmin = (double *)(L.h_coarse + 2 * ns);
        L.h_frefine = L.h_fmin + ns;
        L.h_gaps = L.h_frefine + 9 * ns;
    }
    srv->slot_bytes = slot_bytes;
    srv->pf_max = pf_max;
    return MOCO_OK;
}

// Enqueue one batch on its lane: frames host -> device, the search per group,
// results device -> host, completion event.  Requests of the int8 form whose
// templates share a geometry (and digit base) form one group, run as one
// launch per stage over every source's frames (run_int8_multi, its template
// tables staged with the frames); the others form one group per source (a
// run_stack each).  Groups run side by side on the lane's sub-streams, each on
// its own slice of the lane's scratch (max_slots frames of the largest
// per-frame scratch, so a group of requests a .. b-1 owns frames a .. b-1 of
// it).
int server_enqueue(moco_server *srv, SrvLane &L)
{
    auto key = [](const SrvRequest &q) {
        const moco::Tmpl &t = *q.tmpl;
        return std::make_tuple((int)q.form, t.g.m, t.g.n, t.g.w, t.g.ds, (int)t.g.dtype,
                               t.i8.npad, t.i8.trow, t.i8.padl, t.i8.dbits, t.i8.nq, q.source);
    };
    std::stable_sort(L.reqs.begin(), L.reqs.end(),
                     [&](const SrvRequest &x, const SrvRequest &y) { return key(x) < key(y); });
    const size_t nb = L.reqs.size();
    std::vector<size_t> off(nb);
    size_t o = 0;
    for (size_t k = 0; k < nb; ++k) {
        off[k] = o;
        o += L.reqs[k].fbytes;
    }
    // the groups, and the multi-template tables of the int8 ones
    struct Group {
        size_t a, b;
        bool multi;
        int nblocks;
        size_t meta_off;
    };
    std::vector<Group> groups;
    size_t meta_used = 0;
    std::vector<const moco::Tmpl *> tl;
    for (size_t a = 0; a < nb;) {
        const SrvRequest &q = L.reqs[a];
        size_t b = a + 1;
        const bool multi =
            q.form == MOCO_FORM_INT8_MFMA &&
            (q.g.ds == 0 || moco::refine_rolling(q.g, L.d_frames + off[a], q.tmpl->raw));
        if (multi) {
            while (b < nb && L.reqs[b].form == MOCO_FORM_INT8_MFMA &&
                   int8_multi_key_equal(*L.reqs[b].tmpl, *q.tmpl))
                ++b;
        } else {
            while (b < nb && L.reqs[b].source == q.source) ++b;
        }
        Group gr{a, b, multi, 0, meta_used};
        if (multi) {
            const int F = (int)(b - a);
            tl.resize(F);
            for (int f = 0; f < F; ++f) tl[f] = L.reqs[a + f].tmpl;
            Int8MultiTables ht;
            ht.place(L.h_meta + meta_used, F);
            gr.nblocks = fill_int8_multi(tl.data(), F, ht);
            meta_used = align_up(meta_used + Int8MultiTables::bytes(F), 256);
            if (meta_used > L.meta_bytes) return fail(MOCO_ENOMEM, "server tables overflow");
        }
        groups.push_back(gr);
        a = b;
    }
    for (size_t k = 0; k < nb; ++k) {
        const SrvRequest &q = L.reqs[k];
        HIP_TRY(hipMemcpyAsync(L.d_frames + off[k], srv->h_slots + (size_t)q.slot * srv->slot_bytes,
                               q.fbytes, hipMemcpyHostToDevice, L.stream));
    }
    if (meta_used)
        HIP_TRY(hipMemcpyAsync(L.d_meta, L.h_meta, meta_used, hipMemcpyHostToDevice, L.stream));
    // one group runs on the lane's stream; several fork onto its sub-streams
    const bool fork = groups.size() > 1;
    if (fork) HIP_TRY(hipEventRecord(L.staged, L.stream));
    bool used[kSrvSubStreams] = {};
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group &gr = groups[gi];
        const size_t a = gr.a, b = gr.b;
        const SrvRequest &q = L.reqs[a];
        const int k = (int)(gi % kSrvSubStreams);
        const hipStream_t gs = fork ? L.sub[k] : L.stream;
        if (fork && !used[k]) {
            HIP_TRY(hipStreamWaitEvent(L.sub[k], L.staged, 0));
            used[k] = true;
        }
        moco_outputs out{};
        out.shifts = L.d_shifts + 2 * a;
        out.coarse = L.d_coarse + 2 * a;
        out.fmin = L.d_fmin + a;
        out.frefine = L.d_frefine + 9 * a;
        out.gaps = L.d_gaps + 2 * a;
        int rc;
        if (gr.multi) {
            Int8MultiTables dt;
            dt.place(L.d_meta + gr.meta_off, (int)(b - a));
            rc = run_int8_multi(srv->ctx, L.d_frames + off[a], *q.tmpl, (int)(b - a), gr.nblocks, dt,
                                &out, gs, L.d_scratch + a * srv->pf_max,
                                (b - a) * srv->pf_max);
        } else {
            rc = run_stack(srv->ctx, L.d_frames + off[a], *q.tmpl, (int)(b - a), q.g, q.form,
                           &out, gs, L.d_scratch + a * srv->pf_max, (b - a) * srv->pf_max);
        }
        if (rc) return rc;
    }
    for (int k = 0; k < kSrvSubStreams; ++k)
        if (used[k]) {
            HIP_TRY(hipEventRecord(L.sub_done[k], L.sub[k]));
            HIP_TRY(hipStreamWaitEvent(L.stream, L.sub_done[k], 0));
        }
    const size_t ns = (size_t)srv->max_slots;
    const size_t res = ns * 4 * sizeof(int32_t) + ns * 12 * sizeof(double);
    HIP_TRY(hipMemcpyAsync(L.h_shifts, L.d_shifts, res, hipMemcpyDeviceToHost, L.stream));
    HIP_TRY(hipEventRecord(L.done, L.stream));
    return MOCO_OK;
}

// Publish the results of a finished lane (called with srv->mu held).
void server_publish(moco_server *srv, SrvLane &L)
{
    const auto now = Clock::now();
    for (size_t k = 0; k < L.reqs.size(); ++k) {
        const SrvRequest &q = L.reqs[k];
        moco_result r{};
        r.tag = q.tag;
        r.source = q.source;
        r.status = L.status;
        if (L.status == MOCO_OK) {
            r.shift[0] = L.h_shifts[2 * k];
            r.shift[1] = L.h_shifts[2 * k + 1];
            r.coarse[0] = L.h_coarse[2 * k];
            r.coarse[1] = L.h_coarse[2 * k + 1];
            r.fmin = L.h_fmin[k];
            for (int u = 0; u < 9; ++u) r.frefine[u] = L.h_frefine[9 * k + u];
            r.gaps[0] = L.h_gaps[2 * k];
            r.gaps[1] = L.h_gaps[2 * k + 1];
        }
        r.latency_us = std::chrono::duration<double, std::micro>(now - q.t0).count();
        srv->completed.push_back(r);
        srv->free_slots.push_back(q.slot);
    }
    srv->inflight -= (int)L.reqs.size();
    L.reqs.clear();
    L.active = false;
}

// Launch the waiting requests into the free lane L (called with srv->mu held,
// by the worker or by a submit, never by two at once: srv->launching).  The
// lane is marked as enqueuing meanwhile, so that the worker does not query
// its completion event before this batch has recorded it.
void server_launch(moco_server *srv, SrvLane &L, std::unique_lock<std::mutex> &lk)
{
    while (!srv->pending.empty() && (int)L.reqs.size() < srv->max_slots) {
        L.reqs.push_back(srv->pending.front());
        srv->pending.pop_front();
    }
    L.active = true;
    L.enqueuing = true;
    srv->launching = true;
    lk.unlock();
    int rc;
    {
        DeviceGuard dg(srv->ctx->device);
        rc = dg.ok() ? server_enqueue(srv, L) : fail(MOCO_EDEVICE, "server: cannot select the device");
    }
    if (rc != MOCO_OK) {
        // the batch never reached the GPU in full: wait for what did, then fail it
        (void)hipStreamSynchronize(L.stream);
        for (int k = 0; k < kSrvSubStreams; ++k) (void)hipStreamSynchronize(L.sub[k]);
    }
    lk.lock();
    L.status = rc;
    L.enqueuing = false;
    srv->launching = false;
    if (rc != MOCO_OK) server_publish(srv, L);
    srv->cv_work.notify_all();   // the worker polls the lane, or launches what waits
    srv->cv_done.notify_all();
}

bool server_any_active(const moco_server *srv)
{
    for (const auto &L : srv->lane)
        if (L.active) return true;
    return false;
}

void server_loop(moco_server *srv)
{
    (void)hipSetDevice(srv->ctx->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        if (!server_any_active(srv)) {
            srv->cv_work.wait(lk, [&] {
                return srv->stop || !srv->pending.empty() || server_any_active(srv);
            });
            if (srv->stop && srv->pending.empty() && !server_any_active(srv)) break;
        }
        // launch the waiting requests into a free lane
        if (!srv->launching && !srv->pending.empty() && !srv->stop) {
            SrvLane *fl = nullptr;
            for (auto &L : srv->lane)
                if (!L.active) {
                    fl = &L;
                    break;
                }
            if (fl) {
                server_launch(srv, *fl, lk);
                continue;
            }
        }
        // finish lanes whose batch has completed, oldest first (only this
        // thread publishes a lane whose launches were all issued, so the lane
        // keeps its state while the lock is released for the query)
        bool progressed = false;
        for (auto &L : srv->lane) {
            if (!L.active || L.enqueuing) continue;
            lk.unlock();
            hipError_t q = hipEventQuery(L.done);
            lk.lock();
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) L.status = MOCO_EDEVICE;
            server_publish(srv, L);
            progressed = true;
        }
        if (progressed) {
            srv->cv_done.notify_all();
            continue;
        }
        if (srv->stop && srv->pending.empty() && !server_any_active(srv))
            break;
        // a batch is on the GPU: poll its event again after yielding the lock
        // and the core (a timed wait sleeps for the scheduler's timer slack:
        // one source's single-frame requests took 222 us at p50 with a 20 us
        // wait, 176 us polling)
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
    }
}

}  // namespace

extern "C" {

int moco_server_create(moco_ctx *ctx, size_t device_budget_bytes, int max_slots,
                       moco_server **out)
{
    if (!ctx || !out || max_slots < 1)
        return fail(MOCO_EINVAL, "moco_server_create: null ctx/out or max_slots < 1");
    *out = nullptr;
    moco_server *srv = new (std::nothrow) moco_server;
    if (!srv) return fail(MOCO_ENOMEM, "out of host memory");
    srv->budget = device_budget_bytes ? device_budget_bytes : (size_t)1 << 30;
    srv->max_slots = max_slots;
    int rc = moco_create(ctx->device, srv->budget, &srv->ctx);
    if (rc) {
        delete srv;
        return rc;
    }
    DeviceGuard dg(ctx->device);
    hipError_t e = hipStreamCreateWithFlags(&srv->setup, hipStreamNonBlocking);
    for (auto &L : srv->lane) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.staged, hipEventDisableTiming);
        for (int k = 0; k < kSrvSubStreams && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&L.sub[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&L.sub_done[k], hipEventDisableTiming);
        }
    }
    if (e != hipSuccess) {
        moco_server_destroy(srv);
        return fail(MOCO_EDEVICE, "server streams: %s", hipGetErrorString(e));
    }
    srv->worker = std::thread(server_loop, srv);
    *out = srv;
    return MOCO_OK;
}

int moco_server_add_source(moco_server *srv, int source, const void *h_template,
                           moco_dtype dtype, int m, int n, int w, int downsample)
{
    if (!srv || !h_template) return fail(MOCO_EINVAL, "moco_server_add_source: null argument");
    moco::Geom g;
    int rc = validate(m, n, w, downsample, dtype, &g);
    if (rc) return rc;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->sources.count(source)) return fail(MOCO_EINVAL, "source %d already exists", source);
    DeviceGuard dg(srv->ctx->device);
    const size_t fbytes = (size_t)m * n * dtype_size(dtype);
    void *d_t = nullptr;
    hipError_t e = hipMalloc(&d_t, fbytes);
    if (e != hipSuccess) return fail(MOCO_ENOMEM, "template upload: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d_t, h_template, fbytes, hipMemcpyHostToDevice, srv->setup);
    if (e == hipSuccess) e = hipStreamSynchronize(srv->setup);
    moco_tmpl *tp = nullptr;
    rc = e == hipSuccess ? moco_template_create(srv->ctx, d_t, dtype, m, n, w, downsample,
                                                srv->setup, &tp)
                         : fail(MOCO_EDEVICE, "template upload: %s", hipGetErrorString(e));
    (void)hipFree(d_t);
    if (rc) return rc;
    SrvSource sc;
    sc.tmpl = tp;
    sc.g = g;
    moco_form resolved = MOCO_FORM_AUTO;
    (void)moco_template_form(tp, MOCO_FORM_AUTO, &resolved);
    // the certified FP32 form is not served: float32 sources run the FP64 one
    if (resolved == MOCO_FORM_FFT32_CERTIFIED) resolved = MOCO_FORM_FFT_CERTIFIED;
    sc.form = resolved;
    sc.fbytes = fbytes;
    sc.pf = per_frame_scratch(g, resolved, tp->t);
    const size_t tb = fbytes + (size_t)g.mg * g.ng * 8 + (size_t)g.W * g.W * 16 +
                      (tp->t.int8_ok ? moco::int8_template_bytes(g, tp->t.i8.nq) : 0) +
                      (tp->t.fft_ok ? (size_t)tp->t.fft.qh * tp->t.fft.pp.n * sizeof(double2) : 0);
    // larger frames or scratch than the buffers hold: resize once nothing is in flight
    if (fbytes > srv->slot_bytes || sc.pf > srv->pf_max) {
        // nothing may hold a slot or a lane while the buffers are replaced
        srv->cv_done.wait(lk, [&] {
            return srv->pending.empty() && srv->inflight == 0 && srv->staging == 0;
        });
        srv->tmpl_bytes += tb;
        rc = server_size_buffers(srv, std::max(fbytes, srv->slot_bytes),
                                 std::max(sc.pf, srv->pf_max));
        if (rc) {
            srv->tmpl_bytes -= tb;
            moco_template_destroy(tp);
            return rc;
        }
        srv->free_slots.clear();
        for (int k = srv->max_slots - 1; k >= 0; --k) srv->free_slots.push_back(k);
    } else {
        srv->tmpl_bytes += tb;
    }
    srv->sources[source] = sc;
    return MOCO_OK;
}

int moco_server_submit(moco_server *srv, int source, const void *h_frame, uint64_t tag)
{
    if (!srv || !h_frame) return fail(MOCO_EINVAL, "moco_server_submit: null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->sources.find(source);
    if (it == srv->sources.end()) return fail(MOCO_EINVAL, "unknown source %d", source);
    if (srv->stop) return fail(MOCO_ECANCELED, "server is shutting down");
    if (srv->free_slots.empty()) return MOCO_EBUSY;
    const int slot = srv->free_slots.back();
    srv->free_slots.pop_back();
    const SrvSource &sc = it->second;
    SrvRequest q{tag, source, slot, Clock::now(), &sc.tmpl->t, sc.g, sc.form, sc.fbytes};
    // the copy runs unlocked; `staging` keeps the slot buffers from being
    // replaced (a source that needs larger slots) or freed (destroy) meanwhile
    srv->staging += 1;
    char *dst = srv->h_slots + (size_t)slot * srv->slot_bytes;
    lk.unlock();
    std::memcpy(dst, h_frame, q.fbytes);
    lk.lock();
    srv->staging -= 1;
    if (srv->stop) {
        srv->free_slots.push_back(slot);
        srv->cv_done.notify_all();
        return fail(MOCO_ECANCELED, "server is shutting down");
    }
    srv->pending.push_back(q);
    srv->inflight += 1;
    // an idle server (no batch in flight, so the worker may be asleep): start
    // the batch from here, so that it does not wait for the worker to wake
    // up; while batches run, the worker is awake and gathers what waits into
    // the next one
    if (!srv->launching && !server_any_active(srv)) server_launch(srv, srv->lane[0], lk);
    srv->cv_work.notify_one();
    srv->cv_done.notify_all();
    return MOCO_OK;
}

int moco_server_poll(moco_server *srv, moco_result *results, int max, int timeout_us)
{
    if (!srv || (max > 0 && !results) || max < 0)
        return fail(MOCO_EINVAL, "moco_server_poll: bad arguments");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&] { return !srv->completed.empty(); };
    auto idle = [&] { return timeout_us < 0 && srv->inflight == 0; };
    if (timeout_us != 0 && !ready() && !idle()) {
        // results usually follow within a batch's time: look for them, yielding
        // the lock and the core, for up to kPollSpinUs before sleeping, so that
        // a result is not held up by this thread's wake-up
        const auto t0 = Clock::now();
        const long spin = timeout_us < 0 ? kPollSpinUs : std::min<long>(timeout_us, kPollSpinUs);
        const auto until = t0 + std::chrono::microseconds(spin);
        while (!ready() && !idle() && Clock::now() < until) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
        if (timeout_us < 0) {
            srv->cv_done.wait(lk, [&] { return ready() || srv->inflight == 0; });
        } else if (!ready()) {
            const auto left = std::chrono::microseconds(timeout_us) -
                              std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - t0);
            if (left.count() > 0) srv->cv_done.wait_for(lk, left, ready);
        }
    }
    int k = 0;
    while (k < max && !srv->completed.empty()) {
        results[k++] = srv->completed.front();
        srv->completed.pop_front();
    }
    return k;
}

int moco_server_pending(moco_server *srv)
{
    if (!srv) return 0;
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->inflight;
}

int moco_server_destroy(moco_server *srv)
{
    if (!srv) return 0;
    int cancelled = 0;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->stop = true;
        // submits still copying into their slots finish (and cancel themselves),
        // and a batch being launched by a submit is fully enqueued
        srv->cv_done.wait(lk, [&] { return srv->staging == 0 && !srv->launching; });
        cancelled = (int)srv->pending.size();
        for (auto &q : srv->pending) srv->free_slots.push_back(q.slot);
        srv->inflight -= cancelled;
        srv->pending.clear();
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    {
        DeviceGuard dg(srv->ctx ? srv->ctx->device : 0);
        for (auto &L : srv->lane) {
            if (L.stream) (void)hipStreamSynchronize(L.stream);
            for (int k = 0; k < kSrvSubStreams; ++k)
                if (L.sub[k]) (void)hipStreamSynchronize(L.sub[k]);
            lane_free(L);
            if (L.done) (void)hipEventDestroy(L.done);
            if (L.staged) (void)hipEventDestroy(L.staged);
            for (int k = 0; k < kSrvSubStreams; ++k) {
                if (L.sub_done[k]) (void)hipEventDestroy(L.sub_done[k]);
                if (L.sub[k]) (void)hipStreamDestroy(L.sub[k]);
            }
            if (L.stream) (void)hipStreamDestroy(L.stream);
        }
        for (auto &kv : srv->sources) moco_template_destroy(kv.second.tmpl);
        if (srv->h_slots) (void)hipHostFree(srv->h_slots);
        if (srv->setup) (void)hipStreamDestroy(srv->setup);
    }
    if (srv->ctx) moco_destroy(srv->ctx);
    delete srv;
    return cancelled;
}

}  // extern "C"
