// Internal declarations shared by the C ABI (capi.cpp) and the HIP kernels.
// Not installed; the public interface is include/moco.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "moco.h"

namespace moco {

// Geometry of one search: full-resolution m x n, `ds` levels of 2x2
// downsampling (0: none), searched grid mg x ng = (m >> ds) x (n >> ds),
// window w (W = 2w-1 shifts per axis).
struct Geom {
    int m, n, mg, ng, w, W, ds;
    moco_dtype dtype;
};
constexpr int kMaxLevels = 4;

// Geometry of the int8 form: grid columns padded to a multiple of 32, and the
// template rows laid out with `padl` leading zero bytes in rows of `trow`.
struct Int8Geom {
    int npad, padl, trow;
};

// Template side of the int8 form (device memory owned by the template).  Digits
// of base 2^dbits: 128 with nq = 3 template planes (the two digits and their
// sum; three digit products per term), or 256 with nq = 2 (four products).
struct Int8Tmpl {
    int8_t *tp = nullptr;          // [mg][nq][8][trow] digit rows of the template, 8 byte phases
    int32_t vmax = -1;             // bound of the template's pixel values (-1: none)
    long long *atab = nullptr;     // [W][W] sum of Y^2 over the frame-side rows of D at (s,t);
                                   // the template energy at (s,t) is this table at (-s,-t)
    int npad = 0, padl = 0, trow = 0;
    int dbits = 8, nq = 2;
};

// One-dimensional transform plan: length n = product of the radices, applied
// in order; ns[p] is the product of the radices before pass p.  mag_* are
// ceil(2^32 / d) for d = n / radix[p] and d = ns[p] (division by multiply).
constexpr int kFftMaxLen = 2048;
constexpr int kFftMaxPass = 16;
struct FftPlan {
    int n = 0, npass = 0;
    int radix[kFftMaxPass];
    int ns[kFftMaxPass];
    unsigned long long mag_nr[kFftMaxPass];
    unsigned long long mag_ns[kFftMaxPass];
};

// Transform sizes of the FFT form: P >= mg+w-1, Q >= ng+w-1, both 5-smooth;
// qh = Q/2+1 half-spectrum bins.
struct FftGeom {
    int P, Q, qh;
};

// Template side of the FFT forms (device memory owned by the template).
struct FftTmpl {
    FftPlan pp, pq;                 // column (length P) and row (length Q) plans
    int qh = 0;
    double2 *twp = nullptr;         // w_P^k = exp(-2 pi i k/P), k < P
    double2 *twq = nullptr;         // w_Q^k, k < Q
    double2 *spec = nullptr;        // [qh][P] 2-D transform of the zero-padded b'
    // the single-precision form: grids centred on `center` (the template
    // grid's mean, an integer for uint16 data) before the transforms
    double center = 0.0;
    float2 *twp32 = nullptr;        // the twiddle tables rounded to FP32
    float2 *twq32 = nullptr;
    float2 *spec32 = nullptr;       // [qh][P] transform of the zero-padded b' - center
                                    // (computed in FP64, rounded)
    double *btab32 = nullptr;       // [W][W] sum of (b' - center)^2 over D_{s,t}
    double yinf32 = 0.0;            // largest |spec32| (the certificate's |Y|_inf)
};

// The single-precision form's certificate: a bound on the FP32 correlation's
// error from the norms of the centred grids and the largest magnitudes of
// their spectra (the frame's measured by the column kernel):
// |h^ - h| <= hb = 2 (e1 |x|_2 |Y|_inf + e2 (|X|_inf + e1 sqrt(PQ) |x|_2) |y|_2).
struct Cert32 {
    const float *xmax = nullptr;    // [frame][nxb] block maxima of |X_k|^2
    int nxb = 0;
    double e1 = 0.0, e2 = 0.0;      // frame transform; inverse, template and product
    double yinf = 0.0;
    double sqrtpq = 0.0;
};

// Resident, prepared template.  All pointers are device memory owned by it.
struct Tmpl {
    Geom g;
    void *raw;        // m x n pixels of g.dtype (full resolution, for the x2 refine)
    double *coarse;   // mg x ng FP64 (box mean when ds)
    double *btab;     // W x W: sum of b'^2 over D_{s,t}, [s+w-1][t+w-1]
    int32_t pbound;   // bound of the template's pixel values (uint16), -1: none
    double *pyr;      // levels 1 .. ds-1 of the template's image pyramid, FP64, one after
                      // another (nullptr when ds <= 1); level ds is `coarse`
    bool int8_ok;     // the int8 form applies (uint16, template digits fit two planes)
    Int8Tmpl i8;
    bool fft_ok;      // the FFT form applies (transform lengths within kFftMaxLen)
    FftTmpl fft;
};

// Per-frame intermediate results of the coarse search (device).
struct CoarseOut {
    int32_t s, t;     // argmin on the searched grid
};

// A failing HIP call made elsewhere in the process (by the caller, or by a
// framework sharing the thread) leaves a non-sticky error in the thread's
// last-error slot; launchers clear it first so that the status they return
// belongs to their own launch.
inline void clear_stale_error() { (void)hipGetLastError(); }

// ---- launchers (kernels_basic.hip) -------------------------------------
// All return hipSuccess or the launch error; they only enqueue.
// only (may be null): frames whose only[f] is 0 are skipped
hipError_t launch_coarse(const void *frames, moco_dtype dt, int C, const Geom &g, double *coarse,
                         hipStream_t st, const int32_t *only = nullptr);
// atab[frame][W][W]: the frame's energies over D at (s,t) ([-s][-t] when flip),
// of the grid values less `center`; pmax[frame] (may be null): a pixel bound
// for the x2 step (uint16), else INT32_MAX.  Not flipped, grids where
// energy_rows_applicable take the one-pass row kernel.
hipError_t launch_energy(const double *coarse, int C, const Geom &g, bool flip, double *atab,
                         int32_t *pmax, hipStream_t st, double center = 0.0,
                         const int32_t *only = nullptr);
// the same (not flipped) from the frames' pixels, forming the grid values as
// they are read (at most one 2x2 level): the values launch_coarse would write
hipError_t launch_energy_px(const void *frames, int C, const Geom &g, double *atab,
                            int32_t *pmax, hipStream_t st, double center = 0.0,
                            const int32_t *only = nullptr);
bool energy_rows_applicable(const Geom &g);
// only (may be null): frames whose only[f] is 0 are skipped
hipError_t launch_corr_fp64(const double *coarse, const double *tcoarse, int C, const Geom &g,
                            double *h, hipStream_t st, const int32_t *only = nullptr);
// only (may be null): frames whose only[f] is 0 are skipped.  recheck (may be
// null): recheck[f] = 0 when the argmin is certified against a correlation
// error of at most kf sqrt(m'n' Sa Sb) (or the bound of c32, when given) and
// energy errors of at most ke (Sa or Sb), else 1.
hipError_t launch_combine(const double *atab, const double *btab, const double *h, int C,
                          const Geom &g, double *fsurf, double *fmin, int32_t *coarse_st,
                          int32_t *shifts, double *gaps, double *frefine, hipStream_t st,
                          const int32_t *only = nullptr, int32_t *recheck = nullptr,
                          double kf = 0.0, double ke = 0.0, const Cert32 *c32 = nullptr);
// f at each frame's coarse argmin by its definition (FP64 sum of squared
// differences of the searched grids over D), for frames whose skip[f] is 0:
// fmin[f] and fsurf at the argmin get that value and gaps[2f] moves with it.
// fmin holds the combine's value on entry.
hipError_t launch_polish(const void *src, bool raw, int C, const Geom &g, const double *tcoarse,
                         const int32_t *coarse_st, const int32_t *skip, double *fmin,
                         double *fsurf, double *gaps, hipStream_t st);
// Frames the single-precision certificate left (recheck[f] != 0) whose open
// shifts all lie in the 3 x 3 neighbourhood of the computed argmin: exact f
// there by integer sums (uint16 pixels, at most one 2x2 level), the argmin,
// gap and surface values rewritten, recheck cleared and resolved[f] = 3;
// resolved[f] = 0 for every other frame.  atab, btab, h: the tables the
// combine formed f from.
constexpr int kCand32MaxShifts = 4096;   // (2w-1)^2 at most (w <= 32) for launch_cand32
hipError_t launch_cand32(const void *frames, int C, const Geom &g, const double *atab,
                         const double *btab, const double *h, const double *tcoarse, double ke,
                         const Cert32 &c32, int32_t *coarse_st, double *fmin, double *fsurf,
                         double *gaps, int32_t *shifts, int32_t *recheck, int32_t *resolved,
                         hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int count, int32_t v, hipStream_t st);
// p[i] += q[i], i < count
hipError_t launch_add_i32(int32_t *p, const int32_t *q, int count, hipStream_t st);
hipError_t launch_refine(const void *frames, const void *traw, int C, const Geom &g,
                         const int32_t *coarse_st, int32_t *shifts, double *frefine,
                         double *gaps, double *partial, hipStream_t st,
                         const int32_t *pmax = nullptr, int tmax = -1);
// The same for frames of several templates (uint16 rolling kernel only:
// refine_rolling must hold for the frames and every template): traws[f] and
// tmaxs[f] (device arrays) are frame f's template pixels and pixel bound (-1:
// none).
hipError_t launch_refine_multi(const uint16_t *frames, const uint16_t *const *traws,
                               const int32_t *tmaxs, int C, const Geom &g,
                               const int32_t *coarse_st, int32_t *shifts, double *frefine,
                               double *gaps, double *partial, hipStream_t st,
                               const int32_t *pmax);
// one more pyramid level: in C x m x n FP64 -> out C x (m/2) x (n/2)
hipError_t launch_half(const double *in, int C, int m, int n, double *out, hipStream_t st);
// the +-1 step at an intermediate pyramid level (FP64 images of that level):
// in_st (s,t) of the level below -> out_st the best of (2s+u, 2t+v)
hipError_t launch_refine_level(const double *frames, const double *tmpl, int C, int m, int n,
                               const int32_t *in_st, int32_t *out_st, double *partial,
                               hipStream_t st);
size_t refine_level_partial_bytes(int m, int n);   // per frame
int refine_band_rows(const Geom &g);
bool refine_u16_banded(const Geom &g);
size_t refine_partial_bytes(const Geom &g);   // per frame
// uint16, even n and 4-byte aligned frame/template buffers: the rolling kernel
bool refine_rolling(const Geom &g, const void *frames, const void *traw);
int roll_band_rows(const Geom &g, int C);

// ---- int8 form (int8_form.hip) -----------------------------------------
Int8Geom int8_geom(const Geom &g);
bool int8_applicable(const Geom &g);
// the digit-sum form (base 128, three products) also needs template rows of at
// most this many bytes
constexpr int kInt8SumMaxTrow = 512;
size_t int8_template_bytes(const Geom &g, int nq);   // Toeplitz rows + kInt8ZeroTail zero bytes
constexpr size_t kInt8ZeroTail = 1024;
// digits of base 2^dbits (7 or 8); nlimb[frame]: digit planes (2 or 3);
// vmax[frame]: an upper bound of the frame's pixel values (its largest grid
// value), or INT32_MAX when the grid does not cover every pixel (odd sides when
// downsampling)
// edge: prep_edge_bytes(g) scratch per frame.  hz (nullable): the C frames'
// correlation tables ([frame][2 W^2] int32), zeroed by the same launch for a
// correlation that adds row slices (int8_corr_adds_slices).
hipError_t launch_prep_u16(const uint16_t *frames, int C, const Geom &g, int npad, int dbits,
                           int8_t *limbs, int32_t *nlimb, int32_t *vmax, long long *atab,
                           long long *edge, hipStream_t st, int32_t *hz = nullptr);
// A few frames are split over at most kPrepMaxBands bands of rows each (one
// block per band); the bands' partial sums take prep_band_longs(w) int64 per
// frame, after the C frames' edge prefix tables.
constexpr int kPrepMaxBands = 32;
__host__ __device__ inline size_t prep_band_longs(int w)
{
    return 2 * (size_t)(w - 1) + (size_t)kPrepMaxBands * (2 * (size_t)(w - 1) + 3);
}
// Per-frame scratch of the prep pass: the border prefix tables
// [2][2][w-1][w] int64 and the bands' partial sums.
inline size_t prep_edge_bytes(const Geom &g)
{
    return ((size_t)4 * (g.w - 1) * g.w + prep_band_longs(g.w)) * sizeof(long long);
}
hipError_t launch_tpad(const int8_t *tlimbs, const Geom &g, const Int8Tmpl &tt, hipStream_t st);
// The FP64 forms' grid and energies for uint16 frames with at most one 2x2
// level, in one pass over the raw frames (the prep kernel without digit
// planes): grid [frame][mg][ng] FP64 (may be null: energies only), atab
// [frame][W][W] FP64 in grid units, vmax as launch_prep_u16; edge:
// prep_edge_bytes scratch per frame; only (may be null): frames whose
// only[f] is 0 are skipped.
bool prep_grid_applicable(const Geom &g);
// xc: the energies are of X - xc (X the integer grid values: box sums or
// counts), for the single-precision FFT form's centred grids; 0 otherwise.
hipError_t launch_prep_grid(const uint16_t *frames, int C, const Geom &g, double *grid,
                            double *atab, int32_t *vmax, long long *edge, hipStream_t st,
                            const int32_t *only = nullptr, int xc = 0);
// Frames of several templates of one geometry in one correlation launch
// (device arrays): block-column x takes frames bf0[x] .. bfe[x]-1 (at most
// four, consecutive) against the template rows btp[x].
struct Int8Multi {
    int nblocks;
    const int8_t *const *btp;
    const int *bf0, *bfe;
};
// mm (nullable): the frames' templates as above; tt then gives the geometry
// (npad, trow, padl, digit base), which every template of the launch shares.
// tile: shift tiles per block, 32 (one 32x32 tile, ceil(W/32)^2 block groups)
// or 64 (2x2 tiles of 32, ceil(W/64)^2 groups); 0: 32 when W <= 32, else 64.
// h_zeroed: the table h is already zero (the prep launch cleared it), so a
// launch that adds row slices into it does not clear it first.
hipError_t launch_corr_int8(const int8_t *limbs, const int32_t *nlimb, const Int8Tmpl &tt, int C,
                            const Geom &g, long long *h, hipStream_t st,
                            const Int8Multi *mm = nullptr, int tile = 0, bool h_zeroed = false);
// Whether that launch (C frames, tile, nblocks = mm->nblocks or -1) splits the
// template rows over blocks that add into a zeroed table.
bool int8_corr_adds_slices(int C, const Geom &g, int tile, int nblocks = -1);
// btabs (nullable, device array): each frame's own template table
hipError_t launch_combine_i64(const long long *atab, const long long *btab_t, const long long *h,
                              int C, const Geom &g, double *fsurf, double *fmin,
                              int32_t *coarse_st, int32_t *shifts, double *gaps, double *frefine,
                              hipStream_t st, const long long *const *btabs = nullptr);

// ---- FFT form (fft_form.hip) --------------------------------------------
bool fft_plan(int n, FftPlan *pl);
FftGeom fft_geom(const Geom &g);
bool fft_applicable(const Geom &g);
// coefficients of the certificate: |h^ - h| <= kf sqrt(m'n' Sa Sb), energy
// errors <= ke Sa (Sa, Sb: the grids' sums of squares)
void fft_error_coefs(const Geom &g, const FftTmpl &ft, double *kf, double *ke);
// e1, e2 of Cert32 for the template's transform lengths
void fft32_cert_coefs(const FftTmpl &ft, double *e1, double *e2);
// per frame: [qh][mg] and [W][qh] complex elements of esz bytes
size_t fft_s1_bytes(const Geom &g, size_t esz = sizeof(double2));
size_t fft_s2_bytes(const Geom &g, size_t esz = sizeof(double2));
// only (may be null) on the FFT passes: frames whose only[f] is 0 are skipped
hipError_t launch_fft_rows(const double *grid, int C, const Geom &g, const FftTmpl &ft,
                           double2 *s1, hipStream_t st, const int32_t *only = nullptr);
// the same from the frames' pixels (at most one 2x2 level), forming the
// grid's FP64 values (box means, or the pixels) as the rows are read
hipError_t launch_fft_rows_px(const void *frames, int C, const Geom &g, const FftTmpl &ft,
                              double2 *s1, hipStream_t st, const int32_t *only = nullptr);
hipError_t launch_fft_spec(const double2 *s1, const Geom &g, const FftTmpl &ft, double2 *spec,
                           hipStream_t st);
hipError_t launch_fft_corr(const double2 *s1, int C, const Geom &g, const FftTmpl &ft,
                           double2 *s2, double *h, hipStream_t st, const int32_t *only = nullptr);
// The single-precision form: the same passes in FP32 on the grids less
// ft.center (ft.twp32, twq32, spec32); h (of the centred grids) in FP64.
hipError_t launch_fft32_rows(const double *grid, int C, const Geom &g, const FftTmpl &ft,
                             float2 *s1, hipStream_t st);
hipError_t launch_fft32_rows_px(const void *frames, int C, const Geom &g, const FftTmpl &ft,
                                float2 *s1, hipStream_t st);
// xmax (may be null): [frame][*nxb] maxima of |X_k|^2 over the frame's
// spectrum, one per column block (*nxb, may be null, gets their count, at most
// the number of bins)
hipError_t launch_fft32_corr(const float2 *s1, int C, const Geom &g, const FftTmpl &ft,
                             float2 *s2, double *h, hipStream_t st, float *xmax = nullptr,
                             int *nxb = nullptr);

// ---- the corrected stack and its mean image (apply.hip) ---------------
// frames per chunk of the mean's partial sums (0: one chunk of [m][n] FP64
// partial sums exceeds `budget`)
int apply_chunk_frames(int T, int m, int n, size_t budget);
// out (nullable): corrected frames, same dtype; mean (nullable): [m][n] FP64,
// needs partial: ceil(T/kchunk) x m x n FP64
hipError_t launch_apply(const void *frames, moco_dtype dt, const int32_t *shifts, int T, int m,
                        int n, int kchunk, void *out, double *partial, double *mean,
                        hipStream_t st);

}  // namespace moco
