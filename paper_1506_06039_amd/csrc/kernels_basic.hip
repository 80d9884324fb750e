// Stage kernels of the translation search on gfx950 (FP64 exact form).
//
//   coarse   : 2x2 box mean of every frame (the paper's "downsampled" frame,
//              sec. 2 first paragraph; the filter is read as a box mean)
//   sat_sq   : summed-area table of squared grid values; every overlap energy
//              sum of a^2 over D_{s,t} is one rectangle of it (sec. 2, the DP
//              recurrence for g is exactly this table)
//   corr_fp64: h_{s,t} = sum over D_{s,t} of a[i+s][j+t]*b[i][j] (sec. 2,
//              definition of h), direct FP64 sums
//   combine  : f = (A + B - 2h)/Area (sec. 2, energy split), argmin, gap
//   refine   : f at (2s*+u, 2t*+v) on the full grid, u,v in {-1,0,1}
//              (sec. 2, last paragraph), exact sums
//
// For uint16 input every grid value is a multiple of 1/4 below 2^16, so every
// square, product and sum here is an exact FP64 number while the grid's sum
// of squares stays below 2^48; f then rounds exactly once, at the division.
#include <math.h>

#include "moco_internal.h"

namespace moco {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Tie order of the argmin: lexicographic minimum of
// (f, max(|s|,|t|), |s|+|t|, s, t); a NaN f counts as +infinity.
struct Cand {
    double f;   // NaN already mapped to +inf
    int s, t;
    double second;  // best f among all other candidates seen (+inf if none)
};

__device__ inline double nan_to_inf(double f) { return isnan(f) ? INFINITY : f; }

__device__ inline bool precedes(double f1, int s1, int t1, double f2, int s2, int t2)
{
    if (f1 != f2) return f1 < f2;
    int r1 = max(abs(s1), abs(t1)), r2 = max(abs(s2), abs(t2));
    if (r1 != r2) return r1 < r2;
    int l1 = abs(s1) + abs(t1), l2 = abs(s2) + abs(t2);
    if (l1 != l2) return l1 < l2;
    if (s1 != s2) return s1 < s2;
    return t1 < t2;
}

__device__ inline void cand_add(Cand &c, double f, int s, int t)
{
    f = nan_to_inf(f);
    if (c.s == INT32_MIN) {
        c.f = f; c.s = s; c.t = t;
        return;
    }
    if (precedes(f, s, t, c.f, c.s, c.t)) {
        c.second = fmin(c.second, c.f);
        c.f = f; c.s = s; c.t = t;
    } else {
        c.second = fmin(c.second, f);
    }
}

__device__ inline Cand cand_merge(const Cand &x, const Cand &y)
{
    if (y.s == INT32_MIN) return x;
    if (x.s == INT32_MIN) return y;
    Cand r;
    bool ywins = precedes(y.f, y.s, y.t, x.f, x.s, x.t);
    const Cand &w = ywins ? y : x;
    const Cand &l = ywins ? x : y;
    r.f = w.f; r.s = w.s; r.t = w.t;
    r.second = fmin(fmin(x.second, y.second), l.f);
    return r;
}

// Block-wide merge of one candidate per thread; result valid in thread 0.
__device__ Cand block_argmin(Cand c)
{
    __shared__ double sf[kBlock], ss2[kBlock];
    __shared__ int si[kBlock], sj[kBlock];
    int tid = threadIdx.x;
    sf[tid] = c.f; ss2[tid] = c.second; si[tid] = c.s; sj[tid] = c.t;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) {
            Cand x{sf[tid], si[tid], sj[tid], ss2[tid]};
            Cand y{sf[tid + off], si[tid + off], sj[tid + off], ss2[tid + off]};
            Cand r = cand_merge(x, y);
            sf[tid] = r.f; ss2[tid] = r.second; si[tid] = r.s; sj[tid] = r.t;
        }
        __syncthreads();
    }
    Cand r{sf[0], si[0], sj[0], ss2[0]};
    return r;
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(const T *__restrict__ fr, int C, int m, int n,
                                                   int mg, int ng, int ds,
                                                   double *__restrict__ out)
{
    const size_t plane = (size_t)mg * ng;
    const size_t total = (size_t)C * plane;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        size_t f = idx / plane;
        int r = (int)(idx - f * plane);
        int i = r / ng, j = r - (r / ng) * ng;
        const T *a = fr + f * (size_t)m * n;
        double v;
        if (ds) {
            const T *p = a + (size_t)(2 * i) * n + 2 * j;
            double x00 = (double)p[0], x01 = (double)p[1];
            double x10 = (double)p[n], x11 = (double)p[n + 1];
            v = (((x00 + x01) + x10) + x11) / 4.0;
        } else {
            v = (double)a[(size_t)i * n + j];
        }
        out[idx] = v;
    }
}

// Summed-area table of squares: P is (mg+1) x (ng+1), P[0][*] = P[*][0] = 0,
// P[i+1][j+1] = sum of x^2 over rows <= i, cols <= j.  One block per frame.
__global__ __launch_bounds__(kBlock) void k_sat_sq(const double *__restrict__ coarse, int mg,
                                                   int ng, double *__restrict__ sat)
{
    const double *a = coarse + (size_t)blockIdx.x * mg * ng;
    double *P = sat + (size_t)blockIdx.x * (mg + 1) * (ng + 1);
    const int ld = ng + 1;
    for (int j = threadIdx.x; j <= ng; j += blockDim.x) P[j] = 0.0;
    for (int i = threadIdx.x; i < mg; i += blockDim.x) {
        P[(size_t)(i + 1) * ld] = 0.0;
        double acc = 0.0;
        const double *row = a + (size_t)i * ng;
        for (int j = 0; j < ng; ++j) {
            acc += row[j] * row[j];
            P[(size_t)(i + 1) * ld + j + 1] = acc;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < ng; j += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < mg; ++i) {
            size_t k = (size_t)(i + 1) * ld + j + 1;
            acc += P[k];
            P[k] = acc;
        }
    }
}

__device__ inline double rect(const double *P, int ld, int r0, int r1, int c0, int c1)
{
    // inclusive rows r0..r1, cols c0..c1 (empty if r1 < r0 or c1 < c0)
    if (r1 < r0 || c1 < c0) return 0.0;
    return P[(size_t)(r1 + 1) * ld + c1 + 1] - P[(size_t)r0 * ld + c1 + 1] -
           P[(size_t)(r1 + 1) * ld + c0] + P[(size_t)r0 * ld + c0];
}

// Template energies B(s,t): sum of b^2 over rows max(0,-s)..mg-1-max(0,s),
// cols max(0,-t)..ng-1-max(0,t).
__global__ __launch_bounds__(kBlock) void k_btab(const double *__restrict__ satb, int mg, int ng,
                                                 int w, double *__restrict__ btab)
{
    const int W = 2 * w - 1;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < W * W; k += gridDim.x * blockDim.x) {
        int s = k / W - (w - 1), t = k % W - (w - 1);
        btab[k] = rect(satb, ng + 1, max(0, -s), mg - 1 - max(0, s), max(0, -t),
                       ng - 1 - max(0, t));
    }
}

// ---------------------------------------------------------------------------
// Direct FP64 correlation.  Block (frame, s-block): lanes_per_s threads per
// shift row s, each owning TB consecutive t; a ring of s_per_blk zero-padded
// frame rows sits in LDS and advances by one row per template row i, so that
// row i+s is always resident.  Padded row x holds a[r][x-(w-1)].
constexpr int TB = 4;

__global__ __launch_bounds__(kBlock) void k_corr_fp64(const double *__restrict__ coarse,
                                                      const double *__restrict__ tc, int mg,
                                                      int ng, int w, int lanes_per_s,
                                                      int s_per_blk, int rowlen,
                                                      double *__restrict__ hout)
{
    extern __shared__ double lds[];
    double *ring = lds;                                   // s_per_blk x rowlen
    double *trow = lds + (size_t)s_per_blk * rowlen;      // ng
    const int W = 2 * w - 1;
    const int frame = blockIdx.y;
    const double *a = coarse + (size_t)frame * mg * ng;
    const int s0 = -(w - 1) + blockIdx.x * s_per_blk;
    const int s_hi = min(w - 1, s0 + s_per_blk - 1);
    const int tid = threadIdx.x;
    const int sl = tid / lanes_per_s, tl = tid - (tid / lanes_per_s) * lanes_per_s;
    const int s = s0 + sl;
    const bool active = sl < s_per_blk && s <= w - 1;
    const int tt0 = tl * TB;
    // template rows i that overlap some frame row i+s with s in [s0, s_hi]
    const int i_lo = max(0, -s_hi), i_hi = min(mg, mg - s0);

    auto load_row = [&](int r, int slot) {
        double *dst = ring + (size_t)slot * rowlen;
        bool in = r >= 0 && r < mg;
        for (int x = tid; x < rowlen; x += blockDim.x) {
            int c = x - (w - 1);
            dst[x] = (in && c >= 0 && c < ng) ? a[(size_t)r * ng + c] : 0.0;
        }
    };
    // ring slot of frame row r: (r - (i_lo + s0)) mod s_per_blk, non-negative
    const int rbase = i_lo + s0;
    for (int q = 0; q < s_per_blk; ++q) load_row(rbase + q, q);

    double acc[TB];
#pragma unroll
    for (int k = 0; k < TB; ++k) acc[k] = 0.0;

    for (int i = i_lo; i < i_hi; ++i) {
        const double *trow_g = tc + (size_t)i * ng;
        for (int x = tid; x < ng; x += blockDim.x) trow[x] = trow_g[x];
        __syncthreads();
        if (active) {
            int slot = (i + s - rbase) % s_per_blk;
            const double *row = ring + (size_t)slot * rowlen + tt0;
            double win[TB];
#pragma unroll
            for (int k = 0; k < TB; ++k) win[k] = row[k];
            for (int j = 0; j < ng; ++j) {
                double bj = trow[j];
#pragma unroll
                for (int k = 0; k < TB; ++k) acc[k] = fma(win[k], bj, acc[k]);
#pragma unroll
                for (int k = 0; k < TB - 1; ++k) win[k] = win[k + 1];
                win[TB - 1] = row[j + TB];
            }
        }
        __syncthreads();
        // row i+s0 leaves the window; row i+s0+s_per_blk enters in its slot
        int r_out = i + s0;
        load_row(r_out + s_per_blk, (r_out - rbase) % s_per_blk);
    }
    if (active) {
        double *h = hout + (size_t)frame * W * W + (size_t)(s + w - 1) * W;
#pragma unroll
        for (int k = 0; k < TB; ++k)
            if (tt0 + k < W) h[tt0 + k] = acc[k];
    }
}

// ---------------------------------------------------------------------------
// Combine, normalise, argmin.  One block per frame.
__global__ __launch_bounds__(kBlock) void k_combine(const double *__restrict__ sat,
                                                    const double *__restrict__ btab,
                                                    const double *__restrict__ hbuf, int mg,
                                                    int ng, int w, int ds,
                                                    double *__restrict__ fsurf,
                                                    double *__restrict__ fmin_out,
                                                    int32_t *__restrict__ coarse_st,
                                                    int32_t *__restrict__ shifts,
                                                    double *__restrict__ gaps,
                                                    double *__restrict__ frefine)
{
    const int W = 2 * w - 1;
    const int frame = blockIdx.x;
    const double *P = sat + (size_t)frame * (mg + 1) * (ng + 1);
    const double *h = hbuf + (size_t)frame * W * W;
    Cand c{INFINITY, INT32_MIN, 0, INFINITY};
    for (int k = threadIdx.x; k < W * W; k += blockDim.x) {
        int s = k / W - (w - 1), t = k % W - (w - 1);
        double A = rect(P, ng + 1, max(0, s), mg - 1 + min(0, s), max(0, t), ng - 1 + min(0, t));
        double area = (double)(mg - abs(s)) * (double)(ng - abs(t));
        double f = (A + btab[k] - 2.0 * h[k]) / area;
        if (fsurf) fsurf[(size_t)frame * W * W + k] = f;
        cand_add(c, f, s, t);
    }
    Cand r = block_argmin(c);
    if (threadIdx.x == 0) {
        if (fmin_out) fmin_out[frame] = r.f;
        coarse_st[2 * frame] = r.s;
        coarse_st[2 * frame + 1] = r.t;
        if (gaps) gaps[2 * frame] = r.second - r.f;
        if (!ds) {
            shifts[2 * frame] = r.s;
            shifts[2 * frame + 1] = r.t;
            if (gaps) gaps[2 * frame + 1] = INFINITY;
        }
    }
    if (!ds && frefine && threadIdx.x < 9) frefine[(size_t)frame * 9 + threadIdx.x] = NAN;
}

// ---------------------------------------------------------------------------
// Full-resolution x2 step: f at (2s*+u, 2t*+v), u,v in {-1,0,1}.  One block
// per frame; every thread keeps nine sums over a strided slice of template
// pixels.  uint16: exact integer sums (squared differences < 2^32, totals far
// below 2^63); float32: FP64 sums.
template <typename T>
struct RefAcc;
template <>
struct RefAcc<uint16_t> {
    using type = unsigned long long;
    __device__ static type term(uint16_t x, uint16_t y)
    {
        int d = (int)x - (int)y;
        return (unsigned long long)((long long)d * d);
    }
};
template <>
struct RefAcc<float> {
    using type = double;
    __device__ static type term(float x, float y)
    {
        double d = (double)x - (double)y;
        return d * d;
    }
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_refine(const T *__restrict__ frames,
                                                   const T *__restrict__ tmpl, int m, int n,
                                                   const int32_t *__restrict__ coarse_st,
                                                   int32_t *__restrict__ shifts,
                                                   double *__restrict__ frefine,
                                                   double *__restrict__ gaps)
{
    using Acc = typename RefAcc<T>::type;
    const int frame = blockIdx.x;
    const T *a = frames + (size_t)frame * m * n;
    const int cs = coarse_st[2 * frame], ct = coarse_st[2 * frame + 1];
    Acc acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0;
    const int total = m * n;
    for (int p = threadIdx.x; p < total; p += blockDim.x) {
        int i = p / n, j = p - (p / n) * n;
        T bv = tmpl[p];
#pragma unroll
        for (int u = -1; u <= 1; ++u) {
            int r = i + 2 * cs + u;
            bool rin = r >= 0 && r < m;
#pragma unroll
            for (int v = -1; v <= 1; ++v) {
                int c = j + 2 * ct + v;
                if (rin && c >= 0 && c < n)
                    acc[(u + 1) * 3 + (v + 1)] += RefAcc<T>::term(a[(size_t)r * n + c], bv);
            }
        }
    }
    __shared__ Acc red[9][kBlock];
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
#pragma unroll
            for (int q = 0; q < 9; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Cand c{INFINITY, INT32_MIN, 0, INFINITY};
        for (int q = 0; q < 9; ++q) {
            int u = q / 3 - 1, v = q % 3 - 1;
            int s = 2 * cs + u, t = 2 * ct + v;
            double area = (double)(m - abs(s)) * (double)(n - abs(t));
            double f = (double)red[q][0] / area;
            if (frefine) frefine[(size_t)frame * 9 + q] = f;
            cand_add(c, f, s, t);
        }
        shifts[2 * frame] = c.s;
        shifts[2 * frame + 1] = c.t;
        if (gaps) gaps[2 * frame + 1] = c.second - c.f;
    }
}

// Banded x2 step: block (band of template rows, frame).  The frame rows the
// band touches, i0+2s*-1 .. i1+2s*, are staged in LDS; every thread walks
// template pixels of the band and adds the nine squared differences with FP64
// FMAs (exact for uint16: every square is below 2^32 and every partial sum
// far below 2^53).  Partial sums go to [frame][band][9]; k_refine_finish adds
// them in band order and takes the argmin.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_refine_band(const T *__restrict__ frames,
                                                        const T *__restrict__ tmpl, int m, int n,
                                                        int br, const int32_t *__restrict__ coarse_st,
                                                        double *__restrict__ partial)
{
    extern __shared__ __attribute__((aligned(16))) char lds_raw[];
    T *rows = (T *)lds_raw;  // (br + 2) x n
    const int frame = blockIdx.y, band = blockIdx.x, nband = gridDim.x;
    const int i0 = band * br, i1 = min(m, i0 + br);
    const int cs = coarse_st[2 * frame], ct = coarse_st[2 * frame + 1];
    const int S0 = 2 * cs, T0 = 2 * ct;
    const int rbase = i0 + S0 - 1;
    const int nrows = i1 - i0 + 2;
    const T *a = frames + (size_t)frame * m * n;
    for (int idx = threadIdx.x; idx < nrows * n; idx += blockDim.x) {
        int rr = idx / n, c = idx - (idx / n) * n;
        int r = rbase + rr;
        rows[idx] = (r >= 0 && r < m) ? a[(size_t)r * n + c] : (T)0;
    }
    __syncthreads();
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    const int total = (i1 - i0) * n;
    for (int p = threadIdx.x; p < total; p += blockDim.x) {
        int li = p / n, j = p - (p / n) * n;
        int i = i0 + li;
        double bv = (double)tmpl[(size_t)i * n + j];
#pragma unroll
        for (int u = -1; u <= 1; ++u) {
            int r = i + S0 + u;
            if (r < 0 || r >= m) continue;
            const T *rowp = rows + (size_t)(li + u + 1) * n;
#pragma unroll
            for (int v = -1; v <= 1; ++v) {
                int c = j + T0 + v;
                if (c >= 0 && c < n) {
                    double d = (double)rowp[c] - bv;
                    acc[(u + 1) * 3 + (v + 1)] = fma(d, d, acc[(u + 1) * 3 + (v + 1)]);
                }
            }
        }
    }
    // block reduction of the nine sums (fixed tree order)
    __shared__ double red[9][kBlock];
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
#pragma unroll
            for (int q = 0; q < 9; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9)
        partial[((size_t)frame * nband + band) * 9 + threadIdx.x] = red[threadIdx.x][0];
}

// uint16 x2 step in integers.  Block (band of kRefBand template rows, frame).
// The frame rows the band touches, i0+2s*-1 .. i1+2s*, are copied into LDS with
// 16-byte loads (one contiguous span of full rows); a thread then owns four
// template columns j0..j0+3 and a run of the band's rows, reading for each row
// the six frame values at columns j0+2t*-1..j0+2t*+4.
//
// pmax (may be null): per frame, an upper bound of its pixel values; tmax the
// template's (-1: none).  With both, |d| <= M = max(pmax, tmax) and the nine
// sums run in 32 bits (24-bit multiply-adds) while flush*4*M^2 < 2^32, then add
// into 64-bit sums, so no 32-bit sum can wrap.  Without a bound every term goes
// straight into 64 bits.  Partial sums go to [frame][band][9] as exact FP64
// integers (far below 2^53).
constexpr int kRefBand = 32;

__global__ __launch_bounds__(kBlock) void k_refine_u16(const uint16_t *__restrict__ frames,
                                                       const uint16_t *__restrict__ tmpl, int m,
                                                       int n, const int32_t *__restrict__ coarse_st,
                                                       const int32_t *__restrict__ pmax, int tmax,
                                                       double *__restrict__ partial)
{
    extern __shared__ __attribute__((aligned(16))) char lds_raw[];
    uint16_t *srow = (uint16_t *)lds_raw;  // 8 guard elements, (kRefBand + 2) rows of n, 8 guard
    const int frame = blockIdx.y, band = blockIdx.x, nband = gridDim.x;
    const int i0 = band * kRefBand, i1 = min(m, i0 + kRefBand), nb = i1 - i0;
    const int S0 = 2 * coarse_st[2 * frame], T0 = 2 * coarse_st[2 * frame + 1];
    const uint16_t *a = frames + (size_t)frame * m * n;
    const int r0 = i0 + S0 - 1;  // frame row held in LDS row 0
    {
        const int ra = max(r0, 0), rb = min(r0 + nb + 2, m);
        if (rb > ra) {
            const uint16_t *src = a + (size_t)ra * n;
            uint16_t *dst = srow + 8 + (size_t)(ra - r0) * n;
            const size_t cnt = (size_t)(rb - ra) * n;
            const bool v16 = ((n & 7) == 0) && ((((uintptr_t)src) & 15) == 0);
            if (v16) {
                const uint4 *s4 = (const uint4 *)src;
                uint4 *d4 = (uint4 *)dst;  // 16 + 2*(ra-r0)*n bytes into the buffer: aligned
                for (size_t k = threadIdx.x; k < cnt / 8; k += blockDim.x) d4[k] = s4[k];
            } else {
                for (size_t k = threadIdx.x; k < cnt; k += blockDim.x) dst[k] = src[k];
            }
        }
    }
    __syncthreads();
    unsigned long long acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0;
    int flush = 0;  // rows between flushes of the 32-bit sums (0: 64-bit sums only)
    if (pmax && tmax >= 0) {
        const long long M = max((long long)pmax[frame], (long long)tmax);
        const long long lim = M > 0 ? 0xffffffffLL / (4 * M * M) : (1LL << 30);
        flush = (int)min(lim, (long long)(1 << 30));
    }
    const bool even = (n & 1) == 0;
    const int ncg = (n + 3) / 4;
    const int ncgs = ncg < kBlock ? ncg : kBlock;
    const int rg_count = kBlock / ncgs;
    const int rg = threadIdx.x / ncgs;
    if (rg < rg_count) {
        const int rows_per = (nb + rg_count - 1) / rg_count;
        const int la = rg * rows_per, lb = min(nb, la + rows_per);
        for (int cg = threadIdx.x % ncgs; cg < ncg; cg += ncgs) {
            const int j0 = 4 * cg;
            const int c0 = j0 + T0 - 1;  // first frame column of the window
            int kval = 0, qval = 0;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (c0 + k >= 0 && c0 + k < n) kval |= 1 << k;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j0 + q < n) qval |= 1 << q;
            const bool interior = kval == 63 && qval == 15;
            const bool tvec = ((n & 3) == 0) && j0 + 3 < n;
            unsigned acc32[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) acc32[q] = 0;
            int since = 0;
            for (int li = la; li < lb; ++li) {
                const int i = i0 + li;
                int b[4];
                if (tvec) {
                    uint2 t2 = *(const uint2 *)(tmpl + (size_t)i * n + j0);
                    b[0] = (int)(t2.x & 0xffff);
                    b[1] = (int)(t2.x >> 16);
                    b[2] = (int)(t2.y & 0xffff);
                    b[3] = (int)(t2.y >> 16);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        b[q] = (qval >> q & 1) ? (int)tmpl[(size_t)i * n + j0 + q] : 0;
                }
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const int r = i + S0 + u - 1;
                    if (r < 0 || r >= m) continue;
                    // LDS row li+u holds frame row r; the window is its columns c0 .. c0+5
                    const uint16_t *row = srow + 8 + (size_t)(li + u) * n + (c0 - 1);
                    int f[6];
                    if (interior && even) {
                        // c0-1 .. c0+6 lie within this row's neighbourhood of the buffer
                        // (c0 >= 0, c0+5 < n, 8 guard elements at either end); c0-1 is even
                        const uint32_t *p = (const uint32_t *)row;
                        uint32_t q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
                        f[0] = (int)(q0 >> 16);
                        f[1] = (int)(q1 & 0xffff);
                        f[2] = (int)(q1 >> 16);
                        f[3] = (int)(q2 & 0xffff);
                        f[4] = (int)(q2 >> 16);
                        f[5] = (int)(q3 & 0xffff);
                    } else {
                        // edge of the image: read only the columns that exist
#pragma unroll
                        for (int k = 0; k < 6; ++k) f[k] = (kval >> k & 1) ? (int)row[k + 1] : 0;
                    }
                    if (flush > 0) {
#pragma unroll
                        for (int v = 0; v < 3; ++v)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                int d = f[q + v] - b[q];
                                if (!interior && !((kval >> (q + v) & 1) && (qval >> q & 1))) d = 0;
                                acc32[u * 3 + v] += (unsigned)__mul24(d, d);
                            }
                    } else {
#pragma unroll
                        for (int v = 0; v < 3; ++v)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                int d = f[q + v] - b[q];
                                if (!interior && !((kval >> (q + v) & 1) && (qval >> q & 1))) d = 0;
                                acc[u * 3 + v] += (unsigned)__mul24(d, d);
                            }
                    }
                }
                if (flush > 0 && ++since >= flush) {
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        acc[q] += acc32[q];
                        acc32[q] = 0;
                    }
                    since = 0;
                }
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[q] += acc32[q];
        }
    }
    // wave sums, then the four waves in order
    __shared__ unsigned long long red[kBlock / 64][9];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        unsigned long long v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
            lo = __shfl_xor(lo, off);
            hi = __shfl_xor(hi, off);
            v += ((unsigned long long)hi << 32) | lo;
        }
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[w][threadIdx.x];
        partial[((size_t)frame * nband + band) * 9 + threadIdx.x] = (double)t;
    }
}

__global__ __launch_bounds__(kBlock) void k_refine_finish(const double *__restrict__ partial,
                                                          int C, int nband, int m, int n,
                                                          const int32_t *__restrict__ coarse_st,
                                                          int32_t *__restrict__ shifts,
                                                          double *__restrict__ frefine,
                                                          double *__restrict__ gaps)
{
    const int frame = blockIdx.x * blockDim.x + threadIdx.x;
    if (frame >= C) return;
    const int cs = coarse_st[2 * frame], ct = coarse_st[2 * frame + 1];
    Cand c{INFINITY, INT32_MIN, 0, INFINITY};
    for (int q = 0; q < 9; ++q) {
        double e = 0.0;
        for (int b = 0; b < nband; ++b) e += partial[((size_t)frame * nband + b) * 9 + q];
        int u = q / 3 - 1, v = q % 3 - 1;
        int s = 2 * cs + u, t = 2 * ct + v;
        double area = (double)(m - abs(s)) * (double)(n - abs(t));
        double f = e / area;
        if (frefine) frefine[(size_t)frame * 9 + q] = f;
        cand_add(c, f, s, t);
    }
    shifts[2 * frame] = c.s;
    shifts[2 * frame + 1] = c.t;
    if (gaps) gaps[2 * frame + 1] = c.second - c.f;
}

int grid_for(size_t total)
{
    size_t g = (total + kBlock - 1) / kBlock;
    if (g > 65535 * 4) g = 65535 * 4;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_coarse(const void *frames, moco_dtype dt, int C, const Geom &g, double *coarse,
                         hipStream_t st)
{
    clear_stale_error();
    size_t total = (size_t)C * g.mg * g.ng;
    if (total == 0) return hipSuccess;
    if (dt == MOCO_U16)
        k_coarse<uint16_t><<<grid_for(total), kBlock, 0, st>>>(
            (const uint16_t *)frames, C, g.m, g.n, g.mg, g.ng, g.ds, coarse);
    else
        k_coarse<float><<<grid_for(total), kBlock, 0, st>>>((const float *)frames, C, g.m, g.n,
                                                            g.mg, g.ng, g.ds, coarse);
    return hipGetLastError();
}

hipError_t launch_sat_sq(const double *coarse, int C, const Geom &g, double *sat, hipStream_t st)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    k_sat_sq<<<C, kBlock, 0, st>>>(coarse, g.mg, g.ng, sat);
    return hipGetLastError();
}

hipError_t launch_btab(const double *sat_b, const Geom &g, double *btab, hipStream_t st)
{
    clear_stale_error();
    k_btab<<<grid_for((size_t)g.W * g.W), kBlock, 0, st>>>(sat_b, g.mg, g.ng, g.w, btab);
    return hipGetLastError();
}

hipError_t launch_corr_fp64(const double *coarse, const double *tcoarse, int C, const Geom &g,
                            double *h, hipStream_t st)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    int lanes_per_s = (g.W + TB - 1) / TB;
    int s_per_blk = kBlock / lanes_per_s;
    if (s_per_blk > g.W) s_per_blk = g.W;
    if (s_per_blk < 1) return hipErrorInvalidValue;  // W > 4*kBlock is rejected by validation
    int rowlen = g.ng + lanes_per_s * TB + TB;
    size_t lds = ((size_t)s_per_blk * rowlen + g.ng) * sizeof(double);
    while (lds > 64 * 1024 && s_per_blk > 1) {
        --s_per_blk;
        lds = ((size_t)s_per_blk * rowlen + g.ng) * sizeof(double);
    }
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    dim3 grid((g.W + s_per_blk - 1) / s_per_blk, C);
    k_corr_fp64<<<grid, kBlock, lds, st>>>(coarse, tcoarse, g.mg, g.ng, g.w, lanes_per_s, s_per_blk,
                                          rowlen, h);
    return hipGetLastError();
}

hipError_t launch_combine(const double *sat, const double *btab, const double *h, int C,
                          const Geom &g, double *fsurf, double *fmin, int32_t *coarse_st,
                          int32_t *shifts, double *gaps, double *frefine, hipStream_t st)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    k_combine<<<C, kBlock, 0, st>>>(sat, btab, h, g.mg, g.ng, g.w, g.ds, fsurf, fmin, coarse_st,
                                    shifts, gaps, frefine);
    return hipGetLastError();
}

hipError_t launch_refine(const void *frames, const void *traw, int C, const Geom &g,
                         const int32_t *coarse_st, int32_t *shifts, double *frefine,
                         double *gaps, double *partial, hipStream_t st, const int32_t *pmax,
                         int tmax)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    const size_t esz = g.dtype == MOCO_U16 ? 2 : 4;
    int br = refine_band_rows(g);
    if (g.dtype == MOCO_U16 && refine_u16_banded(g)) {
        const int nband = (g.m + kRefBand - 1) / kRefBand;
        const size_t lds = ((size_t)(kRefBand + 2) * g.n + 16) * sizeof(uint16_t);
        dim3 grid(nband, C);
        k_refine_u16<<<grid, kBlock, lds, st>>>((const uint16_t *)frames, (const uint16_t *)traw,
                                               g.m, g.n, coarse_st, pmax, tmax, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_refine_finish<<<(C + kBlock - 1) / kBlock, kBlock, 0, st>>>(partial, C, nband, g.m, g.n,
                                                                      coarse_st, shifts, frefine,
                                                                      gaps);
        return hipGetLastError();
    }
    if (br > 0) {
        const int nband = (g.m + br - 1) / br;
        const size_t lds = (size_t)(br + 2) * g.n * esz;
        dim3 grid(nband, C);
        if (g.dtype == MOCO_U16)
            k_refine_band<uint16_t><<<grid, kBlock, lds, st>>>((const uint16_t *)frames,
                                                               (const uint16_t *)traw, g.m, g.n, br,
                                                               coarse_st, partial);
        else
            k_refine_band<float><<<grid, kBlock, lds, st>>>((const float *)frames,
                                                            (const float *)traw, g.m, g.n, br,
                                                            coarse_st, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_refine_finish<<<(C + kBlock - 1) / kBlock, kBlock, 0, st>>>(partial, C, nband, g.m, g.n,
                                                                      coarse_st, shifts, frefine,
                                                                      gaps);
        return hipGetLastError();
    }
    if (g.dtype == MOCO_U16)
        k_refine<uint16_t><<<C, kBlock, 0, st>>>((const uint16_t *)frames, (const uint16_t *)traw,
                                                 g.m, g.n, coarse_st, shifts, frefine, gaps);
    else
        k_refine<float><<<C, kBlock, 0, st>>>((const float *)frames, (const float *)traw, g.m,
                                              g.n, coarse_st, shifts, frefine, gaps);
    return hipGetLastError();
}

int refine_band_rows(const Geom &g)
{
    // rows of LDS staging: uint16 rows carry a few halo columns
    const size_t esz = g.dtype == MOCO_U16 ? 2 : 4;
    const size_t row = (size_t)(g.n + 16) * esz;
    if (3 * row > 40 * 1024) return 0;  // very wide frames: the unstaged kernel
    int br = (int)(40 * 1024 / row) - 2;
    const int cap = g.dtype == MOCO_U16 ? 32 : 16;
    return br > cap ? cap : br;
}

bool refine_u16_banded(const Geom &g)
{
    return (size_t)(kRefBand + 2) * g.n * sizeof(uint16_t) + 32 <= 48 * 1024;
}

size_t refine_partial_bytes(const Geom &g)
{
    if (g.dtype == MOCO_U16 && refine_u16_banded(g))
        return (size_t)((g.m + kRefBand - 1) / kRefBand) * 9 * sizeof(double);
    int br = refine_band_rows(g);
    if (br <= 0) return 0;
    return (size_t)((g.m + br - 1) / br) * 9 * sizeof(double);
}

}  // namespace moco
