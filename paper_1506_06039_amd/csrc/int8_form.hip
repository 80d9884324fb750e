// Exact integer form of the search for uint16 data on the gfx950 matrix cores.
//
// Grid values are integers X (2x2 box sums when downsampling, raw counts
// otherwise).  The three sums of the energy split (sec. 2: Area*f = sum a^2 +
// sum b^2 - 2 sum ab) are computed exactly:
//
//   * sum of squares over D_{s,t} (sec. 2, the recurrence for g): total energy
//     minus excluded border rows and columns plus the excluded corner, all in
//     int64, from row/column energies and corner prefix tables built while the
//     frame streams in (k_prep_u16);
//   * the correlation h_{s,t} = sum over D of a[i+s][j+t]*b[i][j] (sec. 2,
//     definition of h) on int8 MFMA: each value is split into balanced digits,
//     base 128 (X = d0 + 128*d1 (+ 16384*d2), |d| <= 64) when the template's
//     values allow, with three products per term (d0 e0, d1 e1 and
//     (d0 + d1)(e0 + e1), Karatsuba), else base 256 (d in [-128,127]) with
//     four; every digit product is exact in the int32 accumulators and h is
//     recombined in int64 (k_corr_int8).
//
// The correlation is a band contraction: for template row i and frame column
// k, H[s][t] += A[i+s][k] * B[i][k-t].  M = s (frame rows i+s, read from a
// per-wave ring of frame rows in LDS), N = t (the template row i laid out as a
// Toeplitz operand, read from LDS at a per-lane byte offset from one of eight
// byte-phase copies, so that every read is 8-byte aligned), K = k (32 columns
// per MFMA).
#include <math.h>

#include <algorithm>

#include "moco_internal.h"

namespace moco {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;
constexpr int kWaves = 4;
constexpr int kStrip = 128;          // frame columns per strip
constexpr int kPhases = 8;           // byte-phase copies of each template row
constexpr int kMaxTrow = 1024;       // template row bytes held per phase and digit
constexpr int kMaxTrowSum = kInt8SumMaxTrow;  // the same with a third (digit-sum) template plane

__device__ inline long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        int lo = (int)(unsigned)(v & 0xffffffffLL);
        int hi = (int)(v >> 32);
        lo = __shfl_xor(lo, off);
        hi = __shfl_xor(hi, off);
        v += ((long long)hi << 32) | (unsigned)lo;
    }
    return v;
}

// balanced digit of base 2^b: returns d in [-2^(b-1), 2^(b-1)) with x - d
// divisible by 2^b
__device__ inline int bdigit(int x, int b)
{
    const int half = 1 << (b - 1);
    return ((x + half) & ((1 << b) - 1)) - half;
}

// byte-wise sum of four packed int8 (mod 256 per byte, no carry between bytes)
__device__ inline unsigned byte_add(unsigned x, unsigned y)
{
    return ((x & 0x7f7f7f7fu) + (y & 0x7f7f7f7fu)) ^ ((x ^ y) & 0x80808080u);
}

// ---------------------------------------------------------------------------
// k_prep_u16: one block per frame (a few frames: one per band of rows, and
// k_prep_finish per frame).
//   limbs  [frame][3][mg][npad] int8 balanced digits of base 2^dbits (128 or
//          256), plane 2 written only when needed
//   nlimb  [frame]               2, or 3 when some X needs a third digit
//          (X > 8127 in base 128, X > 32639 in base 256)
//   atab   [frame][W][W] int64   sum of X^2 over D_{s,t} (frame side)
//   edge   [frame][2][2][w-1][w] int64 scratch: for the first (top) and last
//          (bottom) w-1 rows, prefix sums of X^2 over the first q columns (LP)
//          and over the last q columns (RS), q = 0..w-1
template <bool DS>
__device__ inline int grid_value(const uint16_t *a, int n, int i, int j)
{
    if (DS) {
        const uint16_t *p = a + (size_t)(2 * i) * n + 2 * j;
        return (int)p[0] + (int)p[1] + (int)p[n] + (int)p[n + 1];
    }
    return (int)a[(size_t)i * n + j];
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Four consecutive grid values j0..j0+3 of grid row i (zero beyond ng).  vec:
// 0 scalar reads; 1 the raw rows read as 8-byte vectors (rows 8-byte
// aligned: n a multiple of 4); 2 (box sums only) as 16-byte vectors (n a
// multiple of 8).
template <bool DS>
__device__ inline void grid_values4(const uint16_t *a, int n, int ng, int i, int j0, int vec,
                                    int (&X)[4])
{
    if (vec && j0 + 3 < ng) {
        if (DS) {
            // streamed once: non-temporal loads keep the frames out of the caches
            const uint16_t *p0 = a + (size_t)(2 * i) * n + 2 * j0, *p1 = p0 + n;
            unsigned u0[4], u1[4];
            if (vec == 2) {
                const u32x4 r0 = __builtin_nontemporal_load((const u32x4 *)p0);
                const u32x4 r1 = __builtin_nontemporal_load((const u32x4 *)p1);
                u0[0] = r0.x, u0[1] = r0.y, u0[2] = r0.z, u0[3] = r0.w;
                u1[0] = r1.x, u1[1] = r1.y, u1[2] = r1.z, u1[3] = r1.w;
            } else {
                const u32x2 r0a = __builtin_nontemporal_load((const u32x2 *)p0);
                const u32x2 r0b = __builtin_nontemporal_load((const u32x2 *)p0 + 1);
                const u32x2 r1a = __builtin_nontemporal_load((const u32x2 *)p1);
                const u32x2 r1b = __builtin_nontemporal_load((const u32x2 *)p1 + 1);
                u0[0] = r0a.x, u0[1] = r0a.y, u0[2] = r0b.x, u0[3] = r0b.y;
                u1[0] = r1a.x, u1[1] = r1a.y, u1[2] = r1b.x, u1[3] = r1b.y;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                X[q] = (int)(u0[q] & 0xffff) + (int)(u0[q] >> 16) + (int)(u1[q] & 0xffff) +
                       (int)(u1[q] >> 16);
        } else {
            const uint2 r0 = *(const uint2 *)(a + (size_t)i * n + j0);
            X[0] = (int)(r0.x & 0xffff);
            X[1] = (int)(r0.x >> 16);
            X[2] = (int)(r0.y & 0xffff);
            X[3] = (int)(r0.y >> 16);
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) X[q] = (j0 + q < ng) ? grid_value<DS>(a, n, i, j0 + q) : 0;
}

//
// With GRID, the same pass serves the FP64 forms instead: no digit planes;
// the grid values are written as FP64 box means (raw values without
// downsampling) to grid [frame][mg][ng], and the energy table as FP64 in
// grid units to atab_d (the integer sums divided by 16 when downsampling: an
// exact scaling, the same values a FP64 pass over the grid gives), of the
// values less xc (in box-sum units; the grid written is not centred).
//
// With BAND, a few frames are split over bands of band_rows grid rows, one
// block per (band, frame) (grid.x bands, grid.y frames): each band writes its
// digit planes (or grid rows) and the edge prefix rows it owns, and leaves
// in bandp the sums the energy table needs from it; k_prep_finish then forms
// the table per frame.  bandp [frame][prep_band_longs]: the 2(w-1) border
// row energies (top rows 0..w-2, then bottom rows mg-1 down), then per band
// {energies of the first w-1 and of the last w-1 columns (from the right),
// total energy, third-digit flag, largest grid value}.

// Energies of the border columns, rows and the whole grid -> the energy
// table, the third digit plane (when needed) and the per-frame flags.  On
// entry cL[s], cR[s], rT[s], rB[s] (s < w-1) hold the energies of column s,
// column ng-1-s, row s and row mg-1-s; they are turned into prefix sums over
// s = 0..w-1 here.  Every thread of the block (256) calls it.
//
// KU: corner-sum loads each thread issues before using them (a larger KU
// takes more registers and fewer round trips to memory).
template <bool DS, bool GRID, int KU>
__device__ inline void prep_tables(const uint16_t *a, int m, int n, int mg, int ng, int w,
                                   int npad, int dbits, int frame, long long *cL, long long *cR,
                                   long long *rT, long long *rB, long long Etot, int need3,
                                   int xmax, const long long *E, int8_t *L0, int32_t *nlimb,
                                   int32_t *vmax, long long *atab, double *atab_d)
{
    const int W = 2 * w - 1, we = w - 1;
    auto eidx = [&](int tb, int lr, int e, int q) { return ((size_t)(tb * 2 + lr) * we + e) * w + q; };
    // prefix sums: rows excluded from the top / bottom, columns from left / right
    if (threadIdx.x % 64 == 0) {
        long long *v = threadIdx.x == 0 ? cL : threadIdx.x == 64 ? cR : threadIdx.x == 128 ? rT : rB;
        long long acc = 0;
        for (int s = 0; s < w; ++s) {
            const long long x = s < we ? v[s] : 0;
            v[s] = acc;
            acc += x;
        }
    }
    __syncthreads();
    auto put = [&](size_t k, long long v) {
        if (GRID)
            atab_d[(size_t)frame * W * W + k] = DS ? 0.0625 * (double)v : (double)v;
        else
            atab[(size_t)frame * W * W + k] = v;
    };
    // one thread per (column shift t, sign of the row shift); the corner sums
    // run down the rows, their loads unrolled so that several are in flight
    for (int idx = threadIdx.x; idx < 2 * W; idx += blockDim.x) {
        const int tt = idx % W, side = idx / W;
        const int t = tt - we, at = t < 0 ? -t : t;
        const int lr = t > 0 ? 0 : 1;
        const long long colex = t > 0 ? cL[at] : (t < 0 ? cR[at] : 0);
        const long long base = Etot - colex;
        if (side == 0) put((size_t)we * W + tt, base);
        const long long *rx = side ? rB : rT;   // rows excluded at the top (+s) or bottom (-s)
        long long c = 0;
        for (int s0 = 1; s0 < w; s0 += KU) {
            long long ev[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u)
                ev[u] = (t != 0 && s0 + u < w) ? E[eidx(side, lr, s0 + u - 1, at)] : 0;
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int s = s0 + u;
                if (s < w) {
                    c += ev[u];
                    put((size_t)(side ? we - s : we + s) * W + tt, base - rx[s] + c);
                }
            }
        }
    }
    // third digit plane, only for frames that need it
    if (!GRID && need3) {
        const size_t plane = (size_t)mg * npad;
        int8_t *L2 = L0 + 2 * plane;
        const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
        for (int i = wave; i < mg; i += nw)
            for (int j0 = 4 * lane; j0 < npad; j0 += 256) {
                int d2p = 0;
                for (int q = 0; q < 4; ++q) {
                    int j = j0 + q;
                    int X = (j < ng) ? grid_value<DS>(a, n, i, j) : 0;
                    int d0 = bdigit(X, dbits);
                    int x1 = (X - d0) >> dbits;
                    int d1 = bdigit(x1, dbits);
                    int d2 = (x1 - d1) >> dbits;
                    d2p |= (d2 & 255) << (8 * q);
                }
                *(int *)(L2 + (size_t)i * npad + j0) = d2p;
            }
    }
    if (threadIdx.x == 0) {
        if (!GRID) nlimb[frame] = need3 ? 3 : 2;
        // every pixel is a term of some grid value unless a side is odd when downsampling
        const bool covers = !DS || ((m % 2) == 0 && (n % 2) == 0);
        vmax[frame] = covers ? xmax : INT32_MAX;
    }
}

template <bool DS, int kMaxCol4, int NW, bool GRID, bool BAND>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_prep_u16(const uint16_t *__restrict__ raw, int m,
                                                     int n, int mg, int ng, int w, int npad,
                                                     int dbits,
                                                     int8_t *__restrict__ limbs,
                                                     int32_t *__restrict__ nlimb,
                                                     int32_t *__restrict__ vmax,
                                                     long long *__restrict__ atab,
                                                     long long *__restrict__ edge,
                                                     double *__restrict__ grid,
                                                     double *__restrict__ atab_d,
                                                     const int32_t *__restrict__ only,
                                                     int xc, int band_rows,
                                                     long long *__restrict__ bandp,
                                                     int32_t *__restrict__ hz)
{
    const int frame = BAND ? blockIdx.y : blockIdx.x;
    // GRID with `only`: frames whose only[f] is 0 are skipped (the whole block)
    if (GRID && only && !only[frame]) return;
    // dynamic LDS: colE[npad] | rowbuf[NW][2][we1] | rT[w] | rB[w] | cL[w] | cR[w] | etot | need3
    extern __shared__ long long lds_prep[];
    const int we1 = w > 1 ? w - 1 : 1;
    long long *colE = lds_prep;
    long long *rowbuf_base = colE + npad;   // X^2 of the first / last w-1 columns of an edge row
    long long *rT = rowbuf_base + (size_t)NW * 2 * we1;
    long long *rB = rT + w;
    long long *cL = rB + w;
    long long *cR = cL + w;
    long long &etot = cR[w];
    int &need3 = *(int *)(cR + w + 1);
    int &xmax = *((int *)(cR + w + 1) + 1);
    auto rowbuf = [&](int wv, int side) { return rowbuf_base + ((size_t)wv * 2 + side) * we1; };

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const uint16_t *a = raw + (size_t)frame * m * n;
    // vector raw reads need aligned rows: 16 bytes (box sums) or 8 bytes
    const bool al8 = (n % 4) == 0 && (((uintptr_t)a) & 7) == 0;
    const int vec = DS && al8 && (n % 8) == 0 && (((uintptr_t)a) & 15) == 0 ? 2 : (al8 ? 1 : 0);
    const size_t plane = (size_t)mg * npad;
    int8_t *L0 = limbs + (size_t)frame * 3 * plane;
    int8_t *L1 = L0 + plane;
    const int we = w - 1;
    long long *E = edge + (size_t)frame * 4 * we * w;
    // E layout: [tb][lr][e][q]: tb 0 top / 1 bottom, lr 0 LP / 1 RS
    auto eidx = [&](int tb, int lr, int e, int q) { return ((size_t)(tb * 2 + lr) * we + e) * w + q; };
    long long *bp = BAND ? bandp + (size_t)frame * prep_band_longs(w) : nullptr;
    const int i_lo = BAND ? blockIdx.x * band_rows : 0;
    const int i_hi = BAND ? min(mg, i_lo + band_rows) : mg;

    for (int j = threadIdx.x; j < npad; j += blockDim.x) colE[j] = 0;
    if (threadIdx.x == 0) {
        etot = 0;
        need3 = 0;
        xmax = 0;
    }
    __syncthreads();
    int my_xmax = 0;

    long long col[kMaxCol4][4];
#pragma unroll
    for (int c = 0; c < kMaxCol4; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) col[c][q] = 0;
    long long my_etot = 0;
    int my_need3 = 0;

    for (int i = i_lo + wave; i < i_hi; i += NW) {
        const bool top = i < we, bot = i >= mg - we;
        long long rpart = 0;
#pragma unroll
        for (int c = 0; c < kMaxCol4; ++c) {
            int j0 = 4 * (lane + 64 * c);
            if (j0 >= npad) break;
            int d0p = 0, d1p = 0;
            int Xs[4];
            grid_values4<DS>(a, n, ng, i, j0, vec, Xs);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int j = j0 + q;
                int X = Xs[q];
                my_xmax = max(my_xmax, X);
                if (GRID) {
                    if (grid && j < ng)
                        grid[(size_t)frame * mg * ng + (size_t)i * ng + j] =
                            DS ? 0.25 * (double)X : (double)X;
                } else {
                    int d0 = bdigit(X, dbits);
                    int x1 = (X - d0) >> dbits;
                    int d1 = bdigit(x1, dbits);
                    if (((x1 - d1) >> dbits) != 0) my_need3 = 1;
                    d0p |= (d0 & 255) << (8 * q);
                    d1p |= (d1 & 255) << (8 * q);
                }
                // GRID: the energies of X - xc (the single-precision FFT form's
                // centred grid; xc = 0 otherwise); the padding columns j >= ng
                // (X = 0) lie outside the grid and add nothing
                const long long xd = GRID ? (j < ng ? (long long)(X - xc) : 0LL) : (long long)X;
                long long x2 = xd * xd;
                rpart += x2;
                col[c][q] += x2;
                if ((top || bot) && j < ng) {
                    if (j < we) rowbuf(wave, 0)[j] = x2;
                    if (j >= ng - we) rowbuf(wave, 1)[ng - 1 - j] = x2;
                }
            }
            if (!GRID) {
                *(int *)(L0 + (size_t)i * npad + j0) = d0p;
                *(int *)(L1 + (size_t)i * npad + j0) = d1p;
            }
        }
        my_etot += rpart;   // the lane's share, summed over the wave once at the end
        if (top || bot) {
            // a border row's energy (the branch is uniform: a wave takes the row)
            const long long r = wave_sum_i64(rpart);
            if (lane == 0) {
                long long *tT = BAND ? bp : rT, *tB = BAND ? bp + we : rB;
                if (top) tT[i] = r;
                if (bot) tB[mg - 1 - i] = r;
            }
            // prefix sums of this row's X^2 over the first / last q columns
            for (int q = lane; q < w; q += 64) {
                long long lp = 0, rs = 0;
                for (int j = 0; j < q; ++j) {
                    lp += rowbuf(wave, 0)[j];
                    rs += rowbuf(wave, 1)[j];
                }
                if (top) {
                    E[eidx(0, 0, i, q)] = lp;
                    E[eidx(0, 1, i, q)] = rs;
                }
                if (bot) {
                    E[eidx(1, 0, mg - 1 - i, q)] = lp;
                    E[eidx(1, 1, mg - 1 - i, q)] = rs;
                }
            }
        }
    }
    // column energies and totals
#pragma unroll
    for (int c = 0; c < kMaxCol4; ++c) {
        int j0 = 4 * (lane + 64 * c);
        if (j0 >= npad) break;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (j0 + q < ng) atomicAdd((unsigned long long *)&colE[j0 + q], (unsigned long long)col[c][q]);
    }
    {
        const long long wt = wave_sum_i64(my_etot);
        if (lane == 0) atomicAdd((unsigned long long *)&etot, (unsigned long long)wt);
    }
    if (my_need3) need3 = 1;
    atomicMax(&xmax, my_xmax);
    __syncthreads();
    if (BAND) {
        // this band's share of the border-column, total and flag reductions
        long long *P = bp + 2 * we + (size_t)blockIdx.x * (2 * we + 3);
        for (int s = threadIdx.x; s < we; s += blockDim.x) {
            P[s] = colE[s];
            P[we + s] = colE[ng - 1 - s];
        }
        if (threadIdx.x == 0) {
            P[2 * we] = etot;
            P[2 * we + 1] = need3;
            P[2 * we + 2] = xmax;
        }
        return;
    }
    for (int s = threadIdx.x; s < we; s += blockDim.x) {
        cL[s] = colE[s];
        cR[s] = colE[ng - 1 - s];
    }
    if (hz) {
        const int W = 2 * w - 1;
        int32_t *hf = hz + (size_t)frame * 2 * W * W;
        for (int k = threadIdx.x; k < 2 * W * W; k += blockDim.x) hf[k] = 0;
    }
    __syncthreads();
    prep_tables<DS, GRID, 8>(a, m, n, mg, ng, w, npad, dbits, frame, cL, cR, rT, rB, etot, need3,
                             xmax, E, L0, nlimb, vmax, atab, atab_d);
}

// The energy table of each frame from its bands' sums (one block per frame);
// with hz, the frame's 2 W^2 int32 correlation table is zeroed too (for a
// correlation launch that adds row slices into it).
template <bool DS, bool GRID>
__global__ __launch_bounds__(256) void k_prep_finish(const uint16_t *__restrict__ raw, int m, int n,
                                                     int mg, int ng, int w, int npad, int dbits,
                                                     int nbands, int8_t *__restrict__ limbs,
                                                     int32_t *__restrict__ nlimb,
                                                     int32_t *__restrict__ vmax,
                                                     long long *__restrict__ atab,
                                                     const long long *__restrict__ edge,
                                                     double *__restrict__ atab_d,
                                                     const int32_t *__restrict__ only,
                                                     const long long *__restrict__ bandp,
                                                     int32_t *__restrict__ hz)
{
    const int frame = blockIdx.x;
    if (GRID && only && !only[frame]) return;
    // dynamic LDS: cL[w] | cR[w] | rT[w] | rB[w] | acc[2(w-1) + 1]
    extern __shared__ long long lds_fin[];
    long long *cL = lds_fin, *cR = cL + w, *rT = cR + w, *rB = rT + w, *acc = rB + w;
    __shared__ int s_need3, s_xmax;
    const int we = w - 1, W = 2 * w - 1;
    const long long *bp = bandp + (size_t)frame * prep_band_longs(w);
    const int rec = 2 * we + 3;
    for (int s = threadIdx.x; s <= 2 * we; s += blockDim.x) acc[s] = 0;
    if (threadIdx.x == 0) {
        s_need3 = 0;
        s_xmax = 0;
    }
    if (hz) {
        int32_t *hf = hz + (size_t)frame * 2 * W * W;
        for (int k = threadIdx.x; k < 2 * W * W; k += blockDim.x) hf[k] = 0;
    }
    __syncthreads();
    // every band record at once: column sums and the total added, flags
    // merged; each thread's loads are all issued before their first use
    constexpr int PER = 16;
    const int total = nbands * rec;
    for (int i0 = 0; i0 < total; i0 += PER * (int)blockDim.x) {
        long long v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = i0 + u * (int)blockDim.x + (int)threadIdx.x;
            v[u] = idx < total ? bp[2 * we + idx] : 0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = i0 + u * (int)blockDim.x + (int)threadIdx.x;
            if (idx >= total) continue;
            const int s = idx % rec;
            if (s <= 2 * we)
                atomicAdd((unsigned long long *)&acc[s], (unsigned long long)v[u]);
            else if (s == 2 * we + 1) {
                if (v[u]) atomicOr(&s_need3, 1);
            } else {
                atomicMax(&s_xmax, (int)v[u]);
            }
        }
    }
    for (int s = threadIdx.x; s < 2 * we; s += blockDim.x) (s < we ? rT[s] : rB[s - we]) = bp[s];
    __syncthreads();
    for (int s = threadIdx.x; s < we; s += blockDim.x) {
        cL[s] = acc[s];
        cR[s] = acc[we + s];
    }
    __syncthreads();
    const size_t plane = (size_t)mg * npad;
    int8_t *L0 = GRID ? nullptr : limbs + (size_t)frame * 3 * plane;
    prep_tables<DS, GRID, 16>(raw + (size_t)frame * m * n, m, n, mg, ng, w, npad, dbits, frame, cL,
                              cR, rT, rB, acc[2 * we], s_need3, s_xmax,
                              edge + (size_t)frame * 4 * we * w, L0, nlimb, vmax, atab, atab_d);
}

// ---------------------------------------------------------------------------
// Template rows as Toeplitz sources, in eight byte-phase copies so that every
// operand read is 8-byte aligned: TP[i][q][phi][x] = digit q of
// Y[i][x + phi - padl] (zero outside 0..ng-1), q = 0,1, phi = 0..7; with nq = 3
// a third plane q = 2 holds the digit sums e0 + e1 (base-128 digits, so the
// sum stays within int8).
__global__ __launch_bounds__(kBlock) void k_tpad(const int8_t *__restrict__ tl, int mg, int ng,
                                                 int npad, int trow, int padl, int nq,
                                                 int8_t *__restrict__ tp)
{
    const size_t total = (size_t)mg * nq * kPhases * trow;
    const size_t plane = (size_t)mg * npad;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        int x = (int)(idx % trow);
        size_t r = idx / trow;
        int phi = (int)(r % kPhases);
        r /= kPhases;
        int q = (int)(r % nq), i = (int)(r / nq);
        int j = x + phi - padl;
        int8_t v = 0;
        if (j >= 0 && j < ng) {
            const size_t k = (size_t)i * npad + j;
            v = q < 2 ? tl[q * plane + k] : (int8_t)(tl[k] + tl[plane + k]);
        }
        tp[idx] = v;
    }
}

// ---------------------------------------------------------------------------
// Correlation on the matrix cores.
//
// s_waitcnt vmcnt(N) lgkmcnt(0), then s_barrier.  As compiler builtins (not
// inline asm) the wait is visible to the compiler's own counter tracking, so it
// adds no waits of its own for transfers this one already covers; the empty
// asm statements keep memory accesses from moving across.
template <int N>
__device__ __forceinline__ void wait_barrier()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// k_corr_int8: block = 4 waves = 4 frames (one per wave), one (s-group,
// t-group) of NS x NT tiles of 32 shifts.  NPA digit planes of the frame
// starting at PA0 (main pass: planes 0,1; extra pass: plane 2) times the two
// template planes.  Every product is a separate exact int32 accumulator.
//
// KB (base-128 digits, |d| <= 64): the main pass takes three products instead
// of four, d0 e0, d1 e1 and (d0 + d1)(e0 + e1), whose operands stay within
// int8 (Karatsuba); h = H00 + 128 (S - H00 - H11) + 16384 H11.  The template
// carries its digit sums as a third plane; the frame's are formed in the ring
// once a row has landed (a byte-wise add of the row's two planes into a third
// plane of its slot).  The extra pass weights its products by 128^(2+q).
//
// Per template row i and strip of 128 frame columns: each wave reads its A
// operands (frame rows i+s) from its own ring of 32*NS rows and the B operands
// (template row i as a Toeplitz operand) from the shared template buffer, four
// K-chunks of 32 columns, 12 MFMAs per chunk (16 with four products), the LDS
// reads of chunk k+1 interleaved with the MFMAs of chunk k.  Template rows are taken in pairs:
// while rows i, i+1 are in use, template rows i+2, i+3 and frame rows
// i+s_lo+RING+1, +2 stream global -> LDS (no registers) into the other two of
// four statically distinct template buffers (the pair loop is unrolled by two,
// so every LDS read provably targets a buffer other than the ones being
// filled) and two free ring slots; one wait for every transfer and one
// barrier per pair.
//
// Frames of several templates (same geometry) in one launch: btp (nullable)
// gives each block-column x its template rows, and its frames run from
// bf0[x] to bfe[x] - 1 (at most four, all of that template); without btp,
// block-column x takes frames 4x .. 4x+3 of the one template tp.
//
// HALF (one tile, 2w-1 <= 16): the 32x32 MFMA product holds two 16x16 shift
// tiles on its diagonal, rows and columns 0-15 over the first 64 columns of
// each strip and rows and columns 16-31 over the last 64, so a strip takes two
// K-chunks instead of four; the tile is the sum of the two diagonal blocks
// (the off-diagonal ones mix the halves and are dropped).
template <int NS, int NT, int NPA, int PA0, int NDMA, bool KB, bool HALF = false>
__global__ __launch_bounds__(kBlock, 1) void k_corr_int8(
    const int8_t *__restrict__ limbs, const int32_t *__restrict__ nlimb,
    const int8_t *__restrict__ tp_one, const int8_t *__restrict__ zsrc_one, int C, int mg,
    int npad, int trow, int padl, int w, int tgroups, int nslice, long long *__restrict__ hout,
    const int8_t *const *__restrict__ btp, const int *__restrict__ bf0,
    const int *__restrict__ bfe)
{
    static_assert(!HALF || (NS == 1 && NT == 1), "the half tile is one tile");
    constexpr int RING = HALF ? 16 : 32 * NS;   // frame rows an iteration reads
    constexpr int RS = RING + 3;      // ring slots: a pair of rows reads RING + 1, the next
                                      // pair's two arrive meanwhile
    constexpr bool SUMP = KB && PA0 == 0;        // three-product main pass
    constexpr int NA = SUMP ? 3 : NPA;           // frame operands per tile: digits (+ sums)
    constexpr int NB = SUMP ? 3 : 2;             // template operands per tile
    constexpr int NACC = SUMP ? 3 : NPA * 2;
    constexpr int DB = KB ? 7 : 8;               // digit bits
    constexpr int TQ = KB ? 3 : 2;               // template planes held
    constexpr int MAXT = KB ? kMaxTrowSum : kMaxTrow;
    constexpr int SLOT = (SUMP ? 3 : 2) * kStrip + 16;   // LDS bytes per ring slot (+ bank offset)
    // MFMA K-chunks per strip (npad is a multiple of kStrip)
    constexpr int KC = HALF ? kStrip / 64 : kStrip / 32;
    __shared__ __attribute__((aligned(16))) int8_t s_ring[kWaves * RS * SLOT];
    __shared__ __attribute__((aligned(16))) int8_t s_tA[TQ * kPhases * MAXT];
    __shared__ __attribute__((aligned(16))) int8_t s_tB[TQ * kPhases * MAXT];
    __shared__ __attribute__((aligned(16))) int8_t s_tC[TQ * kPhases * MAXT];
    __shared__ __attribute__((aligned(16))) int8_t s_tD[TQ * kPhases * MAXT];

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int rho = lane % 32, h = lane / 32;
    // this block-column's template and frames
    const int8_t *tp = btp ? btp[blockIdx.x] : tp_one;
    const int8_t *zsrc = btp ? tp + (size_t)mg * TQ * kPhases * trow : zsrc_one;  // zero tail
    const int fb0 = btp ? bf0[blockIdx.x] : (int)blockIdx.x * kWaves;
    const int fbe = btp ? bfe[blockIdx.x] : C;
    const int frame = fb0 + wave;
    const int sg = blockIdx.y / tgroups, tg = blockIdx.y % tgroups;
    const int W = 2 * w - 1;
    const int s_lo = -(w - 1) + 32 * NS * sg;
    const int t_lo = -(w - 1) + 32 * NT * tg;
    const int s_hi = min(s_lo + RING - 1, w - 1);
    // template rows of this block: slice blockIdx.z of the rows the shift group
    // overlaps (nslice > 1 splits a few frames' work over many blocks, which then
    // add their exact partial sums into the zeroed table)
    const int r_lo = max(0, -s_hi), r_hi = min(mg, mg - s_lo);
    const int slen = (r_hi - r_lo + nslice - 1) / nslice;
    const int i_lo = r_lo + (int)blockIdx.z * slen, i_hi = min(r_hi, i_lo + slen);
    if (i_lo >= i_hi) return;
    const size_t plane = (size_t)mg * npad;

    // does this wave's frame take part in this pass?
    bool live = frame < fbe;
    if (PA0 > 0) live = live && nlimb[frame] > 2;
    if (PA0 > 0) {
        // skip the whole block when no frame of it needs the extra digit plane
        int any = 0;
        for (int k = 0; k < kWaves; ++k) {
            int f = fb0 + k;
            if (f < fbe && nlimb[f] > 2) any = 1;
        }
        if (!any) return;
    }
    const int8_t *fl = limbs + (size_t)(live ? frame : 0) * 3 * plane + (size_t)PA0 * plane;
    int8_t *my_ring = s_ring + (size_t)wave * RS * SLOT;

    v16i acc[NS][NT][NACC];
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b)
#pragma unroll
            for (int c = 0; c < NACC; ++c) acc[a][b][c] = v16i{0};

    // Frame row r (columns ks..ks+127 of the digit planes) into ring slot
    // (r - s_lo) mod RS: one global -> LDS transfer of four bytes per lane, lanes
    // 0-31 the first plane and 32-63 the second (with one plane, a copy of it
    // into the slot's unused half).  A row outside the frame (or of a frame past
    // the stack) comes from the zero block.  Every lane takes part, so each call
    // is exactly one transfer.  Each wave fills its own ring.
    //
    // The compiler cannot tell ring slots apart, so it would wait for every ring
    // transfer before the next ring read; the slot address goes through an empty
    // asm so that it does not.  The reads of a row are ordered after its
    // transfer by the explicit waits: the rows a pair reads were requested by
    // the previous pair (or before the first), which ended with every transfer
    // retired.
    auto ring_fill = [&](int r, int ks) {
        const int slot = (r - s_lo) % RS;
        const bool have = live && r >= 0 && r < mg;
        const int p = NPA == 2 ? lane / 32 : 0;
        unsigned la = (unsigned)(uintptr_t)(__attribute__((address_space(3))) void *)(
            my_ring + (size_t)slot * SLOT);
        asm volatile("" : "+v"(la));
        // cache policy 2: non-temporal (the frame rows are read once per strip),
        // which leaves L2 to the template rows every block reads
        __builtin_amdgcn_global_load_lds(
            (const void *)(have ? fl + (size_t)p * plane + (size_t)r * npad + ks + (lane % 32) * 4
                                : zsrc + (lane % 32) * 4),
            (__attribute__((address_space(3))) void *)(uintptr_t)la, 4, 0, 2);
    };
    // template row ti into dst, global -> LDS: wave v moves bytes [v Qw, (v+1) Qw)
    // of the row (Qw = rowbytes/4) in exactly NDMA transfers of 1 KB with every
    // lane active.  The last transfer runs up to 1 KB past the quarter: into the
    // next quarter with the very bytes that wave writes there, or for the last
    // quarter past the row (inside the buffer: 3 Qw + NDMA KB <= TQ * 8 * MAXT
    // bytes; and inside the template allocation, whose last row is followed by
    // a 1 KB zero tail), where nothing reads.
    const int rowbytes = TQ * kPhases * trow;     // one template row: every plane, all phases
    const int qw = rowbytes / kWaves;
    auto dma_row = [&](int ti, int8_t *dst) {
        const int8_t *src = tp + (size_t)ti * rowbytes + wave * qw;
#pragma unroll
        for (int c = 0; c < NDMA; ++c)
            __builtin_amdgcn_global_load_lds(
                (const void *)(src + c * 1024 + lane * 16),
                (__attribute__((address_space(3))) void *)(dst + wave * qw + c * 1024), 16, 0, 0);
    };
    // SUMP: the digit-sum plane of frame rows r0 .. r0 + nrows - 1, once their
    // transfers have landed (after a wait): two rows per step, a dword of four
    // columns per lane.  Each wave writes only its own ring, and its later
    // reads of these bytes follow in its own LDS order.
    auto ring_sums = [&](int r0, int nrows) {
        for (int k = 0; k < nrows; k += 2) {
            const int kk = k + lane / 32;
            if (kk < nrows) {
                int8_t *row = my_ring + (size_t)((r0 + kk - s_lo) % RS) * SLOT;
                const int c = (lane % 32) * 4;
                const unsigned x = *(const unsigned *)(row + c);
                const unsigned y = *(const unsigned *)(row + kStrip + c);
                *(unsigned *)(row + 2 * kStrip + c) = byte_add(x, y);
            }
        }
    };

    for (int ks = 0; ks < npad; ks += kStrip) {
        // frame rows for the first pair (template rows i_lo and i_lo + 1):
        // i_lo + s_lo + q, q < RING + 1; template rows i_lo and i_lo + 1
        for (int q = 0; q <= RING; ++q) ring_fill(i_lo + s_lo + q, ks);
        dma_row(i_lo, s_tA);
        if (i_lo + 1 < i_hi) dma_row(i_lo + 1, s_tB);
        wait_barrier<0>();
        if constexpr (SUMP) ring_sums(i_lo + s_lo, RING + 1);

        // MFMAs of template row i (from tcur) against frame rows i + s
        auto rowmma = [&](int i, const int8_t *tcur) {
            // operand addresses of K-chunk 0; chunk kc adds kc*32 bytes.  The byte
            // phase of a template read does not depend on kc (32 is a multiple of 8).
            // HALF: operand row / column rho takes shift rho % 16 over the
            // strip's half rho / 16
            const int rs = HALF ? (rho & 15) : rho;
            const int ch = HALF ? 64 * (rho >> 4) : 0;
            const int8_t *abase[NS][NA];
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int p = 0; p < NA; ++p)
                    abase[st][p] = my_ring + (size_t)((i + 32 * st + rs) % RS) * SLOT +
                                   p * kStrip + 16 * h + ch;
            const int8_t *bbase[NT][NB];
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
                // template bytes B[i][k - t] for k = ks + kc*32 + 16h + e, t = t_lo + 32 tt + rho,
                // read from the phase copy that makes them 8-byte aligned
                int x0 = ks + 16 * h + ch - (t_lo + 32 * tt + rs) + padl;
                int phi = x0 & (kPhases - 1);
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    bbase[tt][q] = tcur + ((size_t)q * kPhases + phi) * trow + (x0 - phi);
            }
            auto load_a = [&](int kc, v4i (&av)[NS][NA]) {
#pragma unroll
                for (int st = 0; st < NS; ++st)
#pragma unroll
                    for (int p = 0; p < NA; ++p) av[st][p] = *(const v4i *)(abase[st][p] + kc * 32);
            };
            auto load_b = [&](int kc, v4i (&bv)[NT][NB]) {
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                    for (int q = 0; q < NB; ++q) {
                        const int2 *src = (const int2 *)(bbase[tt][q] + kc * 32);
                        int2 lo = src[0], hi = src[1];
                        bv[tt][q] = v4i{lo.x, lo.y, hi.x, hi.y};
                    }
            };

            // t-tile 1 reads its template bytes 32 columns before t-tile 0's
            // (t is 32 larger), so its operand at chunk kc + 1 is t-tile 0's at
            // chunk kc: with two t-tiles only t-tile 0 is read after chunk 0
            constexpr int NTL = NT == 2 ? 1 : NT;   // t-tiles read per later chunk
            auto load_b_next = [&](int kc, const v4i (&bv)[NT][NB], v4i (&bn)[NT][NB]) {
#pragma unroll
                for (int tt = 0; tt < NTL; ++tt)
#pragma unroll
                    for (int q = 0; q < NB; ++q) {
                        const int2 *src = (const int2 *)(bbase[tt][q] + kc * 32);
                        int2 lo = src[0], hi = src[1];
                        bn[tt][q] = v4i{lo.x, lo.y, hi.x, hi.y};
                    }
                if constexpr (NT == 2) {
#pragma unroll
                    for (int q = 0; q < NB; ++q) bn[1][q] = bv[0][q];
                }
            };

            v4i av[NS][NA], bv[NT][NB];
            load_a(0, av);
            load_b(0, bv);
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                v4i an[NS][NA], bn[NT][NB];
                if (kc + 1 < KC) {
                    load_a(kc + 1, an);
                    load_b_next(kc + 1, bv, bn);
                }
                if constexpr (SUMP) {
#pragma unroll
                    for (int st = 0; st < NS; ++st)
#pragma unroll
                        for (int tt = 0; tt < NT; ++tt) {
                            acc[st][tt][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                av[st][0], bv[tt][0], acc[st][tt][0], 0, 0, 0);
                            acc[st][tt][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                av[st][NA - 1], bv[tt][NB - 1], acc[st][tt][1], 0, 0, 0);
                            acc[st][tt][NACC - 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                av[st][1 % NA], bv[tt][1], acc[st][tt][NACC - 1], 0, 0, 0);
                        }
                } else {
#pragma unroll
                    for (int st = 0; st < NS; ++st)
#pragma unroll
                        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                            for (int p = 0; p < NPA; ++p)
#pragma unroll
                                for (int q = 0; q < 2; ++q)
                                    acc[st][tt][p * 2 + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                        av[st][p], bv[tt][q], acc[st][tt][p * 2 + q], 0, 0, 0);
                }
                // issue order: one MFMA, one LDS read of the next chunk, ..., then
                // the remaining MFMAs (with one wave per SIMD, a burst of reads
                // would hold back the MFMA issue, and reads sunk next to their
                // uses would stall on their latency)
                constexpr int NRD = NS * NA + NTL * NB;
                constexpr int NMF = NS * NT * NACC;
#pragma unroll
                for (int g = 0; g < (NRD < NMF ? NRD : NMF); ++g) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, NMF, 0);
                __builtin_amdgcn_sched_barrier(0);
                if (kc + 1 < KC) {
#pragma unroll
                    for (int st = 0; st < NS; ++st)
#pragma unroll
                        for (int p = 0; p < NA; ++p) av[st][p] = an[st][p];
#pragma unroll
                    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                        for (int q = 0; q < NB; ++q) bv[tt][q] = bn[tt][q];
                }
            }
        };
        // A pair of template rows i, i+1 (from t0, t1) while the next pair's
        // template rows (into n0, n1, the buffers of the previous pair) and frame
        // rows i + s_lo + RING + 1, + 2 stream in.  One barrier per pair: every
        // transfer of this pair has landed and every wave is done with t0, t1
        // before the next pair reads n0, n1 and refills t0, t1.
        auto pair = [&](int i, const int8_t *t0, const int8_t *t1, int8_t *n0, int8_t *n1) {
            if (i + 2 < i_hi) dma_row(i + 2, n0);
            if (i + 3 < i_hi) dma_row(i + 3, n1);
            ring_fill(i + s_lo + RING + 1, ks);
            ring_fill(i + s_lo + RING + 2, ks);
            rowmma(i, t0);
            if (i + 1 < i_hi) rowmma(i + 1, t1);
            wait_barrier<0>();
            if constexpr (SUMP) ring_sums(i + s_lo + RING + 1, 2);
        };
        for (int i = i_lo; i < i_hi; i += 4) {
            pair(i, s_tA, s_tB, s_tC, s_tD);
            if (i + 2 < i_hi) pair(i + 2, s_tC, s_tD, s_tA, s_tB);
        }
    }

    if (!live) return;
    long long *H = hout + (size_t)frame * W * W;
    // accumulator r of lane (rho, h): row 8 (r / 4) + 4 h + r % 4, column rho
    auto tile_value = [&](int st, int tt, int r) {
        long long v = 0;
        if constexpr (SUMP) {
            const long long h00 = acc[st][tt][0][r], sum = acc[st][tt][1][r];
            const long long h11 = acc[st][tt][NACC - 1][r];
            v = h00 + (sum - h00 - h11) * 128 + h11 * 16384;
        } else {
#pragma unroll
            for (int p = 0; p < NPA; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    v += (long long)acc[st][tt][p * 2 + q][r] * (1LL << (DB * (PA0 + p + q)));
        }
        return v;
    };
    auto put = [&](int s, int t, long long v) {
        size_t k = (size_t)(s + w - 1) * W + (t + w - 1);
        if (nslice > 1)
            atomicAdd((unsigned long long *)&H[k], (unsigned long long)v);
        else if (PA0 == 0)
            H[k] = v;
        else
            H[k] += v;
    };
    if constexpr (HALF) {
        // rows 0-15 are r < 8; row + 16 is r + 8, whose column + 16 sits 16
        // lanes up (every lane takes part in the exchange)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const long long up = tile_value(0, 0, r + 8);
            const unsigned ulo = (unsigned)__shfl_down((int)(unsigned)up, 16);
            const unsigned uhi = (unsigned)__shfl_down((int)(unsigned)((unsigned long long)up >> 32), 16);
            const long long v = tile_value(0, 0, r) + (long long)(((unsigned long long)uhi << 32) | ulo);
            const int s = s_lo + 8 * (r / 4) + 4 * h + (r % 4);
            const int t = t_lo + rho;
            if (rho < 16 && s <= w - 1 && t <= w - 1) put(s, t, v);
        }
        return;
    }
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int s = s_lo + 32 * st + 8 * (r / 4) + 4 * h + (r % 4);
                int t = t_lo + 32 * tt + rho;
                if (s > w - 1 || t > w - 1) continue;
                put(s, t, tile_value(st, tt, r));
            }
}

// ---------------------------------------------------------------------------
// Combine with exact integer energies: E = A(s,t) + B(s,t) - 2h(s,t) is the
// integer sum of squared differences over D; f = E*scale/Area.  B comes from
// the template's own table at (-s,-t).
struct CandI {
    double f;
    int s, t;
    double second;
};

__device__ inline bool precedes_i(double f1, int s1, int t1, double f2, int s2, int t2)
{
    if (f1 != f2) return f1 < f2;
    int r1 = max(abs(s1), abs(t1)), r2 = max(abs(s2), abs(t2));
    if (r1 != r2) return r1 < r2;
    int l1 = abs(s1) + abs(t1), l2 = abs(s2) + abs(t2);
    if (l1 != l2) return l1 < l2;
    if (s1 != s2) return s1 < s2;
    return t1 < t2;
}

// btabs (nullable): each frame's own template table (frames of several
// templates in one launch), else btab_one for every frame.
template <int TB>
__global__ __launch_bounds__(TB) void k_combine_i64(const long long *__restrict__ atab,
                                                        const long long *__restrict__ btab_one,
                                                        const long long *const *__restrict__ btabs,
                                                        const long long *__restrict__ hbuf,
                                                        int mg, int ng, int w, int ds,
                                                        double scale, double *__restrict__ fsurf,
                                                        double *__restrict__ fmin_out,
                                                        int32_t *__restrict__ coarse_st,
                                                        int32_t *__restrict__ shifts,
                                                        double *__restrict__ gaps,
                                                        double *__restrict__ frefine)
{
    const int W = 2 * w - 1;
    const int frame = blockIdx.x;
    const long long *A = atab + (size_t)frame * W * W;
    const long long *Hh = hbuf + (size_t)frame * W * W;
    const long long *btab_t = btabs ? btabs[frame] : btab_one;
    CandI c{INFINITY, INT32_MIN, 0, INFINITY};
    for (int k = threadIdx.x; k < W * W; k += blockDim.x) {
        int si = k / W, ti = k % W;
        int s = si - (w - 1), t = ti - (w - 1);
        long long B = btab_t[(size_t)(W - 1 - si) * W + (W - 1 - ti)];
        long long E = A[k] + B - 2 * Hh[k];
        double area = (double)(mg - abs(s)) * (double)(ng - abs(t));
        double f = ((double)E * scale) / area;
        if (fsurf) fsurf[(size_t)frame * W * W + k] = f;
        if (c.s == INT32_MIN) {
            c.f = f; c.s = s; c.t = t;
        } else if (precedes_i(f, s, t, c.f, c.s, c.t)) {
            c.second = fmin(c.second, c.f);
            c.f = f; c.s = s; c.t = t;
        } else {
            c.second = fmin(c.second, f);
        }
    }
    __shared__ double sf[TB], ss2[TB];
    __shared__ int si_[TB], sj_[TB];
    int tid = threadIdx.x;
    sf[tid] = c.f; ss2[tid] = c.second; si_[tid] = c.s; sj_[tid] = c.t;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) {
            int ys = si_[tid + off];
            if (ys != INT32_MIN) {
                int xs = si_[tid];
                double xf = sf[tid], yf = sf[tid + off];
                double sec = fmin(ss2[tid], ss2[tid + off]);
                if (xs == INT32_MIN) {
                    sf[tid] = yf; si_[tid] = ys; sj_[tid] = sj_[tid + off]; ss2[tid] = sec;
                } else if (precedes_i(yf, ys, sj_[tid + off], xf, xs, sj_[tid])) {
                    ss2[tid] = fmin(sec, xf);
                    sf[tid] = yf; si_[tid] = ys; sj_[tid] = sj_[tid + off];
                } else {
                    ss2[tid] = fmin(sec, yf);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (fmin_out) fmin_out[frame] = sf[0];
        coarse_st[2 * frame] = si_[0];
        coarse_st[2 * frame + 1] = sj_[0];
        if (gaps) gaps[2 * frame] = ss2[0] - sf[0];
        if (!ds) {
            shifts[2 * frame] = si_[0];
            shifts[2 * frame + 1] = sj_[0];
            if (gaps) gaps[2 * frame + 1] = INFINITY;
        }
    }
    if (!ds && frefine && tid < 9) frefine[(size_t)frame * 9 + tid] = NAN;
}

// ---------------------------------------------------------------------------
// Launch shapes of k_corr_int8: the operand-transfer count per wave, the
// tile groups and the row slices.
template <int NS, int NT, int NPA, int PA0, int NDMA, bool KB, bool HALF>
hipError_t launch_corr_ndma(const int8_t *limbs, const int32_t *nlimb, const Int8Tmpl &tt, int C,
                            const Geom &g, int nslice, long long *h, hipStream_t st,
                            const Int8Multi *mm)
{
    const int tgroups = (g.W + 32 * NT - 1) / (32 * NT);
    const int sgroups = (g.W + 32 * NS - 1) / (32 * NS);
    dim3 grid(mm ? mm->nblocks : (C + kWaves - 1) / kWaves, sgroups * tgroups, nslice);
    const int8_t *zsrc = tt.tp + (size_t)g.mg * tt.nq * kPhases * tt.trow;  // zero tail
    k_corr_int8<NS, NT, NPA, PA0, NDMA, KB, HALF><<<grid, kBlock, 0, st>>>(
        limbs, nlimb, tt.tp, zsrc, C, g.mg, tt.npad, tt.trow, tt.padl, g.w, tgroups, nslice, h,
        mm ? mm->btp : nullptr, mm ? mm->bf0 : nullptr, mm ? mm->bfe : nullptr);
    return hipGetLastError();
}

template <int NS, int NT, int NPA, int PA0, bool KB, bool HALF>
hipError_t launch_corr_nq(const int8_t *limbs, const int32_t *nlimb, const Int8Tmpl &tt, int C,
                          const Geom &g, int nslice, long long *h, hipStream_t st,
                          const Int8Multi *mm)
{
    // transfers per wave for a quarter of a template row (nq * 2 * trow bytes);
    // the buffer bound 3 quarters + NDMA KB <= nq * 8 * max row holds for every
    // trow up to that maximum
    switch ((tt.nq * 2 * tt.trow + 1023) / 1024) {
    case 1: return launch_corr_ndma<NS, NT, NPA, PA0, 1, KB, HALF>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    case 2: return launch_corr_ndma<NS, NT, NPA, PA0, 2, KB, HALF>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    case 3: return launch_corr_ndma<NS, NT, NPA, PA0, 3, KB, HALF>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    case 4: return launch_corr_ndma<NS, NT, NPA, PA0, 4, KB, HALF>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    default: return hipErrorInvalidValue;
    }
}

template <int NS, int NT, int NPA, int PA0, bool HALF = false>
hipError_t launch_corr_variant(const int8_t *limbs, const int32_t *nlimb, const Int8Tmpl &tt,
                               int C, const Geom &g, int nslice, long long *h, hipStream_t st,
                               const Int8Multi *mm)
{
    // base-128 digits with a digit-sum plane (three products), or base-256 (four)
    if (tt.nq == 3) {
        if (tt.trow > kMaxTrowSum) return hipErrorInvalidValue;
        return launch_corr_nq<NS, NT, NPA, PA0, true, HALF>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    }
    if (tt.trow > kMaxTrow) return hipErrorInvalidValue;
    return launch_corr_nq<NS, NT, NPA, PA0, false, HALF>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
}

// Row slices per block group: with fewer blocks than compute units (a few
// frames), enough slices to cover the device twice over, each slice at least 4
// template rows (a slice first fills its ring with 32 NS + 1 frame rows).
int corr_slices(int C, const Geom &g, int NS, int NT, int nblocks = -1)
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
            cus = v;
        else
            cus = 256;
    }
    const long long groups = (long long)((g.W + 32 * NS - 1) / (32 * NS)) *
                             ((g.W + 32 * NT - 1) / (32 * NT));
    const long long blocks = (long long)(nblocks >= 0 ? nblocks : (C + kWaves - 1) / kWaves) * groups;
    if (blocks >= cus) return 1;
    const long long want = (2LL * cus + blocks - 1) / blocks;
    const int most = max(1, g.mg / 4);
    return (int)(want < most ? want : most);
}

int grid_for(size_t total)
{
    size_t gsz = (total + kBlock - 1) / kBlock;
    if (gsz > 65535 * 4) gsz = 65535 * 4;
    return (int)(gsz < 1 ? 1 : gsz);
}

}  // namespace

Int8Geom int8_geom(const Geom &g)
{
    Int8Geom r;
    r.npad = (g.ng + kStrip - 1) / kStrip * kStrip;
    const int NT = g.W <= 32 ? 1 : 2;
    const int tgroups = (g.W + 32 * NT - 1) / (32 * NT);
    const int t_max = -(g.w - 1) + 32 * NT * tgroups - 1;
    // padl >= t_max keeps every read in the row; (padl + w) % 8 == 0 makes the
    // first byte of lane rho's operand, padl - t_lo - rho + (multiple of 8), fall
    // in 8-byte groups of eight consecutive lanes (rho = 8g..8g+7), so that each
    // group reads eight distinct bank pairs of the eight phase copies
    r.padl = ((t_max > 0 ? t_max : 0) + 4 + g.w + 7) / 8 * 8 - g.w;
    // trow = 16 (mod 32): the eight phase copies of a row start 4 (mod 8) dwords
    // apart, so eight lanes reading eight phases hit eight disjoint bank pairs
    r.trow = (r.padl + r.npad + g.w + 40 + 31) / 32 * 32 + 16;
    return r;
}

bool int8_applicable(const Geom &g)
{
    // exact int32 accumulation needs fewer than 2^17 terms per shift; the
    // prep kernel holds at most 2048 grid columns and forms grid values from
    // one 2x2 level at most; the correlation kernel holds template rows of at
    // most kMaxTrow bytes
    if (g.dtype != MOCO_U16 || g.ds > 1 || (long long)g.mg * g.ng >= 131072 || g.ng > 2048 ||
        g.w > 512)
        return false;
    return int8_geom(g).trow <= kMaxTrow;
}

size_t int8_template_bytes(const Geom &g, int nq)
{
    // the Toeplitz rows, then kInt8ZeroTail zero bytes (the source of frame
    // rows outside the frame)
    return (size_t)g.mg * nq * kPhases * int8_geom(g).trow + kInt8ZeroTail;
}

// Bands per frame for a launch of C frames: one block per frame once the
// frames alone fill the device; fewer frames are split over bands of rows
// (at least one row per wave) so that about 512 blocks stream them.
int prep_bands(int C, int mg)
{
    if (C >= 256) return 1;
    const int want = (512 + C - 1) / C;
    return std::max(1, std::min(std::min(want, kPrepMaxBands), mg / kWaves));
}

template <bool DS, int kMaxCol4, bool GRID>
void prep_launch_c(const uint16_t *frames, int C, const Geom &g, int npad, int dbits, size_t lds,
                   int8_t *limbs, int32_t *nlimb, int32_t *vmax, long long *atab, long long *edge,
                   double *grid, double *atab_d, const int32_t *only, hipStream_t st, int xc,
                   int32_t *hz)
{
    const int nb = prep_bands(C, g.mg);
    if (nb <= 1) {
        k_prep_u16<DS, kMaxCol4, kWaves, GRID, false><<<C, kWaves * 64, lds, st>>>(
            frames, g.m, g.n, g.mg, g.ng, g.w, npad, dbits, limbs, nlimb, vmax, atab, edge, grid,
            atab_d, only, xc, 0, nullptr, hz);
        return;
    }
    const int rows = (g.mg + nb - 1) / nb;
    const int nbu = (g.mg + rows - 1) / rows;   // bands that hold rows (<= nb)
    // the bands' sums follow the C frames' border prefix tables
    long long *bandp = edge + (size_t)C * 4 * (g.w - 1) * g.w;
    k_prep_u16<DS, kMaxCol4, kWaves, GRID, true><<<dim3(nbu, C), kWaves * 64, lds, st>>>(
        frames, g.m, g.n, g.mg, g.ng, g.w, npad, dbits, limbs, nlimb, vmax, atab, edge, grid,
        atab_d, only, xc, rows, bandp, nullptr);
    k_prep_finish<DS, GRID><<<C, 256, (6 * (size_t)g.w - 1) * sizeof(long long), st>>>(
        frames, g.m, g.n, g.mg, g.ng, g.w, npad, dbits, nbu, limbs, nlimb, vmax, atab, edge, atab_d,
        only, bandp, hz);
}

size_t prep_lds(const Geom &g, int npad, int nw)
{
    const int we1 = g.w > 1 ? g.w - 1 : 1;
    return ((size_t)npad + (size_t)nw * 2 * we1 + 4 * (size_t)g.w + 2) * sizeof(long long);
}

template <bool DS, bool GRID>
void prep_launch(const uint16_t *frames, int C, const Geom &g, int npad, int dbits, int8_t *limbs,
                 int32_t *nlimb, int32_t *vmax, long long *atab, long long *edge, double *grid,
                 double *atab_d, const int32_t *only, hipStream_t st, int xc = 0,
                 int32_t *hz = nullptr)
{
    // 256 grid columns per chunk (64 lanes x 4 columns)
    const int nc = (npad + 255) / 256;
    const size_t lds = prep_lds(g, npad, kWaves);
    if (nc <= 1)
        prep_launch_c<DS, 1, GRID>(frames, C, g, npad, dbits, lds, limbs, nlimb, vmax, atab, edge,
                                   grid, atab_d, only, st, xc, hz);
    else if (nc <= 2)
        prep_launch_c<DS, 2, GRID>(frames, C, g, npad, dbits, lds, limbs, nlimb, vmax, atab, edge,
                                   grid, atab_d, only, st, xc, hz);
    else if (nc <= 4)
        prep_launch_c<DS, 4, GRID>(frames, C, g, npad, dbits, lds, limbs, nlimb, vmax, atab, edge,
                                   grid, atab_d, only, st, xc, hz);
    else
        prep_launch_c<DS, 8, GRID>(frames, C, g, npad, dbits, lds, limbs, nlimb, vmax, atab, edge,
                                   grid, atab_d, only, st, xc, hz);
}

hipError_t launch_prep_u16(const uint16_t *frames, int C, const Geom &g, int npad, int dbits,
                           int8_t *limbs, int32_t *nlimb, int32_t *vmax, long long *atab,
                           long long *edge, hipStream_t st, int32_t *hz)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (dbits != 7 && dbits != 8) return hipErrorInvalidValue;
    if (g.ds)
        prep_launch<true, false>(frames, C, g, npad, dbits, limbs, nlimb, vmax, atab, edge,
                                 nullptr, nullptr, nullptr, st, 0, hz);
    else
        prep_launch<false, false>(frames, C, g, npad, dbits, limbs, nlimb, vmax, atab, edge,
                                  nullptr, nullptr, nullptr, st, 0, hz);
    return hipGetLastError();
}

bool prep_grid_applicable(const Geom &g)
{
    // the border prefix sums take O(w^2) steps per border row: wide windows
    // keep the separate grid and energy kernels
    if (g.dtype != MOCO_U16 || g.ds > 1 || g.ng > 2048 || g.w > 128) return false;
    const int npad = (g.ng + kStrip - 1) / kStrip * kStrip;
    return prep_lds(g, npad, kWaves) <= 64 * 1024;
}


hipError_t launch_prep_grid(const uint16_t *frames, int C, const Geom &g, double *grid,
                            double *atab, int32_t *vmax, long long *edge, hipStream_t st,
                            const int32_t *only, int xc)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (!prep_grid_applicable(g)) return hipErrorInvalidValue;
    const int npad = (g.ng + kStrip - 1) / kStrip * kStrip;
    if (g.ds)
        prep_launch<true, true>(frames, C, g, npad, 8, nullptr, nullptr, vmax, nullptr, edge,
                                grid, atab, only, st, xc);
    else
        prep_launch<false, true>(frames, C, g, npad, 8, nullptr, nullptr, vmax, nullptr, edge,
                                 grid, atab, only, st, xc);
    return hipGetLastError();
}

hipError_t launch_tpad(const int8_t *tlimbs, const Geom &g, const Int8Tmpl &tt, hipStream_t st)
{
    clear_stale_error();
    k_tpad<<<grid_for((size_t)tt.nq * kPhases * g.mg * tt.trow), kBlock, 0, st>>>(
        tlimbs, g.mg, g.ng, tt.npad, tt.trow, tt.padl, tt.nq, tt.tp);
    return hipGetLastError();
}

bool int8_corr_adds_slices(int C, const Geom &g, int tile, int nblocks)
{
    const bool small = tile == 16 || tile == 32 || (tile == 0 && g.W <= 32);
    return (small ? corr_slices(C, g, 1, 1, nblocks) : corr_slices(C, g, 2, 2, nblocks)) > 1;
}

hipError_t launch_corr_int8(const int8_t *limbs, const int32_t *nlimb, const Int8Tmpl &tt, int C,
                            const Geom &g, long long *h, hipStream_t st, const Int8Multi *mm,
                            int tile, bool h_zeroed)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    hipError_t e;
    // (the template rows are padded for 2x2 tiles of 32 only when 2w-1 > 32)
    if ((tile != 0 && tile != 16 && tile != 32 && tile != 64) || (tile == 64 && g.W <= 32) ||
        (tile == 16 && g.W > 16))
        return hipErrorInvalidValue;
    const bool half = tile == 16 || (tile == 0 && g.W <= 16);
    const bool small = half || tile == 32 || (tile == 0 && g.W <= 32);
    const int nb = mm ? mm->nblocks : -1;
    const int nslice = small ? corr_slices(C, g, 1, 1, nb) : corr_slices(C, g, 2, 2, nb);
    if (nslice > 1 && !h_zeroed) {
        // the slices add into a zeroed table
        if ((e = launch_fill_i32((int32_t *)h, 2 * C * g.W * g.W, 0, st)) != hipSuccess) return e;
    }
    if (half) {
        if ((e = launch_corr_variant<1, 1, 2, 0, true>(limbs, nlimb, tt, C, g, nslice, h, st,
                                                        mm)) != hipSuccess)
            return e;
        return launch_corr_variant<1, 1, 1, 2, true>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    }
    if (small) {
        if ((e = launch_corr_variant<1, 1, 2, 0>(limbs, nlimb, tt, C, g, nslice, h, st, mm)) !=
            hipSuccess)
            return e;
        return launch_corr_variant<1, 1, 1, 2>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
    }
    if ((e = launch_corr_variant<2, 2, 2, 0>(limbs, nlimb, tt, C, g, nslice, h, st, mm)) !=
        hipSuccess)
        return e;
    return launch_corr_variant<2, 2, 1, 2>(limbs, nlimb, tt, C, g, nslice, h, st, mm);
}

hipError_t launch_combine_i64(const long long *atab, const long long *btab_t, const long long *h,
                              int C, const Geom &g, double *fsurf, double *fmin,
                              int32_t *coarse_st, int32_t *shifts, double *gaps, double *frefine,
                              hipStream_t st, const long long *const *btabs)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    const double scale = g.ds ? 0.0625 : 1.0;
    // a few frames: four times the threads per frame
    if (C <= 128)
        k_combine_i64<1024><<<C, 1024, 0, st>>>(atab, btab_t, btabs, h, g.mg, g.ng, g.w, g.ds,
                                                 scale, fsurf, fmin, coarse_st, shifts, gaps,
                                                 frefine);
    else
        k_combine_i64<kBlock><<<C, kBlock, 0, st>>>(atab, btab_t, btabs, h, g.mg, g.ng, g.w,
                                                    g.ds, scale, fsurf, fmin, coarse_st, shifts,
                                                    gaps, frefine);
    return hipGetLastError();
}

}  // namespace moco
