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

#include "grid_src.h"
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
// only (may be null): frames whose only[f] is 0 are skipped
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(const T *__restrict__ fr, int C, int m, int n,
                                                   int mg, int ng, int ds,
                                                   double *__restrict__ out,
                                                   const int32_t *__restrict__ only)
{
    const size_t plane = (size_t)mg * ng;
    const size_t total = (size_t)C * plane;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        size_t f = idx / plane;
        if (only && !only[f]) continue;
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

// The same for the frames whose only[f] is set: block (x, frame), the blocks
// of unset frames exit at once (the masked passes of the certified forms
// usually cover few frames of a chunk).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_masked(const T *__restrict__ fr, int m, int n,
                                                          int mg, int ng, int ds,
                                                          double *__restrict__ out,
                                                          const int32_t *__restrict__ only)
{
    const int f = blockIdx.y;
    if (!only[f]) return;
    const size_t plane = (size_t)mg * ng;
    const T *a = fr + (size_t)f * m * n;
    double *o = out + (size_t)f * plane;
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < plane;
         r += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(r / ng), j = (int)(r - (r / ng) * ng);
        double v;
        if (ds) {
            const T *p = a + (size_t)(2 * i) * n + 2 * j;
            double x00 = (double)p[0], x01 = (double)p[1];
            double x10 = (double)p[n], x11 = (double)p[n + 1];
            v = (((x00 + x01) + x10) + x11) / 4.0;
        } else {
            v = (double)a[(size_t)i * n + j];
        }
        o[r] = v;
    }
}

// Same values as k_coarse with downsampling, four grid columns per thread:
// the eight frame pixels of each of the two rows are read with 16-byte loads
// (n a multiple of 8, 16-byte aligned frames) and summed in k_coarse's order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_ds4(const T *__restrict__ fr, int C, int m,
                                                       int n, int mg, int ng,
                                                       double *__restrict__ out)
{
    const int nq = ng / 4;
    const size_t total = (size_t)C * mg * nq;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t f = idx / ((size_t)mg * nq);
        const int r = (int)(idx - f * mg * nq);
        const int i = r / nq, q = r - i * nq;
        const T *p0 = fr + f * (size_t)m * n + (size_t)(2 * i) * n + 8 * q;
        T a[8], b[8];
        static_assert(sizeof(T) == 2 || sizeof(T) == 4, "uint16 or float32");
        if (sizeof(T) == 2) {
            *(uint4 *)a = *(const uint4 *)p0;
            *(uint4 *)b = *(const uint4 *)(p0 + n);
        } else {
            *(uint4 *)a = *(const uint4 *)p0;
            *((uint4 *)a + 1) = *((const uint4 *)p0 + 1);
            *(uint4 *)b = *(const uint4 *)(p0 + n);
            *((uint4 *)b + 1) = *((const uint4 *)(p0 + n) + 1);
        }
        double v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            v[e] = ((((double)a[2 * e] + (double)a[2 * e + 1]) + (double)b[2 * e]) +
                    (double)b[2 * e + 1]) /
                   4.0;
        double *o = out + f * (size_t)mg * ng + (size_t)i * ng + 4 * q;
        *(double2 *)o = double2{v[0], v[1]};
        *(double2 *)(o + 2) = double2{v[2], v[3]};
    }
}

// One more level of the image pyramid: the 2x2 box mean of an FP64 level,
// odd trailing row/column dropped, summed in the same order as the first level.
__global__ __launch_bounds__(kBlock) void k_half(const double *__restrict__ in, int C, int m,
                                                 int n, double *__restrict__ out)
{
    const int mh = m / 2, nh = n / 2;
    const size_t plane = (size_t)mh * nh;
    const size_t total = (size_t)C * plane;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t f = idx / plane;
        const int r = (int)(idx - f * plane);
        const int i = r / nh, j = r - i * nh;
        const double *p = in + f * (size_t)m * n + (size_t)(2 * i) * n + 2 * j;
        out[idx] = (((p[0] + p[1]) + p[n]) + p[n + 1]) / 4.0;
    }
}

// Exclusive prefix sums out[k] = v[0] + ... + v[k-1], k = 0..n (n <= 2*kBlock),
// in a fixed order: pairs per thread, a shuffle scan per wave, wave carries.
// Every thread of the block must call it; it starts and ends with a barrier.
__device__ void block_excl_scan(const double *v, double *out, int n, double *wsum)
{
    __syncthreads();
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const double x0 = 2 * t < n ? v[2 * t] : 0.0, x1 = 2 * t + 1 < n ? v[2 * t + 1] : 0.0;
    const double l = x0 + x1;
    double inc = l;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    double carry = 0.0;
    for (int k = 0; k < wave; ++k) carry += wsum[k];
    const double ex = carry + (inc - l);
    if (2 * t <= n) out[2 * t] = ex;
    if (2 * t + 1 <= n) out[2 * t + 1] = ex + x0;
    __syncthreads();
}

// Frame overlap energies A(s,t) = sum of a'^2 over rows [max(0,s), mg-1+min(0,s)]
// and columns [max(0,t), ng-1+min(0,t)] (the frame side of D at (s,t)), for
// |s|,|t| <= w-1, written [s+w-1][t+w-1].  One block per frame, one pass of
// coalesced column sums over the grid, then only its border: with E = w-1,
//   A = total - (rows cut at the top or bottom) - (columns cut at the left or
//       right) + (the corner block cut twice),
// from the row sums of the E border rows at either end, the column sums of
// the E border columns at either side, and for each corner the 2-D prefix
// sums of its E x E block (a running column sum per row, scanned along the
// row).  All sums run in a fixed order.  flip: write A(s,t) at [-s+w-1][-t+w-1]
// instead (the template's energies over D at (s,t) are its A at (-s,-t)).
// pmax (may be null): per frame,
// ceil(pscale * largest grid value), the pixel bound the x2 step uses, or
// INT32_MAX when pscale is 0.
// The grid comes from src as grid_at<SRC> reads it (an FP64 grid, or the
// frames' pixels).
// Every grid value enters the sums less `center` (0 but in the single-precision
// FFT form, whose correlation is of the centred grids); the pixel bound is of
// the values themselves.
template <int SRC>
__global__ __launch_bounds__(kBlock) void k_energy(const void *__restrict__ src, int m, int n,
                                                   int mg, int ng, int w, bool flip,
                                                   double *__restrict__ atab,
                                                   int32_t *__restrict__ pmax, double pscale,
                                                   double center, const int32_t *__restrict__ only)
{
    if (only && !only[blockIdx.x]) return;
    extern __shared__ double elds[];
    const int E = w - 1, W = 2 * w - 1;
    double *colL = elds, *colR = colL + (E + 1), *rowT = colR + (E + 1), *rowB = rowT + (E + 1);
    double *CL = rowB + (E + 1), *CR = CL + (E + 1), *RT = CR + (E + 1), *RB = RT + (E + 1);
    double *cp = RB + (E + 1), *ks = cp + (E + 1), *red = ks + (E + 2);
    __shared__ double wsum[kBlock / 64];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const void *a = grid_frame<SRC>(src, blockIdx.x, m, n, mg, ng);
    double *A = atab + (size_t)blockIdx.x * W * W;

    // column sums (every column: the total; border columns kept) and the maximum
    double tot = 0.0, mx = 0.0;
    for (int j = tid; j < ng; j += kBlock) {
        double cs = 0.0, cm = 0.0;
#pragma unroll 8
        for (int i = 0; i < mg; ++i) {
            const double v = grid_at<SRC>(a, n, ng, i, j), x = v - center;
            cs = fma(x, x, cs);
            cm = fmax(cm, v);
        }
        tot += cs;
        mx = fmax(mx, cm);
        if (j < E) colL[j] = cs;
        if (j >= ng - E) colR[ng - 1 - j] = cs;
    }
    // border row sums, one wave per row
    for (int rr = wave; rr < 2 * E; rr += kBlock / 64) {
        const int i = rr < E ? rr : mg - 1 - (rr - E);
        double rs = 0.0;
        for (int j = lane; j < ng; j += 64) {
            const double x = grid_at<SRC>(a, n, ng, i, j) - center;
            rs = fma(x, x, rs);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) rs += __shfl_xor(rs, off);
        if (lane == 0) {
            if (rr < E)
                rowT[rr] = rs;
            else
                rowB[rr - E] = rs;
        }
    }
    red[tid] = tot;
    red[kBlock + tid] = mx;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (tid < off) {
            red[tid] += red[tid + off];
            red[kBlock + tid] = fmax(red[kBlock + tid], red[kBlock + tid + off]);
        }
        __syncthreads();
    }
    tot = red[0];
    if (pmax && tid == 0) {
        const double b = ceil(pscale * red[kBlock]);
        pmax[blockIdx.x] = (pscale > 0.0 && b < 2147483647.0) ? (int32_t)b : INT32_MAX;
    }
    block_excl_scan(rowT, RT, E, wsum);
    block_excl_scan(rowB, RB, E, wsum);
    block_excl_scan(colL, CL, E, wsum);
    block_excl_scan(colR, CR, E, wsum);

    // the four corners: bit 1 = rows cut at the bottom (s < 0), bit 0 = columns
    // cut at the right (t < 0)
    for (int c = 0; c < 4; ++c) {
        const bool bottom = c & 2, right = c & 1;
        for (int j = tid; j < E; j += kBlock) cp[j] = 0.0;
        for (int s = 0; s <= E; ++s) {
            if (s > 0) {
                const int row = bottom ? mg - s : s - 1;
                for (int j = tid; j < E; j += kBlock) {
                    const double x = grid_at<SRC>(a, n, ng, row, right ? ng - 1 - j : j) - center;
                    cp[j] = fma(x, x, cp[j]);
                }
            }
            block_excl_scan(cp, ks, E, wsum);  // ks[t]: the s x t corner block
            if (bottom && s == 0) continue;   // s = 0 belongs to the top corners
            const double rcut = bottom ? RB[s] : RT[s];
            const int si = (bottom ? -s : s) + E;
            for (int t = tid + (right ? 1 : 0); t <= E; t += kBlock) {
                const int ti = (right ? -t : t) + E;
                const size_t k = (size_t)si * W + ti;
                A[flip ? (size_t)W * W - 1 - k : k] = ((tot - rcut) - (right ? CR[t] : CL[t])) + ks[t];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_energy_rows: the same table from one pass over the grid's rows, for grids
// of at most 2048 columns and w <= 128 (four waves per frame; a wave takes
// every fourth row, a lane four columns of each 256-column chunk).  The
// energies of the first and last w-1 rows come from fixed-order wave sums,
// the total from each lane's share summed over the wave and then the waves,
// and each lane keeps its columns' energies; then the cuts (rows from the top and bottom, columns from the
// left and right) are made cumulative, and each wave writes one quadrant of
// the table: for s = 1..w-1 it reads the s-th border row's corner values
// again (each lane one or two of the first or last w-1 columns), takes their
// prefix sums over the columns with a wave scan, adds them to its running
// corner sums, and writes row s of the quadrant.  Every sum runs in a fixed
// order, so results are reproducible; with uint16 grids every partial sum is
// exact, as in k_energy.
constexpr int kErWaves = 4;
constexpr int kErMaxChunks = 8;   // 8 x 256 grid columns

// v of another lane by a data-parallel-primitives move of both 32-bit halves;
// lanes without a source (outside the row, or of a masked row) get 0
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// inclusive prefix sum over the 64 lanes of a wave (fixed order): within each
// row of 16 lanes by shifts of 1, 2, 4 and 8 lanes, then lane 15's sum added
// to rows 1 and 3 and lane 31's to rows 2 and 3 (moves within the VALU, not
// through the LDS crossbar)
__device__ inline double wave_incl_scan(double v)
{
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

template <int SRC, int NCH>
__global__ __launch_bounds__(kErWaves * 64) void k_energy_rows(
    const void *__restrict__ src, int m, int n, int mg, int ng, int w, double *__restrict__ atab,
    int32_t *__restrict__ pmax, double pscale, double center, const int32_t *__restrict__ only)
{
    if (only && !only[blockIdx.x]) return;
    const int E = w - 1, W = 2 * w - 1, we1 = E > 0 ? E : 1;
    // LDS: rT[w] | rB[w] | cL[w] | cR[w] | cpart[NW][2][we1] | wtot[NW] | wmax[NW]
    extern __shared__ double erl[];
    double *rT = erl, *rB = rT + w, *cL = rB + w, *cR = cL + w;
    double *cpart = cR + w, *wtot = cpart + kErWaves * 2 * we1, *wmax = wtot + kErWaves;
    const int frame = blockIdx.x, wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const void *a = grid_frame<SRC>(src, frame, m, n, mg, ng);
    auto sq = [&](int i, int j) {
        const double x = grid_at<SRC>(a, n, ng, i, j) - center;
        return x * x;
    };

    double col[NCH][4];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) col[c][q] = 0.0;
    // float pixels as they are, rows 16-byte aligned: four columns per load
    const bool vec4 = SRC == 4 && (n & 3) == 0 && (((uintptr_t)a) & 15) == 0;
    double my_tot = 0.0, my_max = 0.0;   // the lane's share of the total
    for (int i = wave; i < mg; i += kErWaves) {
        double rpart = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j0 = 4 * (lane + 64 * c);
            double v[4];
            if (vec4 && j0 + 3 < ng) {
                const float4 f4 = *(const float4 *)((const float *)a + (size_t)i * n + j0);
                v[0] = f4.x, v[1] = f4.y, v[2] = f4.z, v[3] = f4.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = j0 + q < ng ? grid_at<SRC>(a, n, ng, i, j0 + q) : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double x2 = 0.0;
                if (j0 + q < ng) {
                    const double x = v[q] - center;
                    my_max = fmax(my_max, v[q]);
                    x2 = x * x;
                }
                rpart += x2;
                col[c][q] += x2;
            }
        }
        my_tot += rpart;
        // the row's energy is needed only for the first and last w-1 rows (a
        // whole wave takes the row, so the branch is uniform)
        if (i < E || i >= mg - E) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) rpart += __shfl_xor(rpart, off);
            if (lane == 0) {
                if (i < E) rT[i] = rpart;
                if (i >= mg - E) rB[mg - 1 - i] = rpart;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_tot += __shfl_xor(my_tot, off);
    // per-wave partials: the border columns' energies, the total, the maximum
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * (lane + 64 * c) + q;
            if (j < ng && j < E) cpart[(size_t)wave * 2 * we1 + j] = col[c][q];
            if (j < ng && j >= ng - E) cpart[(size_t)wave * 2 * we1 + we1 + (ng - 1 - j)] = col[c][q];
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_max = fmax(my_max, __shfl_xor(my_max, off));
    if (lane == 0) {
        wtot[wave] = my_tot;
        wmax[wave] = my_max;
    }
    __syncthreads();
    // cumulative cuts: rows from the top / bottom, columns from the left / right
    if (threadIdx.x == 0 || threadIdx.x == 64) {
        double *cut = threadIdx.x == 0 ? rT : rB;
        double acc = 0.0;
        for (int s = 0; s < w; ++s) {
            const double v = s < E ? cut[s] : 0.0;
            cut[s] = acc;
            acc += v;
        }
    } else if (threadIdx.x == 128 || threadIdx.x == 192) {
        const int side = threadIdx.x == 128 ? 0 : 1;
        double *cut = side ? cR : cL;
        double acc = 0.0;
        for (int s = 0; s < w; ++s) {
            cut[s] = acc;
            if (s < E) {
                double ce = 0.0;
                for (int v = 0; v < kErWaves; ++v) ce += cpart[(size_t)v * 2 * we1 + side * we1 + s];
                acc += ce;
            }
        }
    }
    __syncthreads();
    double Etot = 0.0, mx = 0.0;
    for (int v = 0; v < kErWaves; ++v) {
        Etot += wtot[v];
        mx = fmax(mx, wmax[v]);
    }
    if (pmax && threadIdx.x == 0) {
        const double b = ceil(pscale * mx);
        pmax[frame] = (pscale > 0.0 && b < 2147483647.0) ? (int32_t)b : INT32_MAX;
    }
    double *A = atab + (size_t)frame * W * W;
    // the row s = 0 and the column t = 0: no corner
    for (int tt = threadIdx.x; tt < W; tt += blockDim.x) {
        const int t = tt - E, at = t < 0 ? -t : t;
        A[(size_t)E * W + tt] = Etot - (t > 0 ? cL[at] : (t < 0 ? cR[at] : 0.0));
        if (tt != E) {
            const int si = tt, sv = si - E, as = sv < 0 ? -sv : sv;
            A[(size_t)si * W + E] = Etot - (sv > 0 ? rT[as] : rB[as]);
        }
    }
    // quadrant (side, lr) of wave side * 2 + lr: side 0 s > 0 (rows cut at the
    // top), 1 s < 0 (bottom); lr 0 t > 0 (columns cut at the left), 1 t < 0
    // (right).  Lane l holds column offsets l and l + 64 of the band.
    const int side = wave >> 1, lr = wave & 1;
    const double *rx = side ? rB : rT, *cx = lr ? cR : cL;
    double acc0 = 0.0, acc1 = 0.0;
    // unrolled so that several band rows' loads are in flight at once
#pragma unroll 8
    for (int s = 1; s < w; ++s) {
        const int i = side ? mg - s : s - 1;
        // squares of the band row at column offsets 0..E-1 from the cut edge
        const int o0 = lane, o1 = lane + 64;
        double v0 = o0 < E ? sq(i, lr ? ng - 1 - o0 : o0) : 0.0;
        double v1 = o1 < E ? sq(i, lr ? ng - 1 - o1 : o1) : 0.0;
        // prefix over offsets: corner(s, t) adds the sums over offsets < |t|
        const double p0 = wave_incl_scan(v0);
        // offsets past 63 exist only for w > 65 (the branch is uniform)
        const double p1 = E > 64 ? wave_incl_scan(v1) + __shfl(p0, 63) : 0.0;
        acc0 += p0;   // corner sums for |t| = lane + 1
        acc1 += p1;   // and |t| = lane + 65
        const double base = Etot - rx[s];
        const int si = side ? E - s : E + s;
        for (int k = 0; k < 2; ++k) {
            const int at = lane + 1 + 64 * k;
            if (at <= E) {
                const int tt = lr ? E - at : E + at;
                A[(size_t)si * W + tt] = (base - cx[at]) + (k ? acc1 : acc0);
            }
        }
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
                                                      double *__restrict__ hout,
                                                      const int32_t *__restrict__ only)
{
    if (only && !only[blockIdx.y]) return;
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
// Certificate of an argmin computed from an inexact correlation.  With
// |h^ - h| <= kf sqrt(m'n' Sa Sb) for every shift (Sa, Sb: the grids' sums of
// squares, the energies at shift (0,0)) and energy sums within ke (Sa or Sb),
// every computed f is within Delta/Area + u|f^| of the exact f, where
// Delta = 1.01 (ke (Sa+Sb) + 2u sqrt(Sa Sb) + 2 kf sqrt(m'n' Sa Sb)) also
// covers the rounding of A + B - 2h and of the division.  If the computed gap
// between the best and the second-best f exceeds twice the largest such bound
// (smallest overlap area (m'-w+1)(n'-w+1)), no other shift can reach the
// computed argmin's exact f, so it is the exact argmin of eq. (f) and its
// ties do not arise.  A lone shift (w = 1) is certified; a non-finite best f
// is not.
__device__ bool certified(const double *At, const double *btab, int mg, int ng, int w, double f1,
                          double f2, double kf, double ke)
{
    const double u = 0x1p-53;
    if (!(f1 == f1) || isinf(f1)) return false;
    if (isinf(f2)) return true;
    const int W = 2 * w - 1, c0 = (w - 1) * W + (w - 1);
    const double sa = fmax(At[c0], 0.0), sb = fmax(btab[c0], 0.0);
    const double sab = sqrt(sa) * sqrt(sb);
    const double delta =
        1.01 * (ke * (sa + sb) + 2.0 * u * sab + 2.0 * kf * sqrt((double)mg * (double)ng) * sab);
    const double amin = (double)(mg - (w - 1)) * (double)(ng - (w - 1));
    const double margin = (f2 - f1) - 1.01 * u * (fabs(f1) + fabs(f2));
    return margin > 2.0 * delta / amin;
}

// The single-precision form's certificate: the same rule with the
// correlation's error bound hb of Cert32 (first order in u32 = 2^-24, doubled)
// in place of kf sqrt(m'n' Sa Sb).  Its norms are those of the centred grids:
// |x|_2 = sqrt(Sa), |y|_2 = sqrt(Sb); |X|_inf is the largest magnitude of the
// frame's computed spectrum (its square formed in FP32, three roundings) and
// |Y|_inf that of the template's FP32 spectrum.  The bound holds in 2-norm
// over the whole P x Q output (frame transform error e1 sqrt(PQ) |x|_2 times
// |Y|_inf; template spectrum, product and inverse errors times |X|_inf
// sqrt(PQ) |y|_2; the 1/(PQ) scale), hence for every shift.
// Delta of the single-precision certificate for one frame (false when the
// frame's spectrum maximum is not finite): every computed f of the frame is
// within Delta/Area + u|f^| of the exact f.
// x2: the largest |X_k|^2 of the frame's computed spectrum
__device__ __forceinline__ bool cert32_delta_x2(const double *At, const double *btab, int w,
                                                double ke, float x2, double e1, double e2,
                                                double yinf, double sqrtpq, double *delta)
{
    const double u = 0x1p-53, u32 = 0x1p-24;
    const int W = 2 * w - 1, c0 = (w - 1) * W + (w - 1);
    const double sa = fmax(At[c0], 0.0), sb = fmax(btab[c0], 0.0);
    if (!(x2 <= 3.0e38f)) return false;
    const double xinf = sqrt((double)x2) * (1.0 + 4.0 * u32);
    const double na = sqrt(sa), nb = sqrt(sb);
    const double hb = 2.0 * (e1 * na * yinf + e2 * (xinf + e1 * sqrtpq * na) * nb);
    *delta = 1.01 * ((ke + 4.0 * u) * (sa + sb) + 2.0 * u * na * nb + 2.0 * hb);
    return true;
}

__device__ __forceinline__ bool cert32_delta(const double *At, const double *btab, int w,
                                             double ke, const float *xmax, int nxb, double e1,
                                             double e2, double yinf, double sqrtpq, int frame,
                                             double *delta)
{
    const float *xm = xmax + (size_t)frame * nxb;
    float x2 = 0.0f;
    for (int k = 0; k < nxb; ++k) x2 = fmaxf(x2, xm[k]);
    return cert32_delta_x2(At, btab, w, ke, x2, e1, e2, yinf, sqrtpq, delta);
}

__device__ __forceinline__ bool certified32(const double *At, const double *btab, int mg, int ng,
                                            int w, double f1, double f2, double ke,
                                            const float *xmax, int nxb, double e1, double e2,
                                            double yinf, double sqrtpq, int frame)
{
    const double u = 0x1p-53;
    if (!(f1 == f1) || isinf(f1)) return false;
    if (isinf(f2)) return true;
    double delta;
    if (!cert32_delta(At, btab, w, ke, xmax, nxb, e1, e2, yinf, sqrtpq, frame, &delta))
        return false;
    const double amin = (double)(mg - (w - 1)) * (double)(ng - (w - 1));
    const double margin = (f2 - f1) - 1.01 * u * (fabs(f1) + fabs(f2));
    return margin > 2.0 * delta / amin;
}

__global__ __launch_bounds__(kBlock) void k_combine(const double *__restrict__ atab,
                                                    const double *__restrict__ btab,
                                                    const double *__restrict__ hbuf, int mg,
                                                    int ng, int w, int ds,
                                                    double *__restrict__ fsurf,
                                                    double *__restrict__ fmin_out,
                                                    int32_t *__restrict__ coarse_st,
                                                    int32_t *__restrict__ shifts,
                                                    double *__restrict__ gaps,
                                                    double *__restrict__ frefine,
                                                    const int32_t *__restrict__ only,
                                                    int32_t *__restrict__ recheck, double kf,
                                                    double ke, Cert32 c32)
{
    const int W = 2 * w - 1;
    const int frame = blockIdx.x;
    if (only && !only[frame]) return;
    const double *At = atab + (size_t)frame * W * W;
    const double *h = hbuf + (size_t)frame * W * W;
    Cand c{INFINITY, INT32_MIN, 0, INFINITY};
    for (int k = threadIdx.x; k < W * W; k += blockDim.x) {
        int s = k / W - (w - 1), t = k % W - (w - 1);
        double A = At[k];
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
        if (recheck) {
            const bool ok = c32.xmax
                                ? certified32(At, btab, mg, ng, w, r.f, r.second, ke, c32.xmax,
                                              c32.nxb, c32.e1, c32.e2, c32.yinf, c32.sqrtpq,
                                              frame)
                                : certified(At, btab, mg, ng, w, r.f, r.second, kf, ke);
            recheck[frame] = ok ? 0 : 1;
        }
    }
    if (!ds && frefine && threadIdx.x < 9) frefine[(size_t)frame * 9 + threadIdx.x] = NAN;
}

// f at the coarse argmin by its definition (eq. (f)): the FP64 sum of squared
// differences of the searched grids over D, in a fixed order (exact for uint16
// grids: multiples of 1/16 below 2^32 per term).  One block per frame.
constexpr int kPolishRows = 8;   // rows whose loads a thread issues together

template <int SRC>
__global__ __launch_bounds__(kBlock) void k_polish(const void *__restrict__ src, int m, int n,
                                                   int mg, int ng, int w,
                                                   const double *__restrict__ tcoarse,
                                                   const int32_t *__restrict__ coarse_st,
                                                   const int32_t *__restrict__ skip,
                                                   double *__restrict__ fmin,
                                                   double *__restrict__ fsurf,
                                                   double *__restrict__ gaps)
{
    const int frame = blockIdx.x;
    if (skip && skip[frame]) return;
    const int s = coarse_st[2 * frame], t = coarse_st[2 * frame + 1];
    const void *a = grid_frame<SRC>(src, frame, m, n, mg, ng);
    const int i0 = max(0, -s), i1 = min(mg, mg - s), j0 = max(0, -t), j1 = min(ng, ng - t);
    // thread k takes columns j0 + k, j0 + k + 256, ... of every row of D,
    // kPolishRows rows at a time with every load of a batch issued before
    // the first is used (a fixed order of the terms)
    double acc = 0.0;
    for (int j = j0 + threadIdx.x; j < j1; j += kBlock)
        for (int i = i0; i < i1; i += kPolishRows) {
            double fv[kPolishRows], tv[kPolishRows];
#pragma unroll
            for (int u = 0; u < kPolishRows; ++u) {
                const bool in = i + u < i1;
                fv[u] = in ? grid_at<SRC>(a, n, ng, i + u + s, j + t) : 0.0;
                tv[u] = in ? tcoarse[(size_t)(i + u) * ng + j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kPolishRows; ++u) {
                const double d = fv[u] - tv[u];
                acc = fma(d, d, acc);
            }
        }
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double area = (double)(mg - abs(s)) * (double)(ng - abs(t));
        const double f = red[0] / area;
        const double f0 = fmin[frame];
        if (gaps) gaps[2 * frame] += f0 - f;
        fmin[frame] = f;
        const int W = 2 * w - 1;
        if (fsurf) fsurf[(size_t)frame * W * W + (size_t)(s + w - 1) * W + (t + w - 1)] = f;
    }
}

// An argmin that the single-precision certificate leaves open, settled from
// its candidates (uint16 pixels; the grid is their 2x2 box means, or the
// pixels themselves).  Every computed f of the frame is within
// delta = Delta/Area + u|f^| of the exact f (the certificate's bound), so a
// shift with f^ - delta above U = min over all shifts of (f^ + delta) has an
// exact f above the exact minimum: it is not the argmin and does not tie with
// it.  When every other shift lies in the 3 x 3 neighbourhood of the computed
// argmin, the exact f of those nine shifts (integer sums of squared
// differences of the box sums, i.e. 16 times the box-mean units, or of the
// pixels) settle the exact argmin under the tie order: the frame's coarse
// argmin, f there, its gap (the second-best of the nine, or the least
// computed f outside them) and the nine surface values are written, recheck
// is cleared and resolved set to 3.  Otherwise the frame keeps recheck for
// the FP64 pass.  resolved is written for every frame.  One block per frame.
constexpr int kCandRows = 8;   // template rows whose frame loads a thread issues together
constexpr int kCandBatch = 4;  // shifts whose table loads a thread issues together
constexpr int kCandMaxShifts = kCand32MaxShifts;

template <int SRC>   // 1: 2x2 box sums of uint16 pixels; 2: uint16 pixels
__global__ __launch_bounds__(kBlock) void k_cand32(
    const uint16_t *__restrict__ frames, int m, int n, int mg, int ng, int w, int ds,
    const double *__restrict__ atab, const double *__restrict__ btab,
    const double *__restrict__ hbuf, const double *__restrict__ tcoarse, double ke, Cert32 c32,
    int32_t *__restrict__ coarse_st, double *__restrict__ fmin_out, double *__restrict__ fsurf,
    double *__restrict__ gaps, int32_t *__restrict__ shifts, int32_t *__restrict__ recheck,
    int32_t *__restrict__ resolved)
{
    const int frame = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid == 0) resolved[frame] = 0;
    if (!recheck[frame]) return;
    const int W = 2 * w - 1, WW = W * W;
    if (WW > kCandMaxShifts) return;   // the launcher refuses such windows
    const double u = 0x1p-53;
    const double *At = atab + (size_t)frame * WW;
    const double *h = hbuf + (size_t)frame * WW;
    const int s0 = coarse_st[2 * frame], t0 = coarse_st[2 * frame + 1];
    __shared__ double red[kBlock];
    auto block_min = [&](double v) {
        red[tid] = v;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if (tid < off) red[tid] = fmin(red[tid], red[tid + off]);
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    // Delta, from the frame's spectrum maximum taken over the block
    float x2 = 0.0f;
    for (int k = tid; k < c32.nxb; k += kBlock)
        x2 = fmaxf(x2, c32.xmax[(size_t)frame * c32.nxb + k]);
    x2 = (float)-block_min(-(double)x2);
    double delta;
    if (!cert32_delta_x2(At, btab, w, ke, x2, c32.e1, c32.e2, c32.yinf, c32.sqrtpq, &delta))
        return;
    // every computed f (as the combine forms it) into LDS, kCandBatch shifts'
    // table loads at a time; U, and the least computed f outside the
    // neighbourhood
    __shared__ double sf[kCandMaxShifts];
    double up = INFINITY, fout = INFINITY;
    bool bad = false;
    for (int k0 = tid; k0 < WW; k0 += kCandBatch * kBlock) {
        double a[kCandBatch], b[kCandBatch], c[kCandBatch];
#pragma unroll
        for (int q = 0; q < kCandBatch; ++q) {
            const int k = min(k0 + q * kBlock, WW - 1);
            a[q] = At[k];
            b[q] = btab[k];
            c[q] = h[k];
        }
#pragma unroll
        for (int q = 0; q < kCandBatch; ++q) {
            const int k = k0 + q * kBlock;
            if (k >= WW) break;
            const int s = k / W - (w - 1), t = k % W - (w - 1);
            const double area = (double)(mg - abs(s)) * (double)(ng - abs(t));
            const double f = (a[q] + b[q] - 2.0 * c[q]) / area;
            sf[k] = f;
            if (!isfinite(f)) bad = true;
            up = fmin(up, f + delta / area + 1.01 * u * fabs(f));
            if (abs(s - s0) > 1 || abs(t - t0) > 1) fout = fmin(fout, f);
        }
    }
    if (__syncthreads_or(bad)) return;
    const double U = block_min(up);
    fout = block_min(fout);
    bool far = false;
    for (int k = tid; k < WW; k += kBlock) {
        const int s = k / W - (w - 1), t = k % W - (w - 1);
        if (abs(s - s0) <= 1 && abs(t - t0) <= 1) continue;
        const double area = (double)(mg - abs(s)) * (double)(ng - abs(t));
        const double f = sf[k];
        if (f - delta / area - 1.01 * u * fabs(f) <= U) far = true;
    }
    if (__syncthreads_or(far)) return;

    // exact sums for the nine shifts (s0 + du - 1, t0 + dv - 1).  Every load
    // is made, at an index clamped into the grid, and a term whose frame value
    // lies outside the grid counts zero (it is outside D): no branch around a
    // load, and all of a batch's loads are issued before the first is used.
    // The terms are integers (16 times the box-mean units, or pixel units) and
    // the sums stay below 2^53, so FP64 FMAs add them exactly.
    const uint16_t *fb = frames + (size_t)frame * m * n;
    const double tscale = SRC == 1 ? 4.0 : 1.0;
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    for (int j = tid; j < ng; j += kBlock) {
        for (int i0 = 0; i0 < mg; i0 += kCandRows) {
            // the batch's loads: two pixel pairs per box (its two rows), or
            // one pixel, and the template values
            uint32_t top[kCandRows + 2][3], bot[kCandRows + 2][3];
            double tv[kCandRows];
#pragma unroll
            for (int r = 0; r < kCandRows + 2; ++r)
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const int rr = min(max(i0 + s0 - 1 + r, 0), mg - 1);
                    const int cc = min(max(j + t0 + v - 1, 0), ng - 1);
                    if (SRC == 1) {
                        const char *pb = (const char *)(fb + (size_t)(2 * rr) * n + 2 * cc);
                        top[r][v] = *(const uint32_t *)pb;
                        bot[r][v] = *(const uint32_t *)(pb + 2 * (size_t)n);
                    } else {
                        top[r][v] = fb[(size_t)rr * n + cc];
                        bot[r][v] = 0;
                    }
                }
#pragma unroll
            for (int q = 0; q < kCandRows; ++q)
                tv[q] = tcoarse[(size_t)min(i0 + q, mg - 1) * ng + j] * tscale;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < kCandRows; ++q) {
                const bool row_in = i0 + q < mg;
#pragma unroll
                for (int du = 0; du < 3; ++du) {
                    const int fr = i0 + s0 - 1 + q + du;
                    const bool fr_in = row_in && fr >= 0 && fr < mg;
#pragma unroll
                    for (int dv = 0; dv < 3; ++dv) {
                        const int fc = j + t0 + dv - 1;
                        const uint32_t x = top[q + du][dv], y = bot[q + du][dv];
                        const int a = SRC == 1 ? (int)((x & 0xffffu) + (x >> 16) + (y & 0xffffu) +
                                                       (y >> 16))
                                               : (int)x;
                        const double d =
                            fr_in && fc >= 0 && fc < ng ? (double)a - tv[q] : 0.0;
                        acc[3 * du + dv] = fma(d, d, acc[3 * du + dv]);
                    }
                }
            }
        }
    }
    __shared__ double wsum[kBlock / 64][9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (tid % 64 == 0) wsum[tid / 64][q] = v;
    }
    __syncthreads();
    if (tid != 0) return;
    const double escale = SRC == 1 ? 0.0625 : 1.0;
    Cand c{INFINITY, INT32_MIN, 0, INFINITY};
    for (int q = 0; q < 9; ++q) {
        const int s = s0 + q / 3 - 1, t = t0 + q % 3 - 1;
        if (abs(s) > w - 1 || abs(t) > w - 1) continue;
        double e = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) e += wsum[k][q];
        const double area = (double)(mg - abs(s)) * (double)(ng - abs(t));
        const double f = (e * escale) / area;
        if (fsurf) fsurf[(size_t)frame * WW + (size_t)(s + w - 1) * W + (t + w - 1)] = f;
        cand_add(c, f, s, t);
    }
    c.second = fmin(c.second, fout);
    coarse_st[2 * frame] = c.s;
    coarse_st[2 * frame + 1] = c.t;
    fmin_out[frame] = c.f;
    if (gaps) gaps[2 * frame] = c.second - c.f;
    if (!ds) {
        shifts[2 * frame] = c.s;
        shifts[2 * frame + 1] = c.t;
        if (gaps) gaps[2 * frame + 1] = INFINITY;
    }
    recheck[frame] = 0;
    resolved[frame] = 3;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int count, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_add_i32(int32_t *__restrict__ p, const int32_t *__restrict__ q, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] += q[i];
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
template <>
struct RefAcc<double> {
    using type = double;
    __device__ static type term(double x, double y)
    {
        double d = x - y;
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

// uint16 x2 step, rolling form, for an even row length and 4-byte aligned
// buffers.  One wave owns 64 column groups of four template columns and a band
// of template rows; each lane walks down the band and keeps the three frame
// rows it needs (i+2s*-1, i+2s*, i+2s*+1, columns j0+2t*-1 .. j0+2t*+4) in
// registers, so every frame row is loaded once per lane, one row ahead of use.
// Frame rows are read as four dwords starting at column j0+2t*-2, which is even
// because t* contributes 2t*: the pairs of adjacent columns that the three
// column shifts need are those dwords or byte-aligned joins of two of them.
//
// Narrow mode (pixel bound M <= 32767 for frame and template): differences of
// two pixels come from one packed 16-bit subtract (|d| <= 32767 fits) and their
// squares from one 2-way 16-bit dot product into a 32-bit sum; the sums are
// read as unsigned and flushed into 64 bits every `flush` rows, flush*4*M^2 <
// 2^32, so no 32-bit sum wraps.  Wide mode: each square in 32 bits (d^2 <
// 2^32), added into 64-bit sums.  Terms outside the overlap domain (a frame
// column or row outside the frame, a template column past n) are masked to
// zero; a frame row outside the frame is skipped as a whole.  Partial sums go
// to [frame][band*ncw + cw][9] as exact FP64 integers.
constexpr int kRollMinRows = 8;

typedef short short2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x2a __attribute__((ext_vector_type(2), aligned(4)));

// Operands of one frame row: x[2v+p] holds the frame columns that template
// columns j0+2p, j0+2p+1 meet under column shift 2t*+v-1, i.e. columns
// j0+2t*+v-1+2p and one more, with masked terms zeroed.
struct RollRow {
    uint32_t x[6];
};

template <bool MASK>
__device__ __forceinline__ void roll_join(const uint32_t p[4], RollRow &r,
                                          const uint32_t (&mk)[3][2])
{
    // p[k] holds columns (c, c+1) with c = j0+2t*-2+2k; X[k] holds columns
    // j0+2t*-1+k and j0+2t*+k
    uint32_t X[5];
    X[0] = __builtin_amdgcn_alignbyte(p[1], p[0], 2);
    X[1] = p[1];
    X[2] = __builtin_amdgcn_alignbyte(p[2], p[1], 2);
    X[3] = p[2];
    X[4] = __builtin_amdgcn_alignbyte(p[3], p[2], 2);
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) r.x[2 * v + pr] = MASK ? X[v + 2 * pr] & mk[v][pr] : X[v + 2 * pr];
}

__device__ __forceinline__ uint32_t sub_u16x2(uint32_t f, uint32_t b)
{
    short2v d = __builtin_bit_cast(short2v, f) - __builtin_bit_cast(short2v, b);
    return __builtin_bit_cast(uint32_t, d);
}

__device__ __forceinline__ int sqr_acc(uint32_t d, int acc)
{
    short2v v = __builtin_bit_cast(short2v, d);
    return __builtin_amdgcn_sdot2(v, v, acc, false);
}

// MODE 0: narrow, no flush inside the band; 1: narrow with flushes; 2: wide
template <bool MASK, int MODE>
__device__ __forceinline__ void roll_rows(const uint16_t *__restrict__ fb,
                                          const uint16_t *__restrict__ tmpl, int m, int n, int i0,
                                          int i1, int S0, int j0, int c0, int flush, bool wide_ok,
                                          const uint32_t (&mk)[3][2], unsigned long long (&acc)[9])
{
    int acc32[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc32[q] = 0;
    auto load_frame = [&](int r, uint32_t (&p)[4]) {
        if (r >= 0 && r < m) {
            const char *row = (const char *)(fb + (size_t)r * n);
            if (!MASK) {
                const u32x4a q = *(const u32x4a *)(row + 2u * (unsigned)(c0 - 1));
                p[0] = q.x;
                p[1] = q.y;
                p[2] = q.z;
                p[3] = q.w;
            } else if (r > 0 && r < m - 1 && wide_ok) {
                // may run into the rows before and after: in the frame, masked
                const u32x4a q = *(const u32x4a *)((const char *)fb +
                                                   2u * (unsigned)(r * n + c0 - 1));
                p[0] = q.x;
                p[1] = q.y;
                p[2] = q.z;
                p[3] = q.w;
            } else {
                // a dword outside the row (both its columns: n is even) is read
                // at column 0 instead and masked
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int c = c0 - 1 + 2 * k;
                    const int o = (c >= 0 && c + 1 < n) ? c : 0;
                    p[k] = *(const uint32_t *)(row + 2u * (unsigned)o);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) p[k] = 0;
        }
    };
    auto load_tmpl = [&](int i, uint32_t (&t)[2]) {
        const char *row = (const char *)(tmpl + (size_t)i * n);
        if (!MASK || (i < m - 1 && n >= 6)) {
            // masked lanes (j0 <= n+2) may run into the next row
            const u32x2a q = *(const u32x2a *)(row + 2u * (unsigned)j0);
            t[0] = q.x;
            t[1] = q.y;
        } else {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int o = (j0 + 2 * k + 1 < n) ? j0 + 2 * k : 0;
                t[k] = *(const uint32_t *)(row + 2u * (unsigned)o);
            }
        }
    };
    uint32_t P[4], TB[2];
    RollRow R0, R1, R2;
    load_frame(i0 + S0 - 1, P);
    roll_join<MASK>(P, R0, mk);
    load_frame(i0 + S0, P);
    roll_join<MASK>(P, R1, mk);
    load_frame(i0 + S0 + 1, P);
    load_tmpl(i0, TB);
    int since = 0;
    // a masked term has both its frame and its template value zeroed
    auto one = [&](int u, const RollRow &R, const uint32_t (&Bm)[6]) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            if (MODE != 2) {
                const uint32_t d0 = sub_u16x2(R.x[2 * v], Bm[2 * v]);
                const uint32_t d1 = sub_u16x2(R.x[2 * v + 1], Bm[2 * v + 1]);
                acc32[3 * u + v] = sqr_acc(d1, sqr_acc(d0, acc32[3 * u + v]));
            } else {
#pragma unroll
                for (int pr = 0; pr < 2; ++pr) {
                    const uint32_t fx = R.x[2 * v + pr], bx = Bm[2 * v + pr];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int d = (int)((fx >> (16 * h)) & 0xffffu) -
                                      (int)((bx >> (16 * h)) & 0xffffu);
                        acc[3 * u + v] += (unsigned)d * (unsigned)d;
                    }
                }
            }
        }
    };
    auto step = [&](int i, const RollRow &ra, const RollRow &rb, RollRow &rc) {
        roll_join<MASK>(P, rc, mk);  // frame row i+S0+1
        uint32_t Bm[6];
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int pr = 0; pr < 2; ++pr) Bm[2 * v + pr] = MASK ? TB[pr] & mk[v][pr] : TB[pr];
        if (i + 1 < i1) {
            load_frame(i + S0 + 2, P);
            load_tmpl(i + 1, TB);
        }
        if ((unsigned)(i + S0 - 1) < (unsigned)m) one(0, ra, Bm);
        if ((unsigned)(i + S0) < (unsigned)m) one(1, rb, Bm);
        if ((unsigned)(i + S0 + 1) < (unsigned)m) one(2, rc, Bm);
        if (MODE == 1 && ++since == flush) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                acc[q] += (unsigned)acc32[q];
                acc32[q] = 0;
            }
            since = 0;
        }
    };
    for (int i = i0; i < i1; i += 3) {
        step(i, R0, R1, R2);
        if (i + 1 < i1) step(i + 1, R1, R2, R0);
        if (i + 2 < i1) step(i + 2, R2, R0, R1);
    }
    if (MODE != 2) {
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[q] += (unsigned)acc32[q];
    }
}

// Per-frame mode: narrow and a single flush at the end of a band of `rows`
// rows (the fast kernel), else narrow with flushes or wide (the slow units,
// run by k_refine_slow_finish).
__device__ __forceinline__ int roll_flush(const int32_t *pmax, int tmax, int frame)
{
    if (!pmax || tmax < 0) return -1;  // wide
    const long long M = max((long long)pmax[frame], (long long)tmax);
    if (M > 32767) return -1;
    return M > 0 ? (int)min(0xffffffffLL / (4 * M * M), (long long)(1 << 30)) : (1 << 30);
}

// One wave: frame, band of template rows, 64 column groups (`cw`).
template <bool SLOW>
__device__ __forceinline__ void roll_unit(const uint16_t *__restrict__ frames,
                                          const uint16_t *__restrict__ tmpl, int m, int n, int br,
                                          int ncw, int frame, int unit, int flush,
                                          const int32_t *__restrict__ coarse_st,
                                          double *__restrict__ partial, int units)
{
    const int lane = threadIdx.x % 64;
    const int band = unit / ncw, cw = unit % ncw;
    const int i0 = band * br, i1 = min(m, i0 + br);
    const bool fast = flush >= i1 - i0;
    if (fast == SLOW) return;
    const int S0 = 2 * coarse_st[2 * frame], T0 = 2 * coarse_st[2 * frame + 1];
    // column groups: with more than one wave per band, wave 0 takes the 32
    // groups at either end of the row, where the masked terms are, and the
    // others the middle, so that those read without masks; a lane past the
    // groups gets group ncg (columns n.. : every term masked)
    const int ncg = (n + 3) / 4;
    int g;
    if (ncw == 1)
        g = lane;
    else if (cw == 0)
        g = lane < 32 ? lane : ncg - 64 + lane;
    else
        g = 32 + (cw - 1) * 64 + lane < ncg - 32 ? 32 + (cw - 1) * 64 + lane : ncg;
    if (g > ncg) g = ncg;
    const int j0 = 4 * g;
    const int c0 = j0 + T0 - 1;  // odd: the dword at column c0-1 is aligned
    uint32_t mk[3][2];
    bool clean = true;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            uint32_t b = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = 2 * pr + h, c = c0 + q + v;
                if (j0 + q < n && c >= 0 && c < n) b |= 0xffffu << (16 * h);
            }
            mk[v][pr] = b;
            clean = clean && b == 0xffffffffu;
        }
    const uint16_t *fb = frames + (size_t)frame * m * n;
    // rows 1..m-2 may be read as one 16-byte span from column j0+2t*-2
    // (j0 <= n+2) when that stays inside the frame: |2t*| <= n-8
    const bool wide_ok = abs(T0) + 8 <= n;
    unsigned long long acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0;
    if (!SLOW) {
        if (__all(clean))
            roll_rows<false, 0>(fb, tmpl, m, n, i0, i1, S0, j0, c0, flush, wide_ok, mk, acc);
        else
            roll_rows<true, 0>(fb, tmpl, m, n, i0, i1, S0, j0, c0, flush, wide_ok, mk, acc);
    } else if (flush > 0) {
        roll_rows<true, 1>(fb, tmpl, m, n, i0, i1, S0, j0, c0, flush, wide_ok, mk, acc);
    } else {
        roll_rows<true, 2>(fb, tmpl, m, n, i0, i1, S0, j0, c0, flush, wide_ok, mk, acc);
    }
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
        acc[q] = v;
    }
    if (lane == 0) {
        double *dst = partial + ((size_t)frame * units + unit) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) dst[q] = (double)acc[q];
    }
}

// Fast kernel: one wave per (frame, unit); waves of frames in the slow mode
// return at once.  MULTI: each frame's own template and pixel bound come from
// tmpls, tmaxs (frames of several templates in one launch), else tmpl_one and
// tmax_one serve every frame.  (A separate instantiation: a template pointer
// loaded from memory, even when unused, cost the one-template kernel 18% on
// MI355X, 289 -> 341 us per 2000 frames of 512x512.)
template <bool MULTI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_refine_roll(
    const uint16_t *__restrict__ frames, const uint16_t *__restrict__ tmpl_one, int m, int n,
    int br, int nbr, int ncw, int C, const int32_t *__restrict__ coarse_st,
    const int32_t *__restrict__ pmax, int tmax_one, double *__restrict__ partial,
    const uint16_t *const *__restrict__ tmpls, const int32_t *__restrict__ tmaxs)
{
    const int units = nbr * ncw;
    const long long wid =
        (long long)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    if (wid >= (long long)C * units) return;
    const int frame = (int)(wid / units), unit = (int)(wid % units);
    const uint16_t *tmpl = MULTI ? tmpls[frame] : tmpl_one;
    const int tmax = MULTI ? tmaxs[frame] : tmax_one;
    roll_unit<false>(frames, tmpl, m, n, br, ncw, frame, unit, roll_flush(pmax, tmax, frame),
                     coarse_st, partial, units);
}

// The nine full-resolution sums of one frame from its units' partials (one
// wave: lanes take every 64th partial, then a fixed tree), and the argmin.
__device__ __forceinline__ void refine_finish_wave(const double *__restrict__ partial, int frame,
                                                   int nband, int m, int n,
                                                   const int32_t *__restrict__ coarse_st,
                                                   int32_t *__restrict__ shifts,
                                                   double *__restrict__ frefine,
                                                   double *__restrict__ gaps)
{
    const int lane = threadIdx.x % 64;
    double e9[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) e9[q] = 0.0;
    for (int b = lane; b < nband; b += 64) {
        const double *src = partial + ((size_t)frame * nband + b) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) e9[q] += src[q];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e9[q] += __shfl_xor(e9[q], off);
    if (lane != 0) return;
    const int cs = coarse_st[2 * frame], ct = coarse_st[2 * frame + 1];
    Cand c{INFINITY, INT32_MIN, 0, INFINITY};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double e = e9[q];
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

__global__ __launch_bounds__(kBlock) void k_refine_finish(const double *__restrict__ partial,
                                                          int C, int nband, int m, int n,
                                                          const int32_t *__restrict__ coarse_st,
                                                          int32_t *__restrict__ shifts,
                                                          double *__restrict__ frefine,
                                                          double *__restrict__ gaps)
{
    // one wave per frame
    const int frame = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    if (frame >= C) return;
    refine_finish_wave(partial, frame, nband, m, n, coarse_st, shifts, frefine, gaps);
}

// The rolling refine's slow units and its finish in one launch, one wave per
// frame: a frame in the slow mode (sums too wide for the fast kernel's
// 32-bit flushes) runs its units here first (none for most workloads), then
// the wave forms the frame's nine sums and argmin as k_refine_finish.
template <bool MULTI>
__global__ __launch_bounds__(kBlock) void k_refine_slow_finish(
    const uint16_t *__restrict__ frames, const uint16_t *__restrict__ tmpl_one, int m, int n,
    int br, int nbr, int ncw, int C, const int32_t *__restrict__ coarse_st,
    const int32_t *__restrict__ pmax, int tmax_one, double *__restrict__ partial,
    const uint16_t *const *__restrict__ tmpls, const int32_t *__restrict__ tmaxs,
    int32_t *__restrict__ shifts, double *__restrict__ frefine, double *__restrict__ gaps)
{
    const int frame =
        blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    if (frame >= C) return;
    const int units = nbr * ncw;
    const uint16_t *tmpl = MULTI ? tmpls[frame] : tmpl_one;
    const int tmax = MULTI ? tmaxs[frame] : tmax_one;
    const int flush = roll_flush(pmax, tmax, frame);
    if (flush < br) {
        for (int unit = 0; unit < units; ++unit)
            roll_unit<true>(frames, tmpl, m, n, br, ncw, frame, unit, flush, coarse_st, partial,
                            units);
        // the units' partials (stored by lane 0) before the wave reads them
        __threadfence();
    }
    refine_finish_wave(partial, frame, units, m, n, coarse_st, shifts, frefine, gaps);
}

void launch_finish(const double *partial, int C, int nunits, const Geom &g,
                   const int32_t *coarse_st, int32_t *shifts, double *frefine, double *gaps,
                   hipStream_t st)
{
    k_refine_finish<<<(C + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, st>>>(
        partial, C, nunits, g.m, g.n, coarse_st, shifts, frefine, gaps);
}

int grid_for(size_t total)
{
    size_t g = (total + kBlock - 1) / kBlock;
    if (g > 65535 * 4) g = 65535 * 4;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_coarse(const void *frames, moco_dtype dt, int C, const Geom &g, double *coarse,
                         hipStream_t st, const int32_t *only)
{
    clear_stale_error();
    size_t total = (size_t)C * g.mg * g.ng;
    if (total == 0) return hipSuccess;
    if (!only && g.ds && g.n % 8 == 0 && ((uintptr_t)frames & 15) == 0 && ((uintptr_t)coarse & 15) == 0) {
        const size_t quads = total / 4;   // ng = n/2 is a multiple of 4
        if (dt == MOCO_U16)
            k_coarse_ds4<uint16_t><<<grid_for(quads), kBlock, 0, st>>>(
                (const uint16_t *)frames, C, g.m, g.n, g.mg, g.ng, coarse);
        else
            k_coarse_ds4<float><<<grid_for(quads), kBlock, 0, st>>>(
                (const float *)frames, C, g.m, g.n, g.mg, g.ng, coarse);
        return hipGetLastError();
    }
    if (only && C <= 65535) {
        const size_t plane = (size_t)g.mg * g.ng;
        // few blocks per frame: most frames of a masked pass are unset
        const dim3 grid((unsigned)std::min<size_t>((plane + kBlock - 1) / kBlock, 8), C);
        if (dt == MOCO_U16)
            k_coarse_masked<uint16_t><<<grid, kBlock, 0, st>>>(
                (const uint16_t *)frames, g.m, g.n, g.mg, g.ng, g.ds, coarse, only);
        else
            k_coarse_masked<float><<<grid, kBlock, 0, st>>>(
                (const float *)frames, g.m, g.n, g.mg, g.ng, g.ds, coarse, only);
        return hipGetLastError();
    }
    if (dt == MOCO_U16)
        k_coarse<uint16_t><<<grid_for(total), kBlock, 0, st>>>(
            (const uint16_t *)frames, C, g.m, g.n, g.mg, g.ng, g.ds, coarse, only);
    else
        k_coarse<float><<<grid_for(total), kBlock, 0, st>>>((const float *)frames, C, g.m, g.n,
                                                            g.mg, g.ng, g.ds, coarse, only);
    return hipGetLastError();
}

hipError_t launch_corr_fp64(const double *coarse, const double *tcoarse, int C, const Geom &g,
                            double *h, hipStream_t st, const int32_t *only)
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
                                          rowlen, h, only);
    return hipGetLastError();
}

bool energy_rows_applicable(const Geom &g)
{
    return g.ng <= 256 * kErMaxChunks && g.w <= 128;
}

static size_t energy_rows_lds(const Geom &g)
{
    const int we1 = g.w > 1 ? g.w - 1 : 1;
    return ((size_t)kErWaves * 2 * we1 + 4 * (size_t)g.w + 2 * kErWaves) * sizeof(double);
}

template <int SRC>
static void energy_rows_launch(const void *src, int C, const Geom &g, double *atab, int32_t *pmax,
                               double pscale, double center, hipStream_t st, const int32_t *only)
{
    const int nch = (g.ng + 255) / 256;
    const size_t lds = energy_rows_lds(g);
    const dim3 grid(C), blk(kErWaves * 64);
    if (nch <= 1)
        k_energy_rows<SRC, 1><<<grid, blk, lds, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, atab, pmax, pscale, center, only);
    else if (nch <= 2)
        k_energy_rows<SRC, 2><<<grid, blk, lds, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, atab, pmax, pscale, center, only);
    else if (nch <= 4)
        k_energy_rows<SRC, 4><<<grid, blk, lds, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, atab, pmax, pscale, center, only);
    else
        k_energy_rows<SRC, 8><<<grid, blk, lds, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, atab, pmax, pscale, center, only);
}

hipError_t launch_energy(const double *coarse, int C, const Geom &g, bool flip, double *atab,
                         int32_t *pmax, hipStream_t st, double center, const int32_t *only)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    // pixel bound from the grid: a box mean times four bounds its four pixels
    // (non-negative uint16) when the grid covers every pixel
    double pscale = 0.0;
    if (g.dtype == MOCO_U16) {
        const int b = 1 << g.ds;   // a level-L grid value is the mean of a b x b block
        if (g.m % b == 0 && g.n % b == 0) pscale = (double)b * b;
    }
    if (!flip && energy_rows_applicable(g)) {
        energy_rows_launch<0>(coarse, C, g, atab, pmax, pscale, center, st, only);
        return hipGetLastError();
    }
    const int E = g.w - 1;
    const size_t lds = ((size_t)10 * (E + 1) + 1 + 2 * kBlock) * sizeof(double);
    k_energy<0><<<C, kBlock, lds, st>>>(coarse, g.m, g.n, g.mg, g.ng, g.w, flip, atab, pmax,
                                        pscale, center, only);
    return hipGetLastError();
}

hipError_t launch_energy_px(const void *frames, int C, const Geom &g, double *atab,
                            int32_t *pmax, hipStream_t st, double center, const int32_t *only)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (g.ds > 1) return hipErrorInvalidValue;
    double pscale = 0.0;
    const bool u16 = g.dtype == MOCO_U16;
    if (u16) {
        const int b = 1 << g.ds;
        if (g.m % b == 0 && g.n % b == 0) pscale = (double)b * b;
    }
    if (energy_rows_applicable(g)) {
        if (u16 && g.ds)
            energy_rows_launch<1>(frames, C, g, atab, pmax, pscale, center, st, only);
        else if (u16)
            energy_rows_launch<2>(frames, C, g, atab, pmax, pscale, center, st, only);
        else if (g.ds)
            energy_rows_launch<3>(frames, C, g, atab, pmax, pscale, center, st, only);
        else
            energy_rows_launch<4>(frames, C, g, atab, pmax, pscale, center, st, only);
        return hipGetLastError();
    }
    const int E = g.w - 1;
    const size_t lds = ((size_t)10 * (E + 1) + 1 + 2 * kBlock) * sizeof(double);
    if (u16 && g.ds)
        k_energy<1><<<C, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, g.w, false, atab, pmax,
                                            pscale, center, only);
    else if (u16)
        k_energy<2><<<C, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, g.w, false, atab, pmax,
                                            pscale, center, only);
    else if (g.ds)
        k_energy<3><<<C, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, g.w, false, atab, pmax,
                                            pscale, center, only);
    else
        k_energy<4><<<C, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, g.w, false, atab, pmax,
                                            pscale, center, only);
    return hipGetLastError();
}

hipError_t launch_combine(const double *atab, const double *btab, const double *h, int C,
                          const Geom &g, double *fsurf, double *fmin, int32_t *coarse_st,
                          int32_t *shifts, double *gaps, double *frefine, hipStream_t st,
                          const int32_t *only, int32_t *recheck, double kf, double ke,
                          const Cert32 *c32)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    k_combine<<<C, kBlock, 0, st>>>(atab, btab, h, g.mg, g.ng, g.w, g.ds, fsurf, fmin, coarse_st,
                                    shifts, gaps, frefine, only, recheck, kf, ke,
                                    c32 ? *c32 : Cert32{});
    return hipGetLastError();
}

hipError_t launch_polish(const void *src, bool raw, int C, const Geom &g, const double *tcoarse,
                         const int32_t *coarse_st, const int32_t *skip, double *fmin,
                         double *fsurf, double *gaps, hipStream_t st)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (!fmin) return hipErrorInvalidValue;
    const bool u16 = g.dtype == MOCO_U16;
    if (!raw)
        k_polish<0><<<C, kBlock, 0, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, tcoarse, coarse_st, skip,
                                          fmin, fsurf, gaps);
    else if (g.ds > 1)
        return hipErrorInvalidValue;
    else if (u16 && g.ds)
        k_polish<1><<<C, kBlock, 0, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, tcoarse, coarse_st, skip,
                                          fmin, fsurf, gaps);
    else if (u16)
        k_polish<2><<<C, kBlock, 0, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, tcoarse, coarse_st, skip,
                                          fmin, fsurf, gaps);
    else if (g.ds)
        k_polish<3><<<C, kBlock, 0, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, tcoarse, coarse_st, skip,
                                          fmin, fsurf, gaps);
    else
        k_polish<4><<<C, kBlock, 0, st>>>(src, g.m, g.n, g.mg, g.ng, g.w, tcoarse, coarse_st, skip,
                                          fmin, fsurf, gaps);
    return hipGetLastError();
}

hipError_t launch_cand32(const void *frames, int C, const Geom &g, const double *atab,
                         const double *btab, const double *h, const double *tcoarse, double ke,
                         const Cert32 &c32, int32_t *coarse_st, double *fmin, double *fsurf,
                         double *gaps, int32_t *shifts, int32_t *recheck, int32_t *resolved,
                         hipStream_t st)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (g.dtype != MOCO_U16 || g.ds > 1 || g.W * g.W > kCand32MaxShifts || !fmin || !shifts ||
        !recheck || !resolved || !c32.xmax)
        return hipErrorInvalidValue;
    if (g.ds)
        k_cand32<1><<<C, kBlock, 0, st>>>((const uint16_t *)frames, g.m, g.n, g.mg, g.ng, g.w,
                                          g.ds, atab, btab, h, tcoarse, ke, c32, coarse_st, fmin,
                                          fsurf, gaps, shifts, recheck, resolved);
    else
        k_cand32<2><<<C, kBlock, 0, st>>>((const uint16_t *)frames, g.m, g.n, g.mg, g.ng, g.w,
                                          g.ds, atab, btab, h, tcoarse, ke, c32, coarse_st, fmin,
                                          fsurf, gaps, shifts, recheck, resolved);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int count, int32_t v, hipStream_t st)
{
    clear_stale_error();
    if (count <= 0) return hipSuccess;
    k_fill_i32<<<(count + kBlock - 1) / kBlock, kBlock, 0, st>>>(p, count, v);
    return hipGetLastError();
}

hipError_t launch_add_i32(int32_t *p, const int32_t *q, int count, hipStream_t st)
{
    clear_stale_error();
    if (count <= 0) return hipSuccess;
    k_add_i32<<<(count + kBlock - 1) / kBlock, kBlock, 0, st>>>(p, q, count);
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
    if (refine_rolling(g, frames, traw)) {
        const int br = roll_band_rows(g, C);
        const int nbr = (g.m + br - 1) / br, ncw = ((g.n + 3) / 4 + 63) / 64;
        const int units = nbr * ncw;
        const long long waves = (long long)C * units;
        const long long blocks = (waves + kBlock / 64 - 1) / (kBlock / 64);
        if (blocks > INT32_MAX) return hipErrorInvalidValue;
        k_refine_roll<false><<<(unsigned)blocks, kBlock, 0, st>>>((const uint16_t *)frames,
                                                          (const uint16_t *)traw, g.m, g.n, br,
                                                          nbr, ncw, C, coarse_st, pmax, tmax,
                                                          partial, nullptr, nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_refine_slow_finish<false><<<(C + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, st>>>(
            (const uint16_t *)frames, (const uint16_t *)traw, g.m, g.n, br, nbr, ncw, C,
            coarse_st, pmax, tmax, partial, nullptr, nullptr, shifts, frefine, gaps);
        return hipGetLastError();
    }
    int br = refine_band_rows(g);
    if (g.dtype == MOCO_U16 && refine_u16_banded(g)) {
        const int nband = (g.m + kRefBand - 1) / kRefBand;
        const size_t lds = ((size_t)(kRefBand + 2) * g.n + 16) * sizeof(uint16_t);
        dim3 grid(nband, C);
        k_refine_u16<<<grid, kBlock, lds, st>>>((const uint16_t *)frames, (const uint16_t *)traw,
                                               g.m, g.n, coarse_st, pmax, tmax, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        launch_finish(partial, C, nband, g, coarse_st, shifts, frefine, gaps, st);
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
        launch_finish(partial, C, nband, g, coarse_st, shifts, frefine, gaps, st);
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

hipError_t launch_refine_multi(const uint16_t *frames, const uint16_t *const *traws,
                               const int32_t *tmaxs, int C, const Geom &g,
                               const int32_t *coarse_st, int32_t *shifts, double *frefine,
                               double *gaps, double *partial, hipStream_t st,
                               const int32_t *pmax)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (g.dtype != MOCO_U16 || g.n % 2 != 0 || ((uintptr_t)frames & 3) != 0)
        return hipErrorInvalidValue;
    const int br = roll_band_rows(g, C);
    const int nbr = (g.m + br - 1) / br, ncw = ((g.n + 3) / 4 + 63) / 64;
    const int units = nbr * ncw;
    const long long waves = (long long)C * units;
    const long long blocks = (waves + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    k_refine_roll<true><<<(unsigned)blocks, kBlock, 0, st>>>(frames, nullptr, g.m, g.n, br, nbr,
                                                            ncw, C, coarse_st, pmax, -1, partial,
                                                            traws, tmaxs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_refine_slow_finish<true><<<(C + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, st>>>(
        frames, nullptr, g.m, g.n, br, nbr, ncw, C, coarse_st, pmax, -1, partial, traws, tmaxs,
        shifts, frefine, gaps);
    return hipGetLastError();
}

hipError_t launch_half(const double *in, int C, int m, int n, double *out, hipStream_t st)
{
    clear_stale_error();
    const size_t total = (size_t)C * (m / 2) * (n / 2);
    if (total == 0) return hipSuccess;
    k_half<<<grid_for(total), kBlock, 0, st>>>(in, C, m, n, out);
    return hipGetLastError();
}

// Rows per block of the FP64 level refine (0: rows too wide to stage).
static int level_band_rows(int n)
{
    const size_t row = (size_t)n * sizeof(double);
    if (3 * row > 40 * 1024) return 0;
    const int br = (int)(40 * 1024 / row) - 2;
    return br > 16 ? 16 : br;
}

size_t refine_level_partial_bytes(int m, int n)
{
    const int br = level_band_rows(n);
    return br > 0 ? (size_t)((m + br - 1) / br) * 9 * sizeof(double) : 0;
}

hipError_t launch_refine_level(const double *frames, const double *tmpl, int C, int m, int n,
                               const int32_t *in_st, int32_t *out_st, double *partial,
                               hipStream_t st)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    const int br = level_band_rows(n);
    if (br <= 0) {
        k_refine<double><<<C, kBlock, 0, st>>>(frames, tmpl, m, n, in_st, out_st, nullptr,
                                               nullptr);
        return hipGetLastError();
    }
    const int nband = (m + br - 1) / br;
    k_refine_band<double><<<dim3(nband, C), kBlock, (size_t)(br + 2) * n * sizeof(double), st>>>(
        frames, tmpl, m, n, br, in_st, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    Geom gl{};
    gl.m = m;
    gl.n = n;
    launch_finish(partial, C, nband, gl, in_st, out_st, nullptr, nullptr, st);
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

bool refine_rolling(const Geom &g, const void *frames, const void *traw)
{
    return g.dtype == MOCO_U16 && g.n % 2 == 0 && ((uintptr_t)frames & 3) == 0 &&
           ((uintptr_t)traw & 3) == 0;
}

int roll_band_rows(const Geom &g, int C)
{
    // long bands for big stacks (fewer partial sums), short ones for a few
    // frames so that the launch still spreads over the chip
    return (long long)C * g.m >= 16384 ? 4 * kRollMinRows : kRollMinRows;
}

static size_t refine_partial_bytes_fixed(const Geom &g)
{
    if (g.dtype == MOCO_U16 && refine_u16_banded(g))
        return (size_t)((g.m + kRefBand - 1) / kRefBand) * 9 * sizeof(double);
    int br = refine_band_rows(g);
    if (br <= 0) return 0;
    return (size_t)((g.m + br - 1) / br) * 9 * sizeof(double);
}

size_t refine_partial_bytes(const Geom &g)
{
    // the larger of the rolling layout (shortest bands) and the fixed-band one,
    // which unaligned buffers fall back to
    size_t b = refine_partial_bytes_fixed(g);
    if (g.dtype == MOCO_U16 && g.n % 2 == 0) {
        const size_t nbr = (size_t)(g.m + kRollMinRows - 1) / kRollMinRows;
        const size_t ncw = (size_t)((g.n + 3) / 4 + 63) / 64;
        const size_t r = nbr * ncw * 9 * sizeof(double);
        if (r > b) b = r;
    }
    return b;
}

}  // namespace moco
